// Device helpers shared by the forward and adjoint kernels.
#pragma once

#include "btl_internal.h"

namespace btl {

__device__ __forceinline__ double2 ld2(const float2* p) {
    const float2 v = *p;
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 ld2(const double2* p) { return *p; }
__device__ __forceinline__ void store2(float2* p, double2 v) {
    *p = make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ void store2(double2* p, double2 v) { *p = v; }
// Streaming stores: the next step reads the whole state back, which does not
// fit in the caches, so the written lines are not kept.
__device__ __forceinline__ void store2_stream(float2* p, double2 v) {
    __builtin_nontemporal_store((float)v.x, &p->x);
    __builtin_nontemporal_store((float)v.y, &p->y);
}
__device__ __forceinline__ void store2_stream(double2* p, double2 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

// Value that is the same in every lane, kept in scalar registers.
__device__ __forceinline__ double uniform(double v) {
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(u & 0xffffffffu));
    const int hi = __builtin_amdgcn_readfirstlane((int)(u >> 32));
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double2 uniform2(double2 v) {
    return make_double2(uniform(v.x), uniform(v.y));
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-order sum of v over the 256 threads of the workgroup; the result is
// valid in thread 0.
__device__ __forceinline__ double2 block_sum(double2 v, double2* lds) {
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double2 r = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) {
        r = lds[0];
        for (int i = 1; i < kBlock / 64; ++i) {
            r.x += lds[i].x;
            r.y += lds[i].y;
        }
    }
    return r;
}

// exp(i th) in FP64 (library sincos; used only by the table kernel).
__device__ __forceinline__ double2 expi(double th) {
    double sn, cs;
    sincos(th, &sn, &cs);
    return make_double2(cs, sn);
}

}  // namespace btl
