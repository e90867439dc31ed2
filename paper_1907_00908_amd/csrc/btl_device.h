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

// Workgroups are dealt to the 8 XCDs round-robin (workgroup i to XCD
// i mod 8), each XCD with its own L2.  xcd_tile renumbers them so that every
// XCD walks one contiguous range of tiles: neighbouring tiles, which read
// each other's edge rows, then run on the same XCD close in time and share
// those rows through its L2.  A bijection of [0, G).
constexpr int kXcd = 8;
__device__ __forceinline__ int32_t xcd_tile(int32_t bid, int32_t G) {
    const int32_t k = bid % kXcd, i = bid / kXcd;
    const int32_t q = G / kXcd, r = G % kXcd;
    return (k < r ? k * (q + 1) : r * (q + 1) + (k - r) * q) + i;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Weights of the six populations that make up the population entering a
// node across a membrane at distance d (units of dx) from it, for a straight
// membrane normal to the link (Eqs. B2a_text/B2b_text with theta = 0,
// Eqs. B4a-B4c).  The Dirichlet (c_d) and Neumann (c_n) coefficients of the
// node's own side use d (Eqs. c_d, c_n), those of the far side 1 - d.
// Output order: own side A[0..2] for ghat_ibar(x), ghat_ibar(x + e_i),
// ghat_i(x); far side B[0..2] for ghat_i(x - e_i), ghat_i(x - 2 e_i),
// ghat_ibar(x - e_i).  kdt = kappa dt, edx = eps_D dx.
struct MembCoef {
    double A[3], B[3];
};
__device__ __forceinline__ MembCoef membrane_coefficients(double d, double kdt, double edx) {
    const double e = 1.0 - d;
    // one division for the three reciprocals ro = 1/(2d + 1), rf = 1/(2e + 1)
    // and rF below: with Do = 3 - 2d, Df = 3 - 2e the denominator of rF is
    // ro rf Qd, Qd = Do Df edx + 2 (Do + Df) kdt
    const double Ao = 2.0 * d + 1.0, Af = 2.0 * e + 1.0;
    const double Do = 3.0 - 2.0 * d, Df = 3.0 - 2.0 * e;
    const double Qd = Do * Df * edx + 2.0 * (Do + Df) * kdt;
    const double AA = Ao * Af;
    const double R = 1.0 / (AA * Qd);
    const double ro = Af * Qd * R, rf = Ao * Qd * R;
    const double ho = 2.0 * d - 1.0, hf = 2.0 * e - 1.0;
    // own side
    const double n2 = -ho * ro, n3 = ho * ro, n4 = 2.0 * ro;
    const double d1 = 2.0 * d - 2.0, d2 = -ho * ho * ro, d3 = 2.0 * ho * ro, d4 = (3.0 - 2.0 * d) * ro;
    // far side
    const double fn2 = -hf * rf, fn3 = hf * rf, fn4 = 2.0 * rf;
    const double fd1 = 2.0 * e - 2.0, fd2 = -hf * hf * rf, fd3 = 2.0 * hf * rf, fd4 = (3.0 - 2.0 * e) * rf;
    const double diff = d4 * fd4 * edx;
    const double perm_own = fd4 * n4 * kdt, perm_far = fn4 * d4 * kdt;
    const double rF = AA * AA * R;   // 1 / (diff + (d4 fn4 + n4 fd4) kdt)
    MembCoef c;
    c.A[0] = (diff + perm_own * d1 + perm_far) * rF;
    c.A[1] = (diff * n2 + perm_own * d2 + perm_far * n2) * rF;
    c.A[2] = (diff * n3 + perm_own * d3 + perm_far * n3) * rF;
    const double bk = d4 * n4 * kdt * rF;
    c.B[0] = bk * (1.0 - fd1);
    c.B[1] = bk * (fn2 - fd2);
    c.B[2] = bk * (fn3 - fd3);
    return c;
}

// exp(i th) in FP64 (library sincos; used only by the table kernel).
__device__ __forceinline__ double2 expi(double th) {
    double sn, cs;
    sincos(th, &sn, &cs);
    return make_double2(cs, sn);
}

}  // namespace btl
