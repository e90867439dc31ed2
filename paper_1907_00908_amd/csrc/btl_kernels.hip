// HIP kernels of the hybrid lattice Boltzmann Bloch-Torrey step for gfx950.
//
// The state kept between steps is the post-collision population ghat.  One
// launch of k_step advances every field by one step in "pull" form:
//   1. g'_i(x) = ghat_i(x - e_i)                      streaming (Eq. streaming_LBM)
//      - at a periodic face the source is the wrapped node and the value is
//        multiplied by exp(+-i phi_a), phi_a = L_a (gamma G0)_a F_k
//        (modified periodic BC, Eqs. periodic_phi, collision_BC)
//      - at a mirror face the source is the same node in the reflected
//        direction, possibly of a reflected image field and conjugated
//        (mirroring BC, Sec. 2.4.4)
//      - across a membrane link g'_i(x) = ghat_ibar(x) + t (ghat_i(x-e_i) -
//        ghat_ibar(x)) with t = 1/(1+P), P = eps_D dx/(2 kappa dt)
//        (half-link condition, Eqs. B5, P_def, permeability_BC)
//   2. g_i = g'_i exp(-i gamma (x.G0) f_k dt) exp(-dt/T2)   (Eq. reaction_LBM)
//   3. M = sum_i g_i; the workgroup adds M into the signal partial sum
//      (Eq. M'summation; signal Sec. 2.1)
//   4. ghat_i = g_i + w (w_i M - g_i), w = 1/tau       (Eq. collision_LBM)
// which is the paper's collide -> stream -> react cycle (Eq.
// LBM_process_list_2) started at the stream.  All arithmetic is FP64;
// populations are stored as float2 or double2 (x fastest, one plane per
// direction per field).  Per-step constants enter only through forms that
// keep sum_i g_i exact for any rounded constant (g + w(wM - g), a + t(b - a)).
//
// The signal of a step is reduced deterministically: each workgroup writes a
// partial sum, and the last workgroup of a field to finish (arrival counter)
// adds all partials of that field in a fixed order.
#include "btl_internal.h"

namespace btl {

__device__ __forceinline__ double2 ld2(const float2* p) {
    const float2 v = *p;
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 ld2(const double2* p) { return *p; }
__device__ __forceinline__ void st2(float2* p, double2 v) {
    *p = make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ void st2(double2* p, double2 v) { *p = v; }

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

template <typename V>
__global__ void __launch_bounds__(kBlock) k_init(V* pop, int64_t nsites, double2* E,
                                                  int32_t q, int32_t K) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < nsites * kQ) {
        const int d = (int)(e / nsites);
        st2(pop + e, make_double2(d == 0 ? 0.25 : 0.125, 0.0));
    }
    if (E != nullptr && q >= 0 && e == 0) E[(int64_t)q * (K + 1)] = make_double2(1.0, 0.0);
}

template <typename V>
__global__ void __launch_bounds__(kBlock) k_step(StepArgs a) {
    __shared__ double2 lds[kBlock / 64];
    __shared__ int last_flag;
    const int fi = a.blk_field[blockIdx.x];
    const FieldDesc& fd = a.fields[fi];
    const int32_t ns = fd.nsites;
    const int32_t s = (blockIdx.x - fd.blk0) * kBlock + threadIdx.x;
    const V* __restrict__ src = static_cast<const V*>(a.src);
    V* __restrict__ dst = static_cast<V*>(a.dst);
    const V* __restrict__ me = src + fd.pop;

    double2 Mv = make_double2(0.0, 0.0);
    if (s < ns) {
        const int32_t n0 = fd.n[0], n1 = fd.n[1], n2 = fd.n[2];
        const int32_t j0 = s % n0;
        const int32_t r = s / n0;
        const int32_t j1 = r % n1;
        const int32_t j2 = r / n1;
        const int32_t jj[3] = {j0, j1, j2};
        const int32_t stride[3] = {1, n0, n0 * n1};
        const int32_t nn[3] = {n0, n1, n2};
        const uint32_t word = a.words[fd.words + s];
        const int p = (int)(word & 0xffu);
        const uint32_t mask = word >> 8;
        const double F = a.Fk[a.k];
        const double fdt = a.fdt[a.k];

        double2 g[kQ];
        g[0] = ld2(me + s);
#pragma unroll
        for (int d = 1; d < kQ; ++d) {
            const int ax = (d - 1) >> 1;
            const bool plus = (d & 1) != 0;          // e_d = +axis: pull from j - e
            const int32_t ja = jj[ax];
            const bool face = plus ? (ja == 0) : (ja == nn[ax] - 1);
            double2 v;
            int32_t nb;
            if (!face) {
                nb = plus ? s - stride[ax] : s + stride[ax];
                v = ld2(me + (int64_t)d * ns + nb);
            } else {
                const int f = 2 * ax + (plus ? 0 : 1);
                const int kind = fd.face_kind[f];
                const V* fsrc = src + fd.face_pop[f];
                if ((kind & kFaceMirror) == 0) {
                    nb = plus ? s + (nn[ax] - 1) * stride[ax] : s - (nn[ax] - 1) * stride[ax];
                    v = ld2(fsrc + (int64_t)d * ns + nb);
                } else {
                    nb = s;
                    const int db = plus ? d + 1 : d - 1;   // reflected direction
                    v = ld2(fsrc + (int64_t)db * ns + s);
                }
                if (kind & kFaceConj) v.y = -v.y;
                const double beta = fd.beta[f];
                if (beta != 0.0) {
                    double sn, cs;
                    sincos(beta * F, &sn, &cs);
                    v = cmul(v, make_double2(cs, sn));
                }
            }
            if ((mask >> (d - 1)) & 1u) {
                const int pn = (int)(a.words[fd.words + nb] & 0xffu);
                const double t = a.trans[p * a.n_phase + pn];
                if (t < 1.0) {
                    const int od = (d & 1) ? d + 1 : d - 1;
                    const double2 own = ld2(me + (int64_t)od * ns + s);
                    v.x = own.x + t * (v.x - own.x);
                    v.y = own.y + t * (v.y - own.y);
                }
            }
            g[d] = v;
        }
        // reaction
        const double th = -fdt * (fd.c[0] * j0 + fd.c[1] * j1 + fd.c[2] * j2 + fd.cu);
        double sn, cs;
        sincos(th, &sn, &cs);
        const double dec = a.decay[p];
        const double2 rf = make_double2(cs * dec, sn * dec);
        double2 M = make_double2(0.0, 0.0);
#pragma unroll
        for (int d = 0; d < kQ; ++d) {
            g[d] = cmul(g[d], rf);
            M.x += g[d].x;
            M.y += g[d].y;
        }
        Mv = M;
        // collision
        const double w = a.w[p];
        V* out = dst + fd.pop + s;
#pragma unroll
        for (int d = 0; d < kQ; ++d) {
            const double wd = d == 0 ? 0.25 : 0.125;
            double2 h;
            h.x = g[d].x + w * (wd * M.x - g[d].x);
            h.y = g[d].y + w * (wd * M.y - g[d].y);
            st2(out + (int64_t)d * ns, h);
        }
    }

    if (fd.q < 0) return;   // image fields do not enter the signal
    const double2 bsum = block_sum(Mv, lds);
    if (threadIdx.x == 0) {
        double* pp = &a.partial[blockIdx.x].x;
        __hip_atomic_store(pp, bsum.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(pp + 1, bsum.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t prev = __hip_atomic_fetch_add(a.counter + fi, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        last_flag = (prev == (uint32_t)(fd.nblk - 1));
    }
    __syncthreads();
    if (!last_flag) return;
    __threadfence();
    double2 acc = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < fd.nblk; b += kBlock) {
        double* pp = &a.partial[fd.blk0 + b].x;
        acc.x += __hip_atomic_load(pp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        acc.y += __hip_atomic_load(pp + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const double2 tot = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        const double inv = 1.0 / (double)ns;
        double2* E = reinterpret_cast<double2*>(a.E);
        E[(int64_t)fd.q * (a.K + 1) + a.k + 1] = make_double2(tot.x * inv, tot.y * inv);
        __hip_atomic_store(a.counter + fi, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename V>
__global__ void __launch_bounds__(kBlock) k_mfinal(const V* pop, int64_t nsites, V* out) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= nsites) return;
    double2 m = make_double2(0.0, 0.0);
#pragma unroll
    for (int d = 0; d < kQ; ++d) {
        const double2 v = ld2(pop + (int64_t)d * nsites + s);
        m.x += v.x;
        m.y += v.y;
    }
    st2(out + s, m);
}

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_init(int prec, void* pop, int64_t, const FieldDesc*, int32_t n_fields,
                       const FieldDesc* h, double* E, int32_t, int32_t K, hipStream_t st) {
    for (int f = 0; f < n_fields; ++f) {
        const int64_t ns = h[f].nsites;
        if (prec == 1)
            hipLaunchKernelGGL(k_init<float2>, dim3(grid_for(ns * kQ)), dim3(kBlock), 0, st,
                               static_cast<float2*>(pop) + h[f].pop, ns,
                               reinterpret_cast<double2*>(E), h[f].q, K);
        else
            hipLaunchKernelGGL(k_init<double2>, dim3(grid_for(ns * kQ)), dim3(kBlock), 0, st,
                               static_cast<double2*>(pop) + h[f].pop, ns,
                               reinterpret_cast<double2*>(E), h[f].q, K);
    }
    return hipGetLastError();
}

hipError_t launch_step(int prec, const StepArgs& a, int32_t n_blocks, hipStream_t st) {
    if (prec == 1)
        hipLaunchKernelGGL(k_step<float2>, dim3(n_blocks), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL(k_step<double2>, dim3(n_blocks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_mfinal(int prec, const void* pop, const FieldDesc* h, int32_t n_fields,
                         void* M_out, hipStream_t st) {
    int64_t off = 0;
    for (int f = 0; f < n_fields; ++f) {
        if (h[f].q < 0) continue;
        const int64_t ns = h[f].nsites;
        if (prec == 1)
            hipLaunchKernelGGL(k_mfinal<float2>, dim3(grid_for(ns)), dim3(kBlock), 0, st,
                               static_cast<const float2*>(pop) + h[f].pop, ns,
                               static_cast<float2*>(M_out) + off);
        else
            hipLaunchKernelGGL(k_mfinal<double2>, dim3(grid_for(ns)), dim3(kBlock), 0, st,
                               static_cast<const double2*>(pop) + h[f].pop, ns,
                               static_cast<double2*>(M_out) + off);
        off += ns;
    }
    return hipGetLastError();
}

}  // namespace btl
