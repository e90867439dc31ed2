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
__device__ __forceinline__ void store2(float2* p, double2 v) {
    *p = make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ void store2(double2* p, double2 v) { *p = v; }

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
        store2(pop + e, make_double2(d == 0 ? 0.25 : 0.125, 0.0));
    }
    if (E != nullptr && q >= 0 && e == 0) E[(int64_t)q * (K + 1)] = make_double2(1.0, 0.0);
}

// exp(i th) in FP64 (library sincos; used only in workgroup prologues).
__device__ __forceinline__ double2 expi(double th) {
    double sn, cs;
    sincos(th, &sn, &cs);
    return make_double2(cs, sn);
}

// One step for a tile of TX x TY site columns, each thread walking fd.zc
// sites along z.  Workgroup -> (field, tile) via blk_field and the field's
// tile counts; no per-site integer division.
template <typename V, int TX>
__global__ void __launch_bounds__(kBlock) k_step(StepArgs a) {
    constexpr int TY = kBlock / TX;
    __shared__ double2 lds[kBlock / 64];
    __shared__ double2 face_fac[6];
    __shared__ double2 ex[TX], ey[TY], ez[kMaxZc];
    __shared__ double c_w[kMaxPhase], c_dec[kMaxPhase], c_tr[kMaxPhase * kMaxPhase];
    __shared__ int last_flag;
    const int fi = a.blk_field[blockIdx.x];
    const FieldDesc& fd = a.fields[fi];
    const int32_t ns = fd.nsites;
    const int32_t n0 = fd.n[0], n1 = fd.n[1], n2 = fd.n[2];
    const int32_t b = blockIdx.x - fd.blk0;
    const int32_t tx = b % fd.tiles[0];
    const int32_t rb = b / fd.tiles[0];
    const int32_t ty = rb % fd.tiles[1];
    const int32_t tz = rb / fd.tiles[1];
    const double F = a.Fk[a.k];
    const double fdt = a.fdt[a.k];
    const int32_t z0 = tz * fd.zc;
    // Phase factors of this workgroup, computed once: the six face factors
    // exp(i beta F_k) and the reaction factor exp(-i fdt (c.j + cu)) split
    // per axis over the tile's x, y and z ranges.
    {
        const int t = threadIdx.x;
        if (t < 6) {
            const double beta = fd.beta[t];
            face_fac[t] = beta != 0.0 ? expi(beta * F) : make_double2(1.0, 0.0);
        } else if (t >= 64 && t < 64 + TX) {
            const int l = t - 64;
            ex[l] = expi(-fdt * fd.c[0] * (double)(tx * TX + l));
        } else if (t >= 128 && t < 128 + TY) {
            const int l = t - 128;
            ey[l] = expi(-fdt * fd.c[1] * (double)(ty * TY + l));
        } else if (t >= 192 && t < 192 + fd.zc) {
            const int l = t - 192;
            ez[l] = expi(-fdt * (fd.c[2] * (double)(z0 + l) + fd.cu));
        }
        const int P = a.n_phase;
        if (t < P) {
            c_w[t] = a.w[t];
            c_dec[t] = a.decay[t];
        }
        if (t < P * P) c_tr[(t / P) * kMaxPhase + t % P] = a.trans[t];
    }
    __syncthreads();

    const V* __restrict__ src = static_cast<const V*>(a.src);
    V* __restrict__ dst = static_cast<V*>(a.dst);
    const uint32_t* __restrict__ words = a.words + fd.words;
    const int64_t pop = fd.pop;
    const int32_t j0 = tx * TX + (int32_t)(threadIdx.x % TX);
    const int32_t j1 = ty * TY + (int32_t)(threadIdx.x / TX);
    const int32_t z1 = min(n2, z0 + fd.zc);
    const int32_t st1 = n0, st2 = n0 * n1;
    const double2 exy = cmul(ex[threadIdx.x % TX], ey[threadIdx.x / TX]);

    // Source offset (relative to the site index s) of each pulled direction,
    // fixed for the whole z column for x and y; z faces switch per site.
    // Interior: same field, neighbour site.  Periodic face: same field,
    // wrapped site.  Mirror face: source field of that face, same site,
    // reflected direction.
    int32_t kind[6];
    int64_t fpop[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        kind[f] = fd.face_kind[f];
        fpop[f] = fd.face_pop[f];
    }
    auto face_off = [&](int f, int d, int32_t wrap) -> int64_t {
        const int db = (d & 1) ? d + 1 : d - 1;
        return (kind[f] & kFaceMirror) ? fpop[f] + (int64_t)db * ns
                                       : fpop[f] + (int64_t)d * ns + wrap;
    };
    const bool fx0 = j0 == 0, fx1 = j0 == n0 - 1, fy0 = j1 == 0, fy1 = j1 == n1 - 1;
    const int64_t o1 = fx0 ? face_off(0, 1, n0 - 1) : pop + 1 * (int64_t)ns - 1;
    const int64_t o2 = fx1 ? face_off(1, 2, -(n0 - 1)) : pop + 2 * (int64_t)ns + 1;
    const int64_t o3 = fy0 ? face_off(2, 3, (n1 - 1) * st1) : pop + 3 * (int64_t)ns - st1;
    const int64_t o4 = fy1 ? face_off(3, 4, -(n1 - 1) * st1) : pop + 4 * (int64_t)ns + st1;
    const int64_t o5i = pop + 5 * (int64_t)ns - st2, o5f = face_off(4, 5, (n2 - 1) * st2);
    const int64_t o6i = pop + 6 * (int64_t)ns + st2, o6f = face_off(5, 6, -(n2 - 1) * st2);

    double2 Mv = make_double2(0.0, 0.0);
    if (j0 < n0 && j1 < n1) {
        for (int32_t j2 = z0; j2 < z1; ++j2) {
            const int32_t s = j0 + st1 * j1 + st2 * j2;
            const bool fz0 = j2 == 0, fz1 = j2 == n2 - 1;
            // all loads of the site issued together
            const uint32_t word = words[s];
            double2 g[kQ];
            g[0] = ld2(src + pop + s);
            g[1] = ld2(src + o1 + s);
            g[2] = ld2(src + o2 + s);
            g[3] = ld2(src + o3 + s);
            g[4] = ld2(src + o4 + s);
            g[5] = ld2(src + (fz0 ? o5f : o5i) + s);
            g[6] = ld2(src + (fz1 ? o6f : o6i) + s);
            const int p = (int)(word & 0xfu);
            const uint32_t mask = (word >> 4) & 0x3fu;
            double2 own[kQ];
            if (mask) {
                // outgoing populations at this node, reflected at membranes
#pragma unroll
                for (int d = 1; d < kQ; ++d) {
                    const int od = (d & 1) ? d + 1 : d - 1;
                    own[d] = ld2(src + pop + (int64_t)od * ns + s);
                }
            }
            const bool face[6] = {fx0, fx1, fy0, fy1, fz0, fz1};
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                if (face[f]) {
                    double2 v = g[f + 1];
                    if (kind[f] & kFaceConj) v.y = -v.y;
                    g[f + 1] = cmul(v, face_fac[f]);
                }
            }
            if (mask) {
                // half-link membrane: g' = ghat_opp(x) + t (incoming - ghat_opp(x))
#pragma unroll
                for (int d = 1; d < kQ; ++d) {
                    if ((mask >> (d - 1)) & 1u) {
                        const int pn = (int)((word >> (10 + 3 * (d - 1))) & 0x7u);
                        const double t = c_tr[p * kMaxPhase + pn];
                        if (t < 1.0) {
                            g[d].x = own[d].x + t * (g[d].x - own[d].x);
                            g[d].y = own[d].y + t * (g[d].y - own[d].y);
                        }
                    }
                }
            }
            // reaction: exp(-i fdt (c.j + cu)) exp(-dt/T2)
            const double2 e = cmul(exy, ez[j2 - z0]);
            const double dec = c_dec[p];
            const double2 rf = make_double2(e.x * dec, e.y * dec);
            double2 M = make_double2(0.0, 0.0);
#pragma unroll
            for (int d = 0; d < kQ; ++d) {
                g[d] = cmul(g[d], rf);
                M.x += g[d].x;
                M.y += g[d].y;
            }
            Mv.x += M.x;
            Mv.y += M.y;
            // collision: ghat = g + w (w_d M - g)
            const double w = c_w[p];
            V* out = dst + pop + s;
#pragma unroll
            for (int d = 0; d < kQ; ++d) {
                const double wd = d == 0 ? 0.25 : 0.125;
                double2 h;
                h.x = g[d].x + w * (wd * M.x - g[d].x);
                h.y = g[d].y + w * (wd * M.y - g[d].y);
                store2(out + (int64_t)d * ns, h);
            }
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
    for (int i = threadIdx.x; i < fd.nblk; i += kBlock) {
        double* pp = &a.partial[fd.blk0 + i].x;
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
    store2(out + s, m);
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

template <typename V>
static void launch_step_t(int shape, const StepArgs& a, int32_t n_blocks, hipStream_t st) {
    switch (shape) {
        case kTile64x4:
            hipLaunchKernelGGL((k_step<V, 64>), dim3(n_blocks), dim3(kBlock), 0, st, a);
            break;
        case kTile32x8:
            hipLaunchKernelGGL((k_step<V, 32>), dim3(n_blocks), dim3(kBlock), 0, st, a);
            break;
        default:
            hipLaunchKernelGGL((k_step<V, 16>), dim3(n_blocks), dim3(kBlock), 0, st, a);
            break;
    }
}

hipError_t launch_step(int prec, int shape, const StepArgs& a, int32_t n_blocks, hipStream_t st) {
    if (prec == 1)
        launch_step_t<float2>(shape, a, n_blocks, st);
    else
        launch_step_t<double2>(shape, a, n_blocks, st);
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
