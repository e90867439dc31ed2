// Adjoint of the hybrid lattice Boltzmann Bloch-Torrey step (reverse mode).
//
// The forward step k maps the post-collision populations ghat^k to
//   g'^k = S_k ghat^k          stream with faces and half-link membranes
//   g^k+1 = c_k g'^k           reaction, c_k(x) = exp(-i fdt_k (c.j + cu)) dec_p
//   M = sum_i g_i, E_{k+1} += M / N
//   ghat^{k+1} = g + w (w_i M - g)
// (see btl_kernels.hip).  For a real loss L and complex z the adjoint is
// dL/dz = dL/dRe z + i dL/dIm z.  The kernel below advances the adjoint of the
// post-stream populations, Lambda^k = dL/dg'^k, one step back:
//   lhat = S_k^T Lambda^k                 adjoint pull: read from y + e_j
//   nu_i = (1 - w) lhat_i + w sum_j w_j lhat_j + dL/dE_k / N
//   Lambda^{k-1}_i = conj(c_{k-1}) nu_i
// The transpose of the stream reads the adjoint at the node that pulled from
// y in direction j, with the conjugate of the forward face factor (or, where
// the forward conjugated, the conjugate of the adjoint times the factor), and
// at a membrane link lhat_j = (1 - t) Lambda_jbar(y) + t (pulled adjoint),
// the same split as the forward one.  The quantities of forward step k-1
// (g, M, the pulled values) are recomputed from ghat^{k-1}.
//
// Parameter sensitivities accumulated per step (all real):
//   d/dw_p      sum Re conj(lhat_i) (w_i M - g_i)            collision
//   d/ddec_p    sum Re conj(nu_i) g_i / dec_p               T2 decay
//   d/dt_pair   sum Re conj(Lambda_i) (pulled - own)         membrane links
//   d/df_{k-1}  sum dt (c.j + cu) Im( conj(nu_i) g_i )      reaction phase
//   d/dF_{k-1}  sum -beta t Im( conj(Lambda_i) pulled )      face factors
// Each workgroup sums them in LDS (one row per thread, so the order is fixed)
// and the last workgroup of a field sums the workgroup rows in a fixed order.
#include "btl_device.h"

namespace btl {

template <typename V, int TX>
__global__ void __launch_bounds__(kBlock) k_adj(AdjArgs a) {
    constexpr int TY = kBlock / TX;
    constexpr int RS = kNGMax + 1;               // LDS row stride (odd: fewer bank conflicts)
    __shared__ double c_w[kAdjMaxPhase], c_dec[kAdjMaxPhase], c_tr[kAdjMaxPhase * kAdjMaxPhase];
    __shared__ double acc[kBlock * RS];
    __shared__ int last_flag;
    const int P = a.n_phase;
    const int NG = a.ng;
    const int IW = 0, IDEC = P, IT = 2 * P, IF = 2 * P + P * P, IFF = IF + 1;
    {
        const int t = threadIdx.x;
        if (t < P) {
            c_w[t] = a.w[t];
            c_dec[t] = a.decay[t];
        }
        if (t < P * P) c_tr[t] = a.trans[t];
        for (int g = 0; g < RS; ++g) acc[t * RS + g] = 0.0;
    }
    __syncthreads();
    double* my = acc + threadIdx.x * RS;

    const int fi = a.blk_field[blockIdx.x];
    const FieldDesc& fd = a.fields[fi];
    const int32_t ns = fd.nsites;
    const int32_t n0 = fd.n[0], n1 = fd.n[1], n2 = fd.n[2];
    const int32_t b = blockIdx.x - fd.blk0;
    const int32_t tx = b % fd.tiles[0];
    const int32_t rb = b / fd.tiles[0];
    const int32_t ty = rb % fd.tiles[1];
    const int32_t tz = rb / fd.tiles[1];
    const int32_t z0 = tz * fd.zc;
    const int32_t z1 = min(n2, z0 + fd.zc);
    const int32_t j0 = tx * TX + (int32_t)(threadIdx.x % TX);
    const int32_t j1 = ty * TY + (int32_t)(threadIdx.x / TX);
    const int32_t st1 = n0, st2 = n0 * n1;
    const int64_t pop = fd.pop;
    const V* __restrict__ fwd = static_cast<const V*>(a.fwd);
    const V* __restrict__ lam = static_cast<const V*>(a.lam_in);
    V* __restrict__ out = static_cast<V*>(a.lam_out);
    const uint32_t* __restrict__ words = a.words + fd.words;
    const double2* __restrict__ tabp = a.tab_prev + fd.tab;
    double2 ffac[6], afac[6];
    double beta[6];
    int32_t kind[6], akind[6];
    int64_t fpop[6], apop[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        ffac[f] = uniform2(tabp[n0 + n1 + n2 + f]);
        afac[f] = a.top ? make_double2(1.0, 0.0) : uniform2(a.tab_cur[fd.adj_fac[f]]);
        beta[f] = fd.beta[f];
        kind[f] = fd.face_kind[f];
        akind[f] = fd.adj_kind[f];
        fpop[f] = fd.face_pop[f];
        apop[f] = fd.adj_pop[f];
    }
    const double cx0 = fd.c[0], cx1 = fd.c[1], cx2 = fd.c[2], cu = fd.cu;
    const double dt = a.dt;
    double2 mu = make_double2(0.0, 0.0);
    if (fd.q >= 0) {
        const double2 m = a.dLdE[(int64_t)fd.q * (a.K + 1) + a.k];
        mu = make_double2(m.x / ns, m.y / ns);
    }

    if (j0 < n0 && j1 < n1) {
        const double2 exy = cmul(tabp[j0], tabp[n0 + j1]);
        const bool fx0 = j0 == 0, fx1 = j0 == n0 - 1, fy0 = j1 == 0, fy1 = j1 == n1 - 1;
        for (int32_t j2 = z0; j2 < z1; ++j2) {
            const int32_t s = j0 + st1 * j1 + st2 * j2;
            const int32_t jj[3] = {j0, j1, j2};
            const int32_t nn[3] = {n0, n1, n2};
            const int32_t stv[3] = {1, st1, st2};
            const bool fz0 = j2 == 0, fz1 = j2 == n2 - 1;
            const bool lo[3] = {fx0, fy0, fz0}, hi[3] = {fx1, fy1, fz1};
            const uint32_t word = words[s];
            const int p = (int)(word & 0xfu);
            const uint32_t mask = (word >> 4) & 0x3fu;
            auto nbphase = [&](int d) { return (int)((word >> (10 + 3 * (d - 1))) & 0x7u); };

            // ---- forward step k-1 recomputed at this node ----
            double2 gp[kQ], v[kQ], own[kQ];
            double tl[kQ];
            gp[0] = ld2(fwd + pop + s);
#pragma unroll
            for (int d = 1; d < kQ; ++d) {
                const int ax = (d - 1) >> 1;
                const bool plus = (d & 1) != 0;
                const bool face = plus ? lo[ax] : hi[ax];
                const int od = plus ? d + 1 : d - 1;
                double2 x;
                if (!face) {
                    x = ld2(fwd + pop + (int64_t)d * ns + (plus ? s - stv[ax] : s + stv[ax]));
                } else {
                    const int f = 2 * ax + (plus ? 0 : 1);
                    if (kind[f] & kFaceMirror) {
                        x = ld2(fwd + fpop[f] + (int64_t)od * ns + s);
                    } else {
                        const int32_t w = (nn[ax] - 1) * stv[ax];
                        x = ld2(fwd + fpop[f] + (int64_t)d * ns + (plus ? s + w : s - w));
                    }
                    if (kind[f] & kFaceConj) x.y = -x.y;
                    x = cmul(x, ffac[f]);
                }
                v[d] = x;
                tl[d] = 1.0;
                own[d] = ld2(fwd + pop + (int64_t)od * ns + s);
                if ((mask >> (d - 1)) & 1u) {
                    const double t = c_tr[p * P + nbphase(d)];
                    if (t < 1.0) {
                        tl[d] = t;
                        x.x = own[d].x + t * (x.x - own[d].x);
                        x.y = own[d].y + t * (x.y - own[d].y);
                    }
                }
                gp[d] = x;
            }
            const double2 ezj = tabp[n0 + n1 + j2];
            const double dec = c_dec[p];
            const double2 e = cmul(exy, ezj);
            const double2 c = make_double2(e.x * dec, e.y * dec);
            double2 g[kQ];
            double2 M = make_double2(0.0, 0.0);
#pragma unroll
            for (int d = 0; d < kQ; ++d) {
                g[d] = cmul(gp[d], c);
                M.x += g[d].x;
                M.y += g[d].y;
            }
            const double w = c_w[p];

            // ---- adjoint pull of Lambda^k ----
            double2 lh[kQ];
            if (a.top) {
#pragma unroll
                for (int d = 0; d < kQ; ++d) lh[d] = make_double2(0.0, 0.0);
            } else {
                lh[0] = ld2(lam + pop + s);
#pragma unroll
                for (int d = 1; d < kQ; ++d) {
                    const int ax = (d - 1) >> 1;
                    const bool plus = (d & 1) != 0;      // destination y + e_d
                    const bool face = plus ? hi[ax] : lo[ax];
                    const int od = plus ? d + 1 : d - 1;
                    double2 x;
                    if (!face) {
                        x = ld2(lam + pop + (int64_t)d * ns + (plus ? s + stv[ax] : s - stv[ax]));
                    } else {
                        const int f = 2 * ax + (plus ? 1 : 0);
                        if (akind[f] & kFaceMirror) {
                            x = ld2(lam + apop[f] + (int64_t)od * ns + s);
                        } else {
                            const int32_t w = (nn[ax] - 1) * stv[ax];
                            x = ld2(lam + apop[f] + (int64_t)d * ns + (plus ? s - w : s + w));
                        }
                        if (akind[f] & kFaceConj) {
                            x = cmul(make_double2(x.x, -x.y), afac[f]);
                        } else {
                            x = cmul(make_double2(afac[f].x, -afac[f].y), x);
                        }
                    }
                    // link between this node and y + e_d: membrane bit of the
                    // opposite pull direction at this node
                    if ((mask >> (od - 1)) & 1u) {
                        const double t = c_tr[p * P + nbphase(od)];
                        if (t < 1.0) {
                            const double2 lo_ = ld2(lam + pop + (int64_t)od * ns + s);
                            x.x = lo_.x + t * (x.x - lo_.x);
                            x.y = lo_.y + t * (x.y - lo_.y);
                        }
                    }
                    lh[d] = x;
                }
            }

            // ---- transposed collision and reaction ----
            double2 sl = make_double2(0.0, 0.0);
#pragma unroll
            for (int d = 0; d < kQ; ++d) {
                const double wd = d == 0 ? 0.25 : 0.125;
                sl.x += wd * lh[d].x;
                sl.y += wd * lh[d].y;
            }
            double gw = 0.0, gdec = 0.0, gim = 0.0;
            double2 lo2[kQ];
#pragma unroll
            for (int d = 0; d < kQ; ++d) {
                const double wd = d == 0 ? 0.25 : 0.125;
                // collision: d ghat_d / dw = w_d M - g_d
                gw += lh[d].x * (wd * M.x - g[d].x) + lh[d].y * (wd * M.y - g[d].y);
                double2 nu;
                nu.x = (1.0 - w) * lh[d].x + w * sl.x + mu.x;
                nu.y = (1.0 - w) * lh[d].y + w * sl.y + mu.y;
                // Re and Im of conj(nu) g
                gdec += nu.x * g[d].x + nu.y * g[d].y;
                gim += nu.x * g[d].y - nu.y * g[d].x;
                lo2[d] = cmul(make_double2(c.x, -c.y), nu);
                store2(out + pop + (int64_t)d * ns + s, lo2[d]);
            }
            my[IW + p] += gw;
            my[IDEC + p] += gdec / dec;
            const double thp = cx0 * j0 + cx1 * j1 + cx2 * j2 + cu;
            my[IF] += dt * thp * gim;
            // stream sensitivities of step k-1: membranes and face factors
#pragma unroll
            for (int d = 1; d < kQ; ++d) {
                const int ax = (d - 1) >> 1;
                const bool plus = (d & 1) != 0;
                const bool face = plus ? lo[ax] : hi[ax];
                if (tl[d] < 1.0) {
                    const double2 df = make_double2(v[d].x - own[d].x, v[d].y - own[d].y);
                    my[IT + p * P + nbphase(d)] += lo2[d].x * df.x + lo2[d].y * df.y;
                }
                if (face) {
                    const int f = 2 * ax + (plus ? 0 : 1);
                    if (beta[f] != 0.0) {
                        const double im = lo2[d].x * v[d].y - lo2[d].y * v[d].x;
                        my[IFF] += -beta[f] * tl[d] * im;
                    }
                }
            }
        }
    }

    // ---- workgroup sums, then the last workgroup of the field ----
    __syncthreads();
    if (threadIdx.x < NG) {
        double sacc = 0.0;
        for (int t = 0; t < kBlock; ++t) sacc += acc[t * RS + threadIdx.x];
        __hip_atomic_store(a.gpart + (int64_t)blockIdx.x * NG + threadIdx.x, sacc,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = __hip_atomic_fetch_add(a.counter + fi, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        last_flag = (prev == (uint32_t)(fd.nblk - 1));
    }
    __syncthreads();
    if (!last_flag) return;
    __threadfence();
    if (threadIdx.x < NG) {
        double sacc = 0.0;
        for (int i = 0; i < fd.nblk; ++i)
            sacc += __hip_atomic_load(a.gpart + (int64_t)(fd.blk0 + i) * NG + threadIdx.x,
                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.gfield[((int64_t)(a.k - 1) * a.n_fields + fi) * NG + threadIdx.x] = sacc;
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(a.counter + fi, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums the per-step, per-field records in a fixed order and maps them to the
// user parameters:
//   dL/dD_p   = G_w[p] * dw/dD,     w = 1/tau, tau = 1/2 + dt D/(eps_D dx^2)
//   dL/dT2_p  = G_dec[p] * dec_p * dt / T2_p^2
//   dL/dkappa = (G_t[a][b] + G_t[b][a]) * dt/dkappa, t = 1/(1 + eps_D dx/(2 kappa dt))
//   dL/df_m   = G_f[m] + dt * sum_{k>m} G_F[k]       (F_k = sum_{m<k} f_m dt)
__global__ void k_adj_final(const double* gfield, int32_t K, int32_t n_fields, int32_t P,
                            double dt, double dx, const double* w, const double* T2,
                            const double* kappa, double* dD, double* dT2, double* dkappa,
                            double* df) {
    const int NG = 2 * P + P * P + 2;
    const int t = threadIdx.x;
    auto total = [&](int g) {
        double s = 0.0;
        for (int k = 0; k < K; ++k)
            for (int f = 0; f < n_fields; ++f) s += gfield[((int64_t)k * n_fields + f) * NG + g];
        return s;
    };
    if (t < P) {
        if (dD) {
            const double wp = w[t];
            dD[t] = total(t) * (-wp * wp * dt / (0.25 * dx * dx));
        }
        if (dT2) {
            const double T = T2[t];
            const double dec = isinf(T) ? 1.0 : exp(-dt / T);
            dT2[t] = isinf(T) ? 0.0 : total(P + t) * dec * dt / (T * T);
        }
    }
    if (t < P * P && dkappa) {
        const int i = t / P, j = t % P;
        const double k = kappa[t];
        double g = total(2 * P + i * P + j);
        if (i != j) g += total(2 * P + j * P + i);
        // t = 8 k dt / (dx + 8 k dt) for eps_D = 1/4
        const double den = dx + 8.0 * k * dt;
        dkappa[t] = isinf(k) ? 0.0 : g * 8.0 * dt * dx / (den * den);
    }
    if (t == 0 && df) {
        const int IF = 2 * P + P * P, IFF = IF + 1;
        double suffix = 0.0;   // sum_{k > m} G_F[k]
        for (int m = K - 1; m >= 0; --m) {
            double gf = 0.0;
            for (int f = 0; f < n_fields; ++f) gf += gfield[((int64_t)m * n_fields + f) * NG + IF];
            df[m] = gf + dt * suffix;
            double gF = 0.0;
            for (int f = 0; f < n_fields; ++f) gF += gfield[((int64_t)m * n_fields + f) * NG + IFF];
            suffix += gF;
        }
    }
}

template <typename V>
static void launch_adj_t(int shape, const AdjArgs& a, int32_t n_blocks, hipStream_t st) {
    switch (shape) {
        case kTile64x4:
            hipLaunchKernelGGL((k_adj<V, 64>), dim3(n_blocks), dim3(kBlock), 0, st, a);
            break;
        case kTile32x8:
            hipLaunchKernelGGL((k_adj<V, 32>), dim3(n_blocks), dim3(kBlock), 0, st, a);
            break;
        case kTile128x2:
            hipLaunchKernelGGL((k_adj<V, 128>), dim3(n_blocks), dim3(kBlock), 0, st, a);
            break;
        default:
            hipLaunchKernelGGL((k_adj<V, 16>), dim3(n_blocks), dim3(kBlock), 0, st, a);
            break;
    }
}

hipError_t launch_adj(int prec, int shape, const AdjArgs& a, int32_t n_blocks, hipStream_t st) {
    if (prec == 1)
        launch_adj_t<float2>(shape, a, n_blocks, st);
    else
        launch_adj_t<double2>(shape, a, n_blocks, st);
    return hipGetLastError();
}

hipError_t launch_adj_final(const double* gfield, int32_t K, int32_t n_fields, int32_t P,
                            double dt, double dx, const double* w, const double* T2,
                            const double* kappa, double* dD, double* dT2, double* dkappa,
                            double* df, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_final, dim3(1), dim3(64), 0, st, gfield, K, n_fields, P, dt, dx,
                       w, T2, kappa, dD, dT2, dkappa, df);
    return hipGetLastError();
}

}  // namespace btl
