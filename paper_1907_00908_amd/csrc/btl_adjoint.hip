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
// and, when asked for (GG), what the gamma G0 gradient needs: the reaction
// angle is -fdt (c.j + cu) with c_b = s_b G_b dx and cu = -dx sum_b sigma_b
// G_b, so per step R_b = sum j_b Im(conj(nu_i) g_i) (b = x, y, z) and
// R_0 = sum Im(conj(nu_i) g_i); every face factor is exp(i beta_f F) with
// beta_f linear in G, so per step and face X_f = sum -t Im(conj(Lambda_i)
// pulled).  k_adj_final combines them with d beta_f / d G_b.
// Per-phase sums are kept in registers (selected by the node's phase), the
// membrane-pair sums in one LDS row per thread; workgroup and field sums are
// formed in a fixed order, so the gradients are bitwise reproducible.
#include <type_traits>

#include "btl_device.h"

namespace btl {

// Per-site arithmetic runs in the precision of the stored populations (FP32
// storage: FP32 products, which the stored adjoint rounds to anyway); every
// sum over sites, steps and workgroups is FP64.
template <typename V> struct AdjReal;
template <> struct AdjReal<float2> { using R = float; };
template <> struct AdjReal<double2> { using R = double; };

__device__ __forceinline__ float2 cmulr(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulr(double2 a, double2 b) { return cmul(a, b); }
template <typename V> __device__ __forceinline__ V mk2(double x, double y);
template <> __device__ __forceinline__ float2 mk2<float2>(double x, double y) {
    return make_float2((float)x, (float)y);
}
template <> __device__ __forceinline__ double2 mk2<double2>(double x, double y) {
    return make_double2(x, y);
}
__device__ __forceinline__ void store_stream(float2* p, float2 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}
__device__ __forceinline__ void store_stream(double2* p, double2 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

// NP: phases the per-thread sums are sized for (2 or kAdjMaxPhase); a
// smaller NP shrinks the per-thread LDS row of membrane-pair sums from
// 17 to 5 doubles and the per-phase register sums.
template <typename V, int TX, bool GG, int NQ, int NP>
__device__ __forceinline__ void adj_body(const AdjArgs& a) {
    using R = typename AdjReal<V>::R;
    // planes pz (+z pull) and pz + 1 (-z pull); on the single-layer D2Q5
    // lattice the kernel's z axis is the geometry's y axis and planes 3, 4
    // pull along it (as in the forward step), site words keep plane numbers
    constexpr int pz = NQ == 7 ? 5 : 3;
    auto axis_of = [](int d) { return NQ == 7 ? (d - 1) >> 1 : (d <= 2 ? 0 : 2); };
    constexpr int TY = TX > 0 ? kBlock / TX : 1;
    constexpr int NT = NP * NP;                        // membrane pair sums per thread (LDS row)
    constexpr int RS = NT + 1;                         // odd row stride
    __shared__ double c_tr[kAdjMaxPhase * kAdjMaxPhase];
    __shared__ R c_w[kAdjMaxPhase], c_dec[kAdjMaxPhase], c_rdec[kAdjMaxPhase];
    __shared__ double acc[kBlock * RS];
    __shared__ double red[kNGMax];
    __shared__ V ffac[6], afac[6];   // forward / adjoint face factors of this field
    __shared__ R beta[6];
    const int P = a.n_phase;
    const int NG = a.ng;
    const int IW = 0, IDEC = P, IT = 2 * P, IF = 2 * P + P * P, IFF = IF + 1;
    const int IR = IFF + 1, IX = IR + 4;   // GG only
    {
        const int t = threadIdx.x;
        if (t < P) {
            c_w[t] = (R)a.w[t];
            c_dec[t] = (R)a.decay[t];
            c_rdec[t] = (R)(1.0 / a.decay[t]);
        }
        if (t < P * P) c_tr[t] = a.trans[t];
        for (int g = 0; g < RS; ++g) acc[t * RS + g] = 0.0;
    }
    __syncthreads();
    double* my = acc + threadIdx.x * RS;

    const int32_t lb = a.xcd ? xcd_tile((int32_t)blockIdx.x, (int32_t)gridDim.x)
                             : (int32_t)blockIdx.x;
    const int2 fbk = a.blk_field[lb];   // field, block of the field
    const int fi = fbk.x;
    const FieldDesc& fd = a.fields[fi];
    const int32_t ns = fd.nsites;
    const int32_t n0 = fd.n[0], n1 = fd.n[1], n2 = fd.n[2];
    const int32_t b = fbk.y;
    const int32_t tx = b % fd.tiles[0];
    const int32_t rb = b / fd.tiles[0];
    const int32_t ty = rb % fd.tiles[1];
    const int32_t tz = rb / fd.tiles[1];
    const int32_t z0 = tz * fd.zc;
    const int32_t z1 = min(n2, z0 + fd.zc);
    int32_t j0, j1;
    if constexpr (TX == 0) {   // kTileRows: kBlock consecutive sites of the x-y plane
        const int32_t i = tx * kBlock + (int32_t)threadIdx.x;
        j0 = i % n0;
        j1 = i / n0;
    } else {
        j0 = tx * TX + (int32_t)(threadIdx.x % TX);
        j1 = ty * TY + (int32_t)(threadIdx.x / TX);
    }
    // site index s = j0 + st1 j1 + st2 j2 (site words); populations z-major:
    // plane d of site (j0, j1, j2) at d ps + j0 + st1 j1 + zs j2
    const int32_t st1 = n0, st2 = n0 * n1, ps = st2, zs = NQ * st2;
    // one base pointer per buffer for this field; every access is a 32-bit
    // element offset from it (image-field partners of the same q-sample
    // lie within +-2^31 elements, checked on the host)
    const V* __restrict__ fwd = static_cast<const V*>(a.fwd) + fd.pop;
    const V* __restrict__ lam = a.top ? nullptr : static_cast<const V*>(a.lam_in) + fd.pop;
    V* __restrict__ out = static_cast<V*>(a.lam_out) + fd.pop;
    const int32_t pop = 0;
    const uint32_t* __restrict__ words = a.words + fd.words;
    const double2* __restrict__ tabp = a.tab_prev + fd.tab;
    if (threadIdx.x < 6) {
        const int f = threadIdx.x;
        const double2 ff = tabp[n0 + n1 + n2 + f];
        const double2 af = a.top ? make_double2(1.0, 0.0) : a.tab_cur[fd.adj_fac[f]];
        ffac[f] = mk2<V>(ff.x, ff.y);
        afac[f] = mk2<V>(af.x, af.y);
        beta[f] = (R)fd.beta[f];
    }
    int32_t kind[6], akind[6];
    int32_t fpop[6], apop[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        kind[f] = fd.face_kind[f];
        akind[f] = fd.adj_kind[f];
        fpop[f] = (int32_t)(fd.face_pop[f] - fd.pop);
        apop[f] = (int32_t)(fd.adj_pop[f] - fd.pop);
    }
    __syncthreads();
    const double cx0 = fd.c[0], cx1 = fd.c[1], cx2 = fd.c[2], cu = fd.cu;
    const double dt = a.dt;
    V mu = mk2<V>(0.0, 0.0);
    if (fd.q >= 0) {
        const double2 m = a.dLdE[(int64_t)fd.q * (a.K + 1) + a.k];
        mu = mk2<V>(m.x / ns, m.y / ns);
    }
    // register sums of the per-phase sensitivities (selected by phase)
    double sw[NP], sdec[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) sw[i] = sdec[i] = 0.0;
    double sf = 0.0, sF = 0.0;
    double sR[GG ? 4 : 1] = {0.0}, sX[GG ? 6 : 1] = {0.0};

    if (j0 < n0 && j1 < n1 && z0 < z1) {
        const double2 exyd = cmul(tabp[j0], tabp[n0 + j1]);
        const V exy = mk2<V>(exyd.x, exyd.y);
        const bool fx0 = j0 == 0, fx1 = j0 == n0 - 1, fy0 = j1 == 0, fy1 = j1 == n1 - 1;
        // forward pull offsets (relative to the site index), as in k_step
        auto face_off = [&](int f, int d, int32_t wrap) -> int32_t {
            const int db = (d & 1) ? d + 1 : d - 1;
            return (kind[f] & kFaceMirror) ? fpop[f] + db * ps : fpop[f] + d * ps + wrap;
        };
        // adjoint pull offsets: destination y + e_d
        auto adj_off = [&](int f, int d, int32_t wrap) -> int32_t {
            const int db = (d & 1) ? d + 1 : d - 1;
            return (akind[f] & kFaceMirror) ? apop[f] + db * ps : apop[f] + d * ps + wrap;
        };
        const int32_t o1 = fx0 ? face_off(0, 1, n0 - 1) : pop + 1 * ps - 1;
        const int32_t o2 = fx1 ? face_off(1, 2, -(n0 - 1)) : pop + 2 * ps + 1;
        const int32_t o3 = NQ == 5 ? 0 : fy0 ? face_off(2, 3, (n1 - 1) * st1) : pop + 3 * ps - st1;
        const int32_t o4 = NQ == 5 ? 0 : fy1 ? face_off(3, 4, -(n1 - 1) * st1) : pop + 4 * ps + st1;
        const int32_t q1 = fx1 ? adj_off(1, 1, -(n0 - 1)) : pop + 1 * ps + 1;
        const int32_t q2 = fx0 ? adj_off(0, 2, n0 - 1) : pop + 2 * ps - 1;
        const int32_t q3 = NQ == 5 ? 0 : fy1 ? adj_off(3, 3, -(n1 - 1) * st1) : pop + 3 * ps + st1;
        const int32_t q4 = NQ == 5 ? 0 : fy0 ? adj_off(2, 4, (n1 - 1) * st1) : pop + 4 * ps - st1;
        // z offsets (planes pz, pz + 1) do not depend on the thread: wave-uniform
        const int32_t o5i = pop + pz * ps - zs;
        const int32_t o6i = pop + (pz + 1) * ps + zs;
        const int32_t q5i = pop + pz * ps + zs;
        const int32_t q6i = pop + (pz + 1) * ps - zs;
        const int32_t o5f = face_off(4, pz, (n2 - 1) * zs);
        const int32_t o6f = face_off(5, pz + 1, -(n2 - 1) * zs);
        const int32_t q5f = adj_off(5, pz, -(n2 - 1) * zs);
        const int32_t q6f = adj_off(4, pz + 1, (n2 - 1) * zs);

        // Four values are shared with the z neighbour and carried along the
        // column instead of reloaded (D3Q7 plane numbers, pz = 5): adjoint
        // plane 6 at z is rlown[5] here and rl[6] of z + 1, plane 5 at z + 1
        // is rl[5] here and rlown[6] of z + 1; forward plane 5 at z is
        // rown[6] here and rg[5] of z + 1, plane 6 at z + 1 is rg[6] here
        // and rown[5] of z + 1.
        V c_rl6 = mk2<V>(0.0, 0.0), c_rlo6 = mk2<V>(0.0, 0.0), c_rg5, c_ro5;
        {
            const int32_t sp = j0 + st1 * j1 + zs * z0;
            if (!a.top) {
                c_rl6 = lam[(z0 == 0 ? q6f : q6i) + sp];
                c_rlo6 = lam[pop + pz * ps + sp];
            }
            c_rg5 = fwd[(z0 == 0 ? o5f : o5i) + sp];
            c_ro5 = fwd[pop + (pz + 1) * ps + sp];
        }
        // the site word of the next site is loaded one site ahead: the
        // first use of a word then never waits a memory round trip of its own
        uint32_t word_next = words[j0 + st1 * j1 + st2 * z0];
#pragma nounroll
        for (int32_t j2 = z0; j2 < z1; ++j2) {
            const int32_t s = j0 + st1 * j1 + st2 * j2;
            const int32_t sp = j0 + st1 * j1 + zs * j2;
            const bool fz0 = j2 == 0, fz1 = j2 == n2 - 1;
            // Two load phases per node keep the live register set small:
            // first the adjoint (consumed into lhat), then the forward state.
            const uint32_t word = word_next;
            if (j2 + 1 < z1) word_next = words[s + st2];
            const int p = (int)(word & 0xfu);
            const uint32_t mask = (word >> 4) & 0x3fu;
            auto nbphase = [&](int d) { return (int)((word >> (10 + 3 * (d - 1))) & 0x7u); };
            const bool flo[3] = {fx0, fy0, fz0}, fhi[3] = {fx1, fy1, fz1};

            // ---- adjoint pull of Lambda^k ----
            V lh[NQ];
            if (a.top) {
#pragma unroll
                for (int d = 0; d < NQ; ++d) lh[d] = mk2<V>(0.0, 0.0);
            } else {
                V rl[NQ], rlown[NQ];
                rl[0] = lam[pop + sp];
                rl[1] = lam[q1 + sp];
                rl[2] = lam[q2 + sp];
                if constexpr (NQ == 7) {
                    rl[3] = lam[q3 + sp];
                    rl[4] = lam[q4 + sp];
                }
                rl[pz] = lam[(fz1 ? q5f : q5i) + sp];
                rl[pz + 1] = c_rl6;
#pragma unroll
                for (int d = 1; d <= pz; ++d) {
                    const int od = (d & 1) ? d + 1 : d - 1;
                    rlown[d] = lam[pop + od * ps + sp];
                }
                rlown[pz + 1] = c_rlo6;
                c_rl6 = rlown[pz];
                c_rlo6 = rl[pz];
                lh[0] = rl[0];
#pragma unroll
                for (int d = 1; d < NQ; ++d) {
                    const int ax = axis_of(d);
                    const bool plus = (d & 1) != 0;      // destination y + e_d
                    const int od = plus ? d + 1 : d - 1;
                    V x = rl[d];
                    if (plus ? fhi[ax] : flo[ax]) {
                        const int f = 2 * ax + (plus ? 1 : 0);
                        const V af = afac[f];
                        if (akind[f] & kFaceConj) {
                            x.y = -x.y;
                            x = cmulr(x, af);
                        } else {
                            x = cmulr(V{af.x, -af.y}, x);
                        }
                    }
                    // membrane between this node and y + e_d: bit of the
                    // opposite pull direction at this node
                    if ((mask >> (od - 1)) & 1u) {
                        const double td = c_tr[p * P + nbphase(od)];
                        if (td < 1.0) {
                            const R t = (R)td;
                            const V lo = rlown[d];
                            x.x = lo.x + t * (x.x - lo.x);
                            x.y = lo.y + t * (x.y - lo.y);
                        }
                    }
                    lh[d] = x;
                }
            }
            V sl = mk2<V>(0.0, 0.0);
#pragma unroll
            for (int d = 0; d < NQ; ++d) {
                const R wd = d == 0 ? (R)lattice_w0(NQ) : (R)lattice_w1(NQ);
                sl.x += wd * lh[d].x;
                sl.y += wd * lh[d].y;
            }
            __builtin_amdgcn_sched_barrier(0);

            // ---- forward state of step k-1 around this node ----
            V rg[NQ], rown[NQ];
            rg[0] = fwd[pop + sp];
            rg[1] = fwd[o1 + sp];
            rg[2] = fwd[o2 + sp];
            if constexpr (NQ == 7) {
                rg[3] = fwd[o3 + sp];
                rg[4] = fwd[o4 + sp];
            }
            rg[pz] = c_rg5;
            rg[pz + 1] = fwd[(fz1 ? o6f : o6i) + sp];
#pragma unroll
            for (int d = 1; d < NQ; ++d) {
                const int od = (d & 1) ? d + 1 : d - 1;
                if (d != pz) rown[d] = fwd[pop + od * ps + sp];
            }
            rown[pz] = c_ro5;
            c_rg5 = rown[pz + 1];
            c_ro5 = rg[pz + 1];
            const double2 ezd = tabp[n0 + n1 + j2];
            const R dec = c_dec[p];
            const R w = c_w[p];
            const V e = cmulr(exy, mk2<V>(ezd.x, ezd.y));
            const V c = V{e.x * dec, e.y * dec};
            const V cc = V{c.x, -c.y};

            // ---- per direction: forward step k-1 recomputed, transposed
            // collision and reaction, sensitivities ----
            V M = mk2<V>(0.0, 0.0);
            R glg = 0, gdec = 0, gim = 0;
#pragma unroll
            for (int d = 0; d < NQ; ++d) {
                const int ax = d > 0 ? axis_of(d) : 0;
                const bool plus = (d & 1) != 0;
                const bool face = d > 0 && (plus ? flo[ax] : fhi[ax]);
                const int f = 2 * ax + (plus ? 0 : 1);
                V vv = rg[d];
                if (face) {
                    if (kind[f] & kFaceConj) vv.y = -vv.y;
                    vv = cmulr(vv, ffac[f]);
                }
                V gpd = vv;
                R tl = 1;
                V dv = mk2<V>(0.0, 0.0);
                if (d > 0 && ((mask >> (d - 1)) & 1u)) {
                    const double td = c_tr[p * P + nbphase(d)];
                    if (td < 1.0) {
                        const R t = (R)td;
                        const V ow = rown[d];
                        tl = t;
                        dv = V{vv.x - ow.x, vv.y - ow.y};
                        gpd.x = ow.x + t * dv.x;
                        gpd.y = ow.y + t * dv.y;
                    }
                }
                const V g = cmulr(gpd, c);
                M.x += g.x;
                M.y += g.y;
                glg += lh[d].x * g.x + lh[d].y * g.y;
                V nu;
                nu.x = (1 - w) * lh[d].x + w * sl.x + mu.x;
                nu.y = (1 - w) * lh[d].y + w * sl.y + mu.y;
                gdec += nu.x * g.x + nu.y * g.y;
                gim += nu.x * g.y - nu.y * g.x;
                const V lo2 = cmulr(cc, nu);
                store_stream(out + pop + d * ps + sp, lo2);
                if (tl < 1) my[p * P + nbphase(d)] += (double)(lo2.x * dv.x + lo2.y * dv.y);
                if (face) {
                    sF += (double)(-beta[f] * tl * (lo2.x * vv.y - lo2.y * vv.x));
                    if constexpr (GG) sX[f] += (double)(-tl * (lo2.x * vv.y - lo2.y * vv.x));
                }
            }
            // collision: sum_d Re conj(lhat_d) (w_d M - g_d)
            const double gw = (double)(sl.x * M.x + sl.y * M.y - glg);
            const double gd = (double)(gdec * c_rdec[p]);
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                sw[i] += (p == i) ? gw : 0.0;
                sdec[i] += (p == i) ? gd : 0.0;
            }
            sf += dt * (cx0 * j0 + cx1 * j1 + cx2 * j2 + cu) * (double)gim;
            if constexpr (GG) {
                sR[0] += (double)j0 * (double)gim;
                sR[1] += (double)j1 * (double)gim;
                sR[2] += (double)j2 * (double)gim;
                sR[3] += (double)gim;
            }
        }
    }

    // ---- workgroup sums (fixed order) into this step's slot; k_adj_gsum adds
    // the workgroups of each field after the segment (no fence or arrival
    // counter at the end of every workgroup) ----
    if (threadIdx.x < NG) red[threadIdx.x] = 0.0;
    __syncthreads();
    // register sums: wave reduction, then the four waves in order
    {
        double v[2 * NP + 2 + (GG ? kNGGrad : 0)];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            v[i] = wave_sum(sw[i]);
            v[NP + i] = wave_sum(sdec[i]);
        }
        v[2 * NP] = wave_sum(sf);
        v[2 * NP + 1] = wave_sum(sF);
        if constexpr (GG) {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[2 * NP + 2 + i] = wave_sum(sR[i]);
#pragma unroll
            for (int i = 0; i < 6; ++i) v[2 * NP + 6 + i] = wave_sum(sX[i]);
        }
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int wave = 0; wave < kBlock / 64; ++wave) {
            if (wv == wave && lane == 0) {
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    if (i < P) {
                        red[IW + i] += v[i];
                        red[IDEC + i] += v[NP + i];
                    }
                }
                red[IF] += v[2 * NP];
                red[IFF] += v[2 * NP + 1];
                if constexpr (GG) {
#pragma unroll
                    for (int i = 0; i < kNGGrad; ++i) red[IR + i] += v[2 * NP + 2 + i];
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x < P * P) {
        double sacc = 0.0;
        for (int t = 0; t < kBlock; ++t) sacc += acc[t * RS + threadIdx.x];
        red[IT + threadIdx.x] = sacc;
    }
    __syncthreads();
    if (threadIdx.x < NG)
        a.gpart[((int64_t)a.slot * gridDim.x + fd.blk0 + b) * NG + threadIdx.x] = red[threadIdx.x];
}

template <typename V, int TX, bool GG, int NQ, int NP>
__global__ void __launch_bounds__(kBlock) k_adj(AdjArgs a) {
    adj_body<V, TX, GG, NQ, NP>(a);
}
// FP32 storage: held to 128 VGPRs (four waves per SIMD), which it fits
// without spilling
template <typename V, int TX, bool GG, int NQ, int NP>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_adj_w4(AdjArgs a) {
    adj_body<V, TX, GG, NQ, NP>(a);
}

// One thread per (step slot, field, accumulator): the field's workgroup sums
// in workgroup order.
__global__ void __launch_bounds__(kBlock) k_adj_gsum(const double* __restrict__ gpart,
                                                     const FieldDesc* __restrict__ fields,
                                                     int32_t n_fields, int32_t nblk_total,
                                                     int32_t ng, int32_t k_first, int32_t nsteps,
                                                     double* gfield, int32_t f_off,
                                                     int32_t nf_total) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)nsteps * n_fields * ng) return;
    const int32_t g = (int32_t)(t % ng);
    const int32_t f = (int32_t)((t / ng) % n_fields);
    const int32_t j = (int32_t)(t / ((int64_t)ng * n_fields));
    const FieldDesc& fd = fields[f];
    const double* p = gpart + ((int64_t)j * nblk_total + fd.blk0) * ng + g;
    double sacc = 0.0;
    for (int32_t i = 0; i < fd.nblk; ++i) sacc += p[(int64_t)i * ng];
    gfield[((int64_t)(k_first + j) * nf_total + f_off + f) * ng + g] = sacc;
}

// Sums the per-step, per-field records in a fixed order and maps them to the
// user parameters:
//   dL/dD_p   = G_w[p] * dw/dD,     w = 1/tau, tau = 1/2 + dt D/(eps_D dx^2)
//   dL/dT2_p  = G_dec[p] * dec_p * dt / T2_p^2
//   dL/dkappa[a][b] = (G_t[a][b] + G_t[b][a]) / 2 * dt/dkappa (a != b),
//                     t = 1/(1 + eps_D dx/(2 kappa dt))
//   dL/df_m   = G_f[m] + dt * sum_{k>m} G_F[k]       (F_k = sum_{m<k} f_m dt)
// With `sub` reaction sub-steps per step, f_m dt is the sum of `sub`
// samples times dt/sub, so each sample of step m gets dL/df_m / sub.
// One workgroup: the totals are block sums over (step, field), the suffix
// sums of G_F a chunked scan (thread t owns a contiguous range of steps),
// and each gamma G0 component one wave striding over the steps; every sum
// runs in a fixed order.
constexpr int kFinalBlock = 1024;
__global__ void __launch_bounds__(kFinalBlock)
k_adj_final(const double* gfield, int32_t K, int32_t n_fields, int32_t P, double dt, double dx,
            const double* w, const double* T2, const double* kappa, double* dD, double* dT2,
            double* dkappa, double* df, int32_t sub, int32_t NG, const double* gmeta,
            const double* fdt, const double* Fk, int32_t Q, double* dgG0, double eps,
            int32_t yz_swap, int32_t* nonfinite) {
    constexpr int NW = kFinalBlock / 64;
    __shared__ double red[NW];
    __shared__ double tot[2 * kAdjMaxPhase + kAdjMaxPhase * kAdjMaxPhase];
    __shared__ double scan[kFinalBlock];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t nkf = (int64_t)K * n_fields;
    // per-phase and per-pair totals over all steps and fields
    const int NT = 2 * P + P * P;
    for (int g = 0; g < NT; ++g) {
        double v = 0.0;
        for (int64_t i = t; i < nkf; i += kFinalBlock) v += gfield[i * NG + g];
        v = wave_sum(v);
        if (lane == 0) red[wv] = v;
        __syncthreads();
        if (t == 0) {
            double sacc = 0.0;
            for (int i = 0; i < NW; ++i) sacc += red[i];
            tot[g] = sacc;
        }
        __syncthreads();
    }
    // a non-finite gradient is reported to the host (sticky flag)
    auto flag = [nonfinite](double v) {
        if (nonfinite != nullptr && !isfinite(v)) *nonfinite = 1;
    };
    if (t < P) {
        if (dD) {
            const double wp = w[t];
            dD[t] = tot[t] * (-wp * wp * dt / (eps * dx * dx));
            flag(dD[t]);
        }
        if (dT2) {
            const double T = T2[t];
            const double dec = isinf(T) ? 1.0 : exp(-dt / T);
            dT2[t] = isinf(T) ? 0.0 : tot[P + t] * dec * dt / (T * T);
            flag(dT2[t]);
        }
    }
    if (t < P * P && dkappa) {
        const int i = t / P, j = t % P;
        const double k = kappa[t];
        // gradient per matrix entry: the two entries of a pair share the
        // pair's derivative equally, so that they sum to dL/dkappa_pair
        double g = tot[2 * P + i * P + j];
        if (i != j) g = 0.5 * (g + tot[2 * P + j * P + i]);
        // t = 2 k dt / (eps_D dx + 2 k dt)
        const double den = eps * dx + 2.0 * k * dt;
        dkappa[t] = isinf(k) ? 0.0 : g * 2.0 * dt * eps * dx / (den * den);
        flag(dkappa[t]);
    }
    if (df) {   // the same for every thread: the barriers below are uniform
        const int IF = 2 * P + P * P, IFF = IF + 1;
        auto field_sum = [&](int32_t m, int idx) {
            double v = 0.0;
            for (int f = 0; f < n_fields; ++f) v += gfield[((int64_t)m * n_fields + f) * NG + idx];
            return v;
        };
        const int32_t chunk = (K + kFinalBlock - 1) / kFinalBlock;
        const int32_t m0 = min(K, t * chunk), m1 = min(K, m0 + chunk);
        double cF = 0.0;
        for (int32_t m = m0; m < m1; ++m) cF += field_sum(m, IFF);
        scan[t] = cF;
        __syncthreads();
        // scan[t] becomes the sum of the chunks t .. end
        for (int off = 1; off < kFinalBlock; off <<= 1) {
            const double v = t + off < kFinalBlock ? scan[t + off] : 0.0;
            __syncthreads();
            scan[t] += v;
            __syncthreads();
        }
        double suffix = t + 1 < kFinalBlock ? scan[t + 1] : 0.0;   // sum_{k >= m1} G_F[k]
        for (int32_t m = m1 - 1; m >= m0; --m) {
            const double v = (field_sum(m, IF) + dt * suffix) / sub;
            for (int j = 0; j < sub; ++j) df[(int64_t)m * sub + j] = v;
            flag(v);
            suffix += field_sum(m, IFF);
        }
    }
    // dL/d(gamma G0)_b of q-sample q, summed over its fields and the steps:
    //   fdt_k dx (s_b R_b - sigma_b R_0) + F_k sum_f (d beta_f / d G_b) X_f
    if (dgG0) {
        const int IR = 2 * P + P * P + 2, IX = IR + 4;
        for (int i = wv; i < 3 * Q; i += NW) {
            const int q = i / 3, b = i % 3;
            double acc = 0.0;
            for (int f = 0; f < n_fields; ++f) {
                const double* gm = gmeta + (int64_t)f * kGMeta;
                if ((int)gm[0] != q) continue;
                const double sb = gm[1 + b], sgb = gm[4 + b];
                for (int32_t k = lane; k < K; k += 64) {
                    const double* r = gfield + ((int64_t)k * n_fields + f) * NG;
                    double xs = 0.0;
                    for (int fc = 0; fc < 6; ++fc) xs += gm[7 + 3 * fc + b] * r[IX + fc];
                    acc += fdt[k] * dx * (sb * r[IR + b] - sgb * r[IR + 3]) + Fk[k] * xs;
                }
            }
            acc = wave_sum(acc);
            // kernel axes back to the geometry's: the single-layer lattice
            // runs with the geometry's y axis as the kernel's z axis
            // (its z component is not a parameter there: the layer has no
            // extent along z, and the input must be 0; reported as 0)
            const int bg = yz_swap ? (b == 1 ? 2 : b == 2 ? 1 : 0) : b;
            if (lane == 0) {
                dgG0[3 * q + bg] = (yz_swap && bg == 2) ? 0.0 : acc;
                flag(acc);
            }
        }
    }
}

template <typename V, int TX, int NQ, int NP>
static void launch_adj_np(const AdjArgs& a, int32_t n_blocks, hipStream_t st) {
    // the gamma G0 sensitivities take their own instantiation (more
    // accumulators); FP32 without them is held to four waves per SIMD
    if (a.gradg)
        hipLaunchKernelGGL((k_adj<V, TX, true, NQ, NP>), dim3(n_blocks), dim3(kBlock), 0, st, a);
    else if constexpr (std::is_same<V, float2>::value)
        hipLaunchKernelGGL((k_adj_w4<V, TX, false, NQ, NP>), dim3(n_blocks), dim3(kBlock), 0, st,
                           a);
    else
        hipLaunchKernelGGL((k_adj<V, TX, false, NQ, NP>), dim3(n_blocks), dim3(kBlock), 0, st, a);
}

template <typename V, int TX, int NQ>
static void launch_adj_tx(const AdjArgs& a, int32_t n_blocks, hipStream_t st) {
    if (a.n_phase <= 2)
        launch_adj_np<V, TX, NQ, 2>(a, n_blocks, st);
    else
        launch_adj_np<V, TX, NQ, kAdjMaxPhase>(a, n_blocks, st);
}

template <typename V>
static void launch_adj_t(int shape, const AdjArgs& a, int32_t n_blocks, hipStream_t st) {
    if (a.nq == 5) {   // single layer: y rows walked as columns, 256 x 1 tiles
        launch_adj_tx<V, 256, 5>(a, n_blocks, st);
        return;
    }
    switch (shape) {
        case kTile64x4: launch_adj_tx<V, 64, 7>(a, n_blocks, st); break;
        case kTile32x8: launch_adj_tx<V, 32, 7>(a, n_blocks, st); break;
        case kTile128x2: launch_adj_tx<V, 128, 7>(a, n_blocks, st); break;
        case kTileRows: launch_adj_tx<V, 0, 7>(a, n_blocks, st); break;
        default: launch_adj_tx<V, 16, 7>(a, n_blocks, st); break;
    }
}

hipError_t launch_adj(int prec, int shape, const AdjArgs& a, int32_t n_blocks, hipStream_t st) {
    if (prec == 1)
        launch_adj_t<float2>(shape, a, n_blocks, st);
    else
        launch_adj_t<double2>(shape, a, n_blocks, st);
    return hipGetLastError();
}

hipError_t launch_adj_gsum(const double* gpart, const FieldDesc* d_fields, int32_t n_fields,
                           int32_t nblk_total, int32_t ng, int32_t k_first, int32_t nsteps,
                           double* gfield, int32_t f_off, int32_t nf_total, hipStream_t st) {
    const int64_t n = (int64_t)nsteps * n_fields * ng;
    if (n > 0)
        hipLaunchKernelGGL(k_adj_gsum, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, st, gpart, d_fields, n_fields, nblk_total, ng, k_first, nsteps,
                           gfield, f_off, nf_total);
    return hipGetLastError();
}

__global__ void k_mark() {}

hipError_t launch_mark(hipStream_t st) {
    hipLaunchKernelGGL(k_mark, dim3(1), dim3(64), 0, st);
    return hipGetLastError();
}

hipError_t launch_adj_final(const double* gfield, int32_t K, int32_t n_fields, int32_t P,
                            double dt, double dx, const double* w, const double* T2,
                            const double* kappa, double* dD, double* dT2, double* dkappa,
                            double* df, int32_t sub, int32_t ng, const double* gmeta,
                            const double* fdt, const double* Fk, int32_t Q, double* dgG0,
                            double eps, int32_t yz_swap, int32_t* nonfinite, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_final, dim3(1), dim3(kFinalBlock), 0, st, gfield, K, n_fields, P, dt, dx,
                       w, T2, kappa, dD, dT2, dkappa, df, sub, ng, gmeta, fdt, Fk, Q, dgG0,
                       eps, yz_swap, nonfinite);
    return hipGetLastError();
}

}  // namespace btl
