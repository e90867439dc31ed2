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
//   3. M = sum_i g_i; each wave adds M into its signal partial sum
//      (Eq. M'summation; signal Sec. 2.1)
//   4. ghat_i = g_i + w (w_i M - g_i), w = 1/tau       (Eq. collision_LBM)
// which is the paper's collide -> stream -> react cycle (Eq.
// LBM_process_list_2) started at the stream.  The classical LBM of Appendix A
// (Eq. A12) shares steps 1 and 3 and moves the reaction into step 4.  All
// arithmetic is FP64; populations are stored as float2 or double2, per field
// z-major: [z][direction][y][x] (the seven planes of one z layer lie
// together, so the tiles that run at the same time read and write one
// compact region).  Per-step constants enter only through forms that keep
// sum_i g_i exact for any rounded constant (g + w(wM - g), a + t(b - a)).
//
// With membrane positions given, a membrane link whose six-node stencil lies
// inside the field takes the general condition for a straight membrane at
// that position (Eqs. B2a_text/B2b_text, B4a-B4c) instead of the half-link
// form (GM = true; other links keep the half-link form).  With membrane
// normals as well (CV = true), links whose stencil for the condition at any
// angle exists (Appendix B, Eqs. phi_1, phi_2) take the population k_links
// evaluated for them from the host-built term list (a weighted sum of
// post-collision populations around the link), link-parallel, before the
// step.
//
// The signal of a step is reduced deterministically: each wave writes its
// partial sum to a per-step slot, and k_esum (one launch per 32 steps) adds
// the partials of every field in a fixed order.
#include <type_traits>

#include "btl_device.h"

namespace btl {

template <typename V>
__global__ void __launch_bounds__(kBlock) k_init(V* pop, int64_t nsites, int64_t st2, double2* E,
                                                  int32_t q, int32_t K, int32_t nq) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < nsites * nq) {
        const int d = (int)((e / st2) % nq);   // z-major layout: [z][plane][y][x]
        store2(pop + e, make_double2(d == 0 ? lattice_w0(nq) : lattice_w1(nq), 0.0));
    }
    if (E != nullptr && q >= 0 && e == 0) E[(int64_t)q * (K + 1)] = make_double2(1.0, 0.0);
}

// Entry e of the phase table of step k (see FieldDesc::tab).
__device__ __forceinline__ double2 table_entry(const StepArgs& a, int32_t e, int32_t k) {
    const int fi = a.tab_field[e];
    const FieldDesc& fd = a.fields[fi];
    const int32_t l = e - fd.tab;
    const double fdt = a.fdt[k];
    const int32_t n0 = fd.n[0], n1 = fd.n[1], n2 = fd.n[2];
    if (l < n0) return expi(-fdt * fd.c[0] * (double)l);
    if (l < n0 + n1) return expi(-fdt * fd.c[1] * (double)(l - n0));
    if (l < n0 + n1 + n2) return expi(-fdt * (fd.c[2] * (double)(l - n0 - n1) + fd.cu));
    const double beta = fd.beta[l - n0 - n1 - n2];
    return beta != 0.0 ? expi(beta * a.Fk[k]) : make_double2(1.0, 0.0);
}

__global__ void __launch_bounds__(kBlock) k_tables(StepArgs a, int32_t nsteps) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)nsteps * a.T) return;
    const int32_t ks = (int32_t)(i / a.T);
    const int32_t e = (int32_t)(i - (int64_t)ks * a.T);
    a.tab[i] = table_entry(a, e, a.k + ks);
}

// One step for a tile of TX x TY site columns (TX = 0: a run of kBlock
// consecutive sites of the x-y plane), each thread walking fd.zc sites along
// z.  Workgroup -> (field, block) via blk_field, whose order the host picks,
// and the field's tile counts; no per-site integer division.  The signal
// partials go to the field-major slot of the block, whatever the order.
//
// CL = true runs the classical LBM (Appendix A, Eq. A12) with the same
// streaming: step 2 is skipped and step 4 adds dt w_i R M with
// R = -i gamma (x.G0) f_{k+1} - 1/T2, the reaction term of the collision that
// follows the moment M(t^{k+1}).  The last step stores the plain collision,
// whose moment is M(t^K).
template <typename V, int TX, bool CL, bool GM, int NQ, bool CV, bool FIRST>
__device__ __forceinline__ void step_body(const StepArgs& a) {
    constexpr int TY = TX > 0 ? kBlock / TX : 1;
    constexpr double W0 = lattice_w0(NQ), W1 = lattice_w1(NQ);
    static_assert(!FIRST || (!CL && !CV), "the first-step form is for the hybrid scheme "
                                          "without curved links");
    // Plane p >= 1 moves along kernel direction kd(p): D3Q7 p itself; the
    // single-layer D2Q5 lattice runs with its y axis as the kernel's z axis
    // (planes 3, 4 pull along z), while site words and membrane positions
    // keep the geometry's own direction numbering, which is p.
    auto face_of = [](int p) { return NQ == 7 ? p - 1 : (p <= 2 ? p - 1 : p + 1); };
    __shared__ double c_w[kMaxPhase], c_dec[kMaxPhase], c_tr[kMaxPhase * kMaxPhase];
    __shared__ double c_kdt[GM ? kMaxPhase * kMaxPhase : 1];
    __shared__ double2 c_ez[CL ? 1 : kMaxZc];   // z phase factors of this tile's column range
    // per-phase constants in LDS: lane-indexed lookups then go through the
    // LDS counter and never wait on outstanding global loads or stores
    {
        const int t = threadIdx.x, P = a.n_phase;
        if (t < P) {
            c_w[t] = a.w[t];
            c_dec[t] = CL ? a.rdt[t] : a.decay[t];
        }
        if (t < P * P) c_tr[t] = a.trans[t];
        if (GM && t < P * P) c_kdt[t] = a.kdt[t];
    }
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
    const double2* __restrict__ tab = a.tab + fd.tab;
    const double2* __restrict__ ez = tab + n0 + n1;
    // the z phase factors of the column range [z0, z0 + zc) go to LDS once
    // (zc <= kMaxZc), so that the pipelined per-site loads do not carry them
    if (!CL)
        for (int i = threadIdx.x; i < fd.zc && z0 + i < n2; i += kBlock) c_ez[i] = ez[z0 + i];
    __syncthreads();
    double2 face_fac[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) face_fac[f] = uniform2(tab[n0 + n1 + n2 + f]);
    const int P = a.n_phase;

    // one base pointer per buffer for this field; every access is a 32-bit
    // element offset from it (image-field partners of the same q-sample lie
    // within +-2^31 elements, checked on the host)
    const V* __restrict__ src = static_cast<const V*>(a.src) + fd.pop;
    V* __restrict__ dst = static_cast<V*>(a.dst) + fd.pop;
    // FIRST: the first step of a forward starts from the equilibrium at
    // M = 1, where plane 0 holds w0 and every other plane w1 at every site;
    // those constants, rounded to the storage type as a stored state would
    // be, stand in for the loads (no initial state is written or read)
    V cw0, cw1;
    store2(&cw0, make_double2(W0, 0.0));
    store2(&cw1, make_double2(W1, 0.0));
    auto lds = [&](int32_t off, const V& c) -> V {
        if constexpr (FIRST) {
            (void)off;
            return c;
        } else {
            (void)c;
            return src[off];
        }
    };
    const uint32_t* __restrict__ words = a.words + fd.words;
    const float* __restrict__ gmt = GM && fd.gm >= 0 ? a.gm + fd.gm : nullptr;
    // curved membranes (CV): per pull link -1 or the link's term list
    const uint8_t* __restrict__ cvmp = CV && fd.cv >= 0 ? a.cvm + fd.cv : nullptr;
    const int32_t pop = 0;
    int32_t j0, j1;
    if constexpr (TX == 0) {   // kTileRows: kBlock consecutive sites of the x-y plane
        const int32_t i = tx * kBlock + (int32_t)threadIdx.x;
        j0 = i % n0;
        j1 = i / n0;
    } else {
        j0 = tx * TX + (int32_t)(threadIdx.x % TX);
        j1 = ty * TY + (int32_t)(threadIdx.x / TX);
    }
    const int32_t z1 = min(n2, z0 + fd.zc);
    // site index s = j0 + st1 j1 + st2 j2 (site words, membrane positions);
    // populations: plane d of site (j0, j1, j2) at d ps + j0 + st1 j1 + zs j2
    const int32_t st1 = n0, st2 = n0 * n1, ps = st2, zs = NQ * st2;
    const double2 exy = CL ? make_double2(0.0, 0.0)
                           : cmul(tab[min(j0, n0 - 1)], tab[n0 + min(j1, n1 - 1)]);
    // classical: dt R = ra + i rb with rb = -f_{k+1} dt (c.j + cu)
    const bool cl_term = CL && a.k + 1 < a.K;
    const double fdt1 = cl_term ? a.fdt[a.k + 1] : 0.0;
    const double rb_xy = -fdt1 * (fd.c[0] * (double)j0 + fd.c[1] * (double)j1 + fd.cu);
    const double rb_z = -fdt1 * fd.c[2];

    // Source offset (relative to the site index s) of each pulled direction,
    // fixed for the whole z column for x and y; z faces switch per site.
    // Interior: same field, neighbour site.  Periodic face: same field,
    // wrapped site.  Mirror face: source field of that face, same site,
    // reflected direction.
    int32_t kind[6];
    int32_t fpop[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        kind[f] = fd.face_kind[f];
        fpop[f] = (int32_t)(fd.face_pop[f] - fd.pop);
    }
    auto face_off = [&](int f, int d, int32_t wrap) -> int32_t {
        const int db = (d & 1) ? d + 1 : d - 1;
        return (kind[f] & kFaceMirror) ? fpop[f] + db * ps : fpop[f] + d * ps + wrap;
    };
    const bool fx0 = j0 == 0, fx1 = j0 == n0 - 1, fy0 = j1 == 0, fy1 = j1 == n1 - 1;
    const int32_t o1 = fx0 ? face_off(0, 1, n0 - 1) : pop + 1 * ps - 1;
    const int32_t o2 = fx1 ? face_off(1, 2, -(n0 - 1)) : pop + 2 * ps + 1;
    const int32_t o3 = fy0 ? face_off(2, 3, (n1 - 1) * st1) : pop + 3 * ps - st1;
    const int32_t o4 = fy1 ? face_off(3, 4, -(n1 - 1) * st1) : pop + 4 * ps + st1;
    // z pulls of planes pz (+z) and pz + 1 (-z): interior and face offsets
    constexpr int pz = NQ == 7 ? 5 : 3;
    const int32_t o5i = pop + pz * ps - zs, o5f = face_off(4, pz, (n2 - 1) * zs);
    const int32_t o6i = pop + (pz + 1) * ps + zs, o6f = face_off(5, pz + 1, -(n2 - 1) * zs);

    // Loads of one site: the site word, the pulled populations and the
    // outgoing populations of the node itself (reflected at membrane links).
    // Along the column two of them are shared between neighbours: plane pz
    // at site j2 is both the node's own population of direction pz + 1 and
    // the pz pull of site j2 + 1, and plane pz + 1 at site j2 + 1 is both the
    // pz + 1 pull of site j2 and the own population of direction pz of site
    // j2 + 1.  Each is loaded once and carried to the next site (cz_g, cz_o),
    // so a site issues NQ + 3 loads (D3Q7: 12 of the 14 values it uses).
    // Without the general membrane condition the z column is
    // software-pipelined: the loads of site j2 + 1 are issued before the
    // stores of site j2, so waiting for a site's data never waits for
    // earlier stores.
    struct SiteLoads {
        uint32_t word;
        V g[NQ];          // g[pz] is carried, not loaded
        V own[NQ - 1];    // own[pz - 1] is carried, not loaded
        float gv[GM ? NQ - 1 : 1];   // membrane positions of the pull links
        uint32_t cvm;                 // pull links under the curved rule (bit d - 1)
    };
    auto cv_of = [](const SiteLoads& L, int d) -> bool {
        if constexpr (CV) return ((L.cvm >> (d - 1)) & 1u) != 0;
        else return false;
    };
    auto issue = [&](int32_t j2, SiteLoads& L) {
        const int32_t s = j0 + st1 * j1 + st2 * j2;
        const int32_t sp = j0 + st1 * j1 + zs * j2;
        L.word = words[s];
        L.g[0] = lds(pop + sp, cw0);
        L.g[1] = lds(o1 + sp, cw1);
        L.g[2] = lds(o2 + sp, cw1);
        if constexpr (NQ == 7) {
            L.g[3] = lds(o3 + sp, cw1);
            L.g[4] = lds(o4 + sp, cw1);
        }
        L.g[pz + 1] = lds((j2 == n2 - 1 ? o6f : o6i) + sp, cw1);
#pragma unroll
        for (int d = 1; d < NQ; ++d) {
            const int od = (d & 1) ? d + 1 : d - 1;
            if (d != pz) L.own[d - 1] = lds(pop + od * ps + sp, cw1);
        }
        if constexpr (GM) {
#pragma unroll
            for (int d = 1; d < NQ; ++d) L.gv[d - 1] = gmt ? gmt[(d - 1) * ns + s] : 0.0f;
        }
        if constexpr (CV) L.cvm = cvmp ? (uint32_t)cvmp[s] : 0u;
    };
    // General membrane links of a site (GM): which links take the general
    // condition, and the three stencil populations of the first two of them,
    // loaded as soon as the site's own data have arrived (a site with more
    // general links loads the others when it computes them).
    struct GmPre {
        uint32_t gen;
        uint32_t cvb;       // the general links that take the curved rule
        int d0, d1;
        V st0[3], st1[3];   // ghat_ibar(x + e_i), ghat_i(x - 2 e_i), ghat_ibar(x - e_i)
        int c0;             // the first curved link
        V cvv;              // its arriving population (left by k_links)
    };
    // plane offsets of the stencil of pull link d (relative to the site)
    auto stencil_off = [&](int d, int32_t* o) {
        const int od = (d & 1) ? d + 1 : d - 1;
        const int32_t sa = d <= 2 ? 1 : (NQ == 7 && d <= 4) ? st1 : zs;
        const int32_t e = (d & 1) ? sa : -sa;
        o[0] = od * ps + e;
        o[1] = d * ps - 2 * e;
        o[2] = od * ps - e;
    };
    auto prep = [&](int32_t j2, const SiteLoads& L, GmPre& G) {
        G.gen = 0;
        G.cvb = 0;
        G.d0 = 0;
        G.d1 = 0;
        G.c0 = 0;
        if constexpr (GM) {
            const uint32_t word = L.word;
            const int p = (int)(word & 0xfu);
            const uint32_t mask = (word >> 4) & 0x3fu;
#pragma unroll
            for (int d = 1; d < NQ; ++d) {
                const bool cvd = cv_of(L, d);
                if (((mask >> (d - 1)) & 1u) && (L.gv[d - 1] != 0.0f || cvd)) {
                    const int pn = (int)((word >> (10 + 3 * (d - 1))) & 0x7u);
                    if (c_tr[p * P + pn] < 1.0) {
                        G.gen |= 1u << d;
                        if (cvd) G.cvb |= 1u << d;
                    }
                }
            }
            const int32_t sp = j0 + st1 * j1 + zs * j2;
            if constexpr (CV) {
                // the arriving population of the first curved link
                if (G.cvb) {
                    G.c0 = __builtin_ctz(G.cvb);
                    G.cvv = dst[sp + G.c0 * ps];
                }
            }
            // stencils of the first two links with the theta = 0 rule
            const uint32_t g0 = G.gen & ~G.cvb;
            if (g0) {
                int32_t o[3];
                G.d0 = __builtin_ctz(g0);
                stencil_off(G.d0, o);
                G.st0[0] = lds(sp + o[0], cw1);
                G.st0[1] = lds(sp + o[1], cw1);
                G.st0[2] = lds(sp + o[2], cw1);
                const uint32_t rest = g0 & (g0 - 1);
                if (rest) {
                    G.d1 = __builtin_ctz(rest);
                    stencil_off(G.d1, o);
                    G.st1[0] = lds(sp + o[0], cw1);
                    G.st1[1] = lds(sp + o[1], cw1);
                    G.st1[2] = lds(sp + o[2], cw1);
                }
            }
        }
    };
    // carried along the column: the pz pull and the direction-pz own
    // population of the next site to compute (loaded for the first site)
    V cz_g, cz_o;
    auto compute = [&](int32_t j2, const SiteLoads& L, const GmPre& G, double2& Macc) {
        const int32_t s = j0 + st1 * j1 + st2 * j2;
        const int32_t sp = j0 + st1 * j1 + zs * j2;
        const bool fz0 = j2 == 0, fz1 = j2 == n2 - 1;
        const uint32_t word = L.word;
        const int p = (int)(word & 0xfu);
        const uint32_t mask = (word >> 4) & 0x3fu;
        V own[NQ - 1];
#pragma unroll
        for (int d = 1; d < NQ; ++d) own[d - 1] = d == pz ? cz_o : L.own[d - 1];
        double2 g[NQ];
#pragma unroll
        for (int d = 0; d < NQ; ++d) g[d] = ld2(d == pz ? &cz_g : &L.g[d]);
        cz_g = L.own[pz];       // plane pz at j2: the pz pull of j2 + 1
        cz_o = L.g[pz + 1];     // plane pz + 1 at j2 + 1 (an interior pull when j2 + 1 < n2)
        const bool face[6] = {fx0, fx1, fy0, fy1, fz0, fz1};
#pragma unroll
        for (int p = 1; p < NQ; ++p) {
            const int f = face_of(p);
            if (face[f]) {
                double2 v = g[p];
                if (kind[f] & kFaceConj) v.y = -v.y;
                g[p] = cmul(v, face_fac[f]);
            }
        }
        if (mask) {
            // half-link membrane: g' = ghat_opp(x) + t (incoming - ghat_opp(x)),
            // except on the links that take the general condition (G.gen)
#pragma unroll
            for (int d = 1; d < NQ; ++d) {
                if (((mask >> (d - 1)) & 1u) && !((G.gen >> d) & 1u)) {
                    const int pn = (int)((word >> (10 + 3 * (d - 1))) & 0x7u);
                    const double t = c_tr[p * P + pn];
                    if (t < 1.0) {
                        const double2 o = ld2(&own[d - 1]);
                        g[d].x = o.x + t * (g[d].x - o.x);
                        g[d].y = o.y + t * (g[d].y - o.y);
                    }
                }
            }
            if (GM) {
                // general condition, one link at a time (rolled: the code
                // exists once); the stencil x - 2e_d .. x + e_d lies inside
                // the field (checked on the host)
                uint32_t gen = G.gen;
                while (gen) {
                    const int d = __builtin_ctz(gen);
                    gen &= gen - 1;
                    if (CV && ((G.cvb >> d) & 1u)) {
                        // membrane at an angle: k_links left the link's
                        // arriving population at (site, d) of the
                        // destination state before this step
                        double2 r;
                        if (d == G.c0) r = ld2(&G.cvv);
                        else r = ld2(dst + sp + d * ps);
#pragma unroll
                        for (int k = 1; k < NQ; ++k)
                            if (d == k) g[k] = r;
                        continue;
                    }
                    // own[k-1] holds ghat_{opp(k)}(x): both populations of x
                    // on the link's axis are already loaded
                    double2 b1 = g[1], o = ld2(&own[0]), a3 = ld2(&own[1]);
                    float v = L.gv[0];
#pragma unroll
                    for (int k = 2; k < NQ; ++k)
                        if (d == k) {
                            const int ok = (k & 1) ? k + 1 : k - 1;
                            b1 = g[k];
                            o = ld2(&own[k - 1]);
                            a3 = ld2(&own[ok - 1]);
                            v = L.gv[k - 1];
                        }
                    const int pn = (int)((word >> (10 + 3 * (d - 1))) & 0x7u);
                    const double dd = v > 0.0f ? (double)v : 1.0 + (double)v;
                    const MembCoef c = membrane_coefficients(dd, c_kdt[p * P + pn], a.edx);
                    double2 a2, b2, b3;
                    if (d == G.d0) {
                        a2 = ld2(&G.st0[0]);
                        b2 = ld2(&G.st0[1]);
                        b3 = ld2(&G.st0[2]);
                    } else if (d == G.d1) {
                        a2 = ld2(&G.st1[0]);
                        b2 = ld2(&G.st1[1]);
                        b3 = ld2(&G.st1[2]);
                    } else {
                        int32_t o3[3];
                        stencil_off(d, o3);
                        const V s0 = lds(sp + o3[0], cw1), s1 = lds(sp + o3[1], cw1),
                                s2 = lds(sp + o3[2], cw1);
                        a2 = ld2(&s0);
                        b2 = ld2(&s1);
                        b3 = ld2(&s2);
                    }
                    double2 r;
                    r.x = c.A[0] * o.x + c.A[1] * a2.x + c.A[2] * a3.x
                        + c.B[0] * b1.x + c.B[1] * b2.x + c.B[2] * b3.x;
                    r.y = c.A[0] * o.y + c.A[1] * a2.y + c.A[2] * a3.y
                        + c.B[0] * b1.y + c.B[1] * b2.y + c.B[2] * b3.y;
#pragma unroll
                    for (int k = 1; k < NQ; ++k)
                        if (d == k) g[k] = r;
                }
            }
        }
        double2 M = make_double2(0.0, 0.0);
        if (!CL) {
            // reaction: exp(-i fdt (c.j + cu)) exp(-dt/T2)
            const double2 e = cmul(exy, uniform2(c_ez[j2 - z0]));   // same for every lane
            const double dec = c_dec[p];
            const double2 rf = make_double2(e.x * dec, e.y * dec);
#pragma unroll
            for (int d = 0; d < NQ; ++d) g[d] = cmul(g[d], rf);
        }
#pragma unroll
        for (int d = 0; d < NQ; ++d) {
            M.x += g[d].x;
            M.y += g[d].y;
        }
        Macc.x += M.x;
        Macc.y += M.y;
        // classical reaction term dt R M (zero on the last step)
        double2 RM = make_double2(0.0, 0.0);
        if (CL) {
            const double ra = cl_term ? -c_dec[p] : 0.0;
            const double rb = rb_xy + rb_z * (double)j2;
            RM = make_double2(ra * M.x - rb * M.y, ra * M.y + rb * M.x);
        }
        // collision: ghat = g + w (w_d M - g)  [+ w_d dt R M]
        const double w = c_w[p];
        V* out = dst + sp;
#pragma unroll
        for (int d = 0; d < NQ; ++d) {
            const double wd = d == 0 ? W0 : W1;
            double2 h;
            h.x = g[d].x + w * (wd * M.x - g[d].x);
            h.y = g[d].y + w * (wd * M.y - g[d].y);
            if (CL) {
                h.x += wd * RM.x;
                h.y += wd * RM.y;
            }
            store2_stream(out + d * ps, h);
        }
    };

    double2 Mv = make_double2(0.0, 0.0);
    if (j0 < n0 && j1 < n1 && z0 < z1) {
        {
            const int32_t sp = j0 + st1 * j1 + zs * z0;
            cz_g = lds((z0 == 0 ? o5f : o5i) + sp, cw1);
            cz_o = lds(pop + (pz + 1) * ps + sp, cw1);
        }
        if constexpr (GM || std::is_same<V, double2>::value) {
            // one site at a time: the general condition's stencil loads and
            // coefficient arithmetic leave no registers for a second site in
            // flight, and the occupancy this keeps pays more than the overlap.
            // FP64 storage too: a site's loads are twice the bytes of an FP32
            // site, and one site in flight (92 VGPRs, five waves per SIMD)
            // ran at 0.769 of peak on the 256^3 batch against 0.744 with two
            // (168 VGPRs, three waves)
            SiteLoads A;
            GmPre G;
            for (int32_t j2 = z0; j2 < z1; ++j2) {
                issue(j2, A);
                prep(j2, A, G);
                compute(j2, A, G, Mv);
            }
        } else {
            SiteLoads A, B;
            GmPre G;
            issue(z0, A);
            int32_t j2 = z0;
            // two sites per trip so that A and B swap roles without copies
            for (; j2 + 1 < z1; j2 += 2) {
                prep(j2, A, G);
                issue(j2 + 1, B);
                compute(j2, A, G, Mv);
                prep(j2 + 1, B, G);
                if (j2 + 2 < z1) issue(j2 + 2, A);
                compute(j2 + 1, B, G, Mv);
            }
            if (j2 < z1) {
                prep(j2, A, G);
                compute(j2, A, G, Mv);
            }
        }
    }

    if (fd.q < 0) return;   // image fields do not enter the signal
    // Per-wave partial of the signal; k_esum adds them up in a fixed order
    // after the step (no fence or atomic here: a device-scope release at the
    // end of every workgroup stalled the whole step).
    const double mx = wave_sum(Mv.x), my = wave_sum(Mv.y);
    if ((threadIdx.x & 63) == 0)
        a.partial[((size_t)(a.k % kTabSteps) * gridDim.x + fd.blk0 + b) * (kBlock / 64) +
                  (threadIdx.x >> 6)] = make_double2(mx, my);
}

// The arriving population of every curved membrane link (a membrane at an
// angle to the link, Appendix B) of every field, one thread per (link, group
// of fields): the host-built term list of the link -- a weighted sum of
// post-collision populations of step k around it, each times the periodic
// face factors its node lies beyond -- evaluated in FP64 and stored at
// (receiving site, pull direction) of the destination state, where the step
// kernel then reads it.  Workgroup -> (run of kBlock consecutive links,
// group of kLinkFields consecutive fields), the groups of a run on
// consecutive workgroups.  A thread reads its link's term list once for the
// fields of its group that share the geometry of the first of them (their
// populations then load together, kLinkTerms terms at a time: a link waits
// two memory round trips per kLinkTerms terms, not per term and field), and
// evaluates any other field of the group on its own.  Eight terms per batch
// ran the pass 5-12 % faster than four on the 96^3 and 128^3 packings;
// twelve or sixteen, and groups of eight or twelve fields, were slower.
constexpr int kLinkFields = 4;
constexpr int kLinkTerms = 8;

template <typename V>
__global__ void __launch_bounds__(kBlock) k_links(StepArgs a, int32_t n_fields) {
    const int32_t ngrp = (n_fields + kLinkFields - 1) / kLinkFields;
    const int32_t grp = (int32_t)(blockIdx.x % (unsigned)ngrp);
    const int64_t l = (int64_t)(blockIdx.x / (unsigned)ngrp) * kBlock + threadIdx.x;
    const int32_t f0 = grp * kLinkFields, f1 = min(n_fields, f0 + kLinkFields);
    int lead = -1;
    for (int f = f0; f < f1; ++f)
        if (a.fields[f].cv >= 0 && l < a.fields[f].cv_nh) {
            lead = f;
            break;
        }
    if (lead < 0) return;
    const int64_t lead_cv = a.fields[lead].cv;
    int nf = 0;
    int32_t fs[kLinkFields];
    for (int f = lead; f < f1; ++f)
        if (a.fields[f].cv == lead_cv) fs[nf++] = f;
    auto eval = [&](const int32_t* fl, int n) {
        const FieldDesc& fd = a.fields[fl[0]];
        const int4 hd = a.cvh[fd.cv_h0 + l];
        const int tend = hd.x + hd.y;
        double2 acc[kLinkFields];
        const V* srcs[kLinkFields];
        const double2* ftab[kLinkFields];
#pragma unroll
        for (int j = 0; j < kLinkFields; ++j) {
            acc[j] = make_double2(0.0, 0.0);
            const FieldDesc& fj = a.fields[fl[j < n ? j : 0]];
            srcs[j] = static_cast<const V*>(a.src) + fj.pop + hd.z;
            ftab[j] = a.tab + fj.tab + fj.n[0] + fj.n[1] + fj.n[2];
        }
        for (int t0 = hd.x; t0 < tend; t0 += kLinkTerms) {
            CvTerm tm[kLinkTerms];
#pragma unroll
            for (int u = 0; u < kLinkTerms; ++u)
                if (t0 + u < tend) tm[u] = a.cvt[t0 + u];
            V pv[kLinkFields][kLinkTerms];
#pragma unroll
            for (int j = 0; j < kLinkFields; ++j)
                if (j < n) {
#pragma unroll
                    for (int u = 0; u < kLinkTerms; ++u)
                        if (t0 + u < tend) pv[j][u] = srcs[j][tm[u].off];
                }
#pragma unroll
            for (int j = 0; j < kLinkFields; ++j) {
                if (j >= n) break;
#pragma unroll
                for (int u = 0; u < kLinkTerms; ++u) {
                    if (t0 + u >= tend) break;
                    double2 v = ld2(&pv[j][u]);
                    if (tm[u].wrap) {
                        for (int fc = 0; fc < 6; ++fc)
                            for (int rp = (tm[u].wrap >> (2 * fc)) & 3; rp > 0; --rp)
                                v = cmul(v, ftab[j][fc]);
                    }
                    acc[j].x += tm[u].w * v.x;
                    acc[j].y += tm[u].w * v.y;
                }
            }
        }
        const int32_t ps = fd.n[0] * fd.n[1];
#pragma unroll
        for (int j = 0; j < kLinkFields; ++j)
            if (j < n)
                store2(static_cast<V*>(a.dst) + a.fields[fl[j]].pop + hd.z + hd.w * ps, acc[j]);
    };
    eval(fs, nf);
    // the group's fields on other geometries, one by one (ragged batches)
    for (int f = lead + 1; f < f1; ++f) {
        const FieldDesc& fd = a.fields[f];
        if (fd.cv >= 0 && fd.cv != lead_cv && l < fd.cv_nh) {
            const int32_t one[1] = {f};
            eval(one, 1);
        }
    }
}

// E_{k+1} = (1/N) sum of the per-wave partials of a primary field, one wave
// per (field, step): lanes stride over the field's partials in order, then a
// fixed shuffle tree, so the signal is bitwise reproducible.
__global__ void __launch_bounds__(kBlock) k_esum(const double2* __restrict__ partial,
                                                 const FieldDesc* __restrict__ fields,
                                                 int32_t n_fields, int32_t nblk_total,
                                                 int32_t k0, int32_t nsteps, double2* E,
                                                 int32_t K, int32_t* nonfinite) {
    const int32_t pair = (int32_t)blockIdx.x * (kBlock / 64) + (int32_t)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (pair >= n_fields * nsteps) return;   // whole waves leave together
    const int32_t fi = pair / nsteps, j = pair % nsteps;
    const FieldDesc& fd = fields[fi];
    if (fd.q < 0) return;
    const int32_t k = k0 + j;
    const double2* p = partial + ((size_t)(k % kTabSteps) * nblk_total + fd.blk0) * (kBlock / 64);
    const int32_t n = fd.nblk * (kBlock / 64);
    double sx = 0.0, sy = 0.0;
    for (int32_t i = lane; i < n; i += 64) {
        sx += p[i].x;
        sy += p[i].y;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) {
        const double inv = 1.0 / (double)fd.nsites;
        const double ex = sx * inv, ey = sy * inv;
        E[(int64_t)fd.q * (K + 1) + k + 1] = make_double2(ex, ey);
        // sticky report for the host (btl_synchronize and later calls)
        if (nonfinite != nullptr && !(isfinite(ex) && isfinite(ey))) *nonfinite = 1;
    }
}

// Two entry points around the same body: FP32 storage without membrane
// positions fits in 128 VGPRs when asked to, which raises the occupancy
// from three to four waves per SIMD; the other variants keep the compiler's
// choice (FP64 storage, one site in flight: 92 VGPRs, five waves).
template <typename V, int TX, bool CL, bool GM, int NQ, bool CV, bool FIRST>
__global__ void __launch_bounds__(kBlock) k_step(StepArgs a) {
    step_body<V, TX, CL, GM, NQ, CV, FIRST>(a);
}
template <typename V, int TX, bool CL, bool GM, int NQ, bool CV, bool FIRST>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_step_w4(StepArgs a) {
    step_body<V, TX, CL, GM, NQ, CV, FIRST>(a);
}
// curved links in FP32 storage: held to three waves per SIMD
template <typename V, int TX, bool CL, bool GM, int NQ, bool CV, bool FIRST>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_step_w3(StepArgs a) {
    step_body<V, TX, CL, GM, NQ, CV, FIRST>(a);
}

// ghat^0 of the classical scheme: the collision of the equilibrium state
// g_i = w_i (M = 1) with its reaction term, ghat_i = w_i (1 + dt R(x, t^0)),
// dt R = -dt/T2 - i f_0 dt (c.j + cu).
template <typename V>
__global__ void __launch_bounds__(kBlock) k_init_classical(V* pop, FieldDesc fd,
                                                            const uint32_t* words,
                                                            const double* fdt,
                                                            const double* rdt, int32_t nq) {
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= fd.nsites) return;
    const int32_t n0 = fd.n[0], n1 = fd.n[1];
    const int32_t j0 = s % n0, r = s / n0, j1 = r % n1, j2 = r / n1;
    const int p = (int)(words[fd.words + s] & 0xfu);
    const double ra = 1.0 - rdt[p];
    const double rb = -fdt[0] * (fd.c[0] * j0 + fd.c[1] * j1 + fd.c[2] * j2 + fd.cu);
    const int64_t st2 = (int64_t)n0 * n1;
    const int64_t sp = j0 + (int64_t)n0 * j1 + (int64_t)nq * st2 * j2;
    for (int d = 0; d < nq; ++d) {
        const double wd = d == 0 ? lattice_w0(nq) : lattice_w1(nq);
        store2(pop + fd.pop + d * st2 + sp, make_double2(wd * ra, wd * rb));
    }
}

template <typename V>
__global__ void __launch_bounds__(kBlock) k_mfinal(const V* pop, int64_t nsites, int64_t st2,
                                                    V* out, int32_t nq) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= nsites) return;
    const int64_t sp = s % st2 + (s / st2) * nq * st2;
    double2 m = make_double2(0.0, 0.0);
    for (int d = 0; d < nq; ++d) {
        const double2 v = ld2(pop + d * st2 + sp);
        m.x += v.x;
        m.y += v.y;
    }
    store2(out + s, m);
}

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// E_0 = 1 of the q-sample of every primary field (one thread per field).
__global__ void __launch_bounds__(kBlock) k_e0(const FieldDesc* __restrict__ fields,
                                               int32_t n_fields, double2* E, int32_t K) {
    const int32_t f = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (f < n_fields && fields[f].q >= 0)
        E[(int64_t)fields[f].q * (K + 1)] = make_double2(1.0, 0.0);
}

hipError_t launch_init(int prec, void* pop, int64_t, const FieldDesc* d_fields, int32_t n_fields,
                       const FieldDesc* h, double* E, int32_t, int32_t K, int32_t nq,
                       hipStream_t st, bool pops) {
    if (!pops) {
        if (E != nullptr && n_fields > 0)
            hipLaunchKernelGGL(k_e0, dim3(grid_for(n_fields)), dim3(kBlock), 0, st, d_fields,
                               n_fields, reinterpret_cast<double2*>(E), K);
        return hipGetLastError();
    }
    for (int f = 0; f < n_fields; ++f) {
        const int64_t ns = h[f].nsites, st2 = (int64_t)h[f].n[0] * h[f].n[1];
        const dim3 grid(grid_for(ns * nq));
        if (prec == 1)
            hipLaunchKernelGGL(k_init<float2>, grid, dim3(kBlock), 0, st,
                               static_cast<float2*>(pop) + h[f].pop, ns, st2,
                               reinterpret_cast<double2*>(E), h[f].q, K, nq);
        else
            hipLaunchKernelGGL(k_init<double2>, grid, dim3(kBlock), 0, st,
                               static_cast<double2*>(pop) + h[f].pop, ns, st2,
                               reinterpret_cast<double2*>(E), h[f].q, K, nq);
    }
    return hipGetLastError();
}

template <typename V, bool CL, bool GM, int NQ, bool CV, int TX, bool FIRST>
static void launch_txf(const StepArgs& a, int32_t n_blocks, hipStream_t st) {
    if constexpr (std::is_same<V, float2>::value && !GM)
        hipLaunchKernelGGL((k_step_w4<V, TX, CL, GM, NQ, CV, FIRST>), dim3(n_blocks), dim3(kBlock),
                           0, st, a);
    else if constexpr (std::is_same<V, float2>::value && CV)
        hipLaunchKernelGGL((k_step_w3<V, TX, CL, GM, NQ, CV, FIRST>), dim3(n_blocks), dim3(kBlock),
                           0, st, a);
    else
        hipLaunchKernelGGL((k_step<V, TX, CL, GM, NQ, CV, FIRST>), dim3(n_blocks), dim3(kBlock), 0,
                           st, a);
}

template <typename V, bool CL, bool GM, int NQ, bool CV, int TX>
static void launch_tx(const StepArgs& a, int32_t n_blocks, hipStream_t st) {
    if constexpr (!CL && !CV) {
        if (a.first) {
            launch_txf<V, CL, GM, NQ, CV, TX, true>(a, n_blocks, st);
            return;
        }
    }
    launch_txf<V, CL, GM, NQ, CV, TX, false>(a, n_blocks, st);
}

template <typename V, bool CL, bool GM, int NQ, bool CV>
static void launch_step_t(int shape, const StepArgs& a, int32_t n_blocks, hipStream_t st) {
    switch (shape) {
        case kTile64x4: launch_tx<V, CL, GM, NQ, CV, 64>(a, n_blocks, st); break;
        case kTile32x8: launch_tx<V, CL, GM, NQ, CV, 32>(a, n_blocks, st); break;
        case kTile128x2: launch_tx<V, CL, GM, NQ, CV, 128>(a, n_blocks, st); break;
        case kTile256x1:
            if constexpr (NQ == 5) launch_tx<V, CL, GM, NQ, CV, 256>(a, n_blocks, st);
            break;
        case kTileRows:
            if constexpr (NQ == 7) launch_tx<V, CL, GM, NQ, CV, 0>(a, n_blocks, st);
            break;
        default: launch_tx<V, CL, GM, NQ, CV, 16>(a, n_blocks, st); break;
    }
}

template <typename V, int NQ>
static void launch_step_q(int shape, const StepArgs& a, int32_t n_blocks, hipStream_t st) {
    const bool gm = a.gm != nullptr;
    const bool cv = gm && a.cvm != nullptr;
    if (a.classical) {
        if (cv) launch_step_t<V, true, true, NQ, true>(shape, a, n_blocks, st);
        else if (gm) launch_step_t<V, true, true, NQ, false>(shape, a, n_blocks, st);
        else launch_step_t<V, true, false, NQ, false>(shape, a, n_blocks, st);
    } else {
        if (cv) launch_step_t<V, false, true, NQ, true>(shape, a, n_blocks, st);
        else if (gm) launch_step_t<V, false, true, NQ, false>(shape, a, n_blocks, st);
        else launch_step_t<V, false, false, NQ, false>(shape, a, n_blocks, st);
    }
}

template <typename V>
static void launch_step_v(int shape, const StepArgs& a, int32_t n_blocks, hipStream_t st) {
    if (a.nq == 5)
        launch_step_q<V, 5>(shape, a, n_blocks, st);
    else
        launch_step_q<V, 7>(shape, a, n_blocks, st);
}

hipError_t launch_step(int prec, int shape, const StepArgs& a, int32_t n_blocks, hipStream_t st) {
    if (prec == 1)
        launch_step_v<float2>(shape, a, n_blocks, st);
    else
        launch_step_v<double2>(shape, a, n_blocks, st);
    return hipGetLastError();
}

hipError_t launch_links(int prec, const StepArgs& a, int32_t max_links, int32_t n_fields,
                        hipStream_t st) {
    if (max_links <= 0 || n_fields <= 0) return hipSuccess;
    const int64_t blocks = (int64_t)((max_links + kBlock - 1) / kBlock) *
                           ((n_fields + kLinkFields - 1) / kLinkFields);
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    if (prec == 1)
        hipLaunchKernelGGL(k_links<float2>, dim3((unsigned)blocks), dim3(kBlock), 0, st, a,
                           n_fields);
    else
        hipLaunchKernelGGL(k_links<double2>, dim3((unsigned)blocks), dim3(kBlock), 0, st, a,
                           n_fields);
    return hipGetLastError();
}

hipError_t launch_init_classical(int prec, void* pop, const FieldDesc* h, int32_t n_fields,
                                 const uint32_t* words, const double* fdt, const double* rdt,
                                 int32_t nq, hipStream_t st) {
    for (int f = 0; f < n_fields; ++f) {
        if (prec == 1)
            hipLaunchKernelGGL(k_init_classical<float2>, dim3(grid_for(h[f].nsites)),
                               dim3(kBlock), 0, st, static_cast<float2*>(pop), h[f], words, fdt,
                               rdt, nq);
        else
            hipLaunchKernelGGL(k_init_classical<double2>, dim3(grid_for(h[f].nsites)),
                               dim3(kBlock), 0, st, static_cast<double2*>(pop), h[f], words, fdt,
                               rdt, nq);
    }
    return hipGetLastError();
}

hipError_t launch_esum(const double2* partial, const FieldDesc* d_fields, int32_t n_fields,
                       int32_t nblk_total, int32_t k0, int32_t nsteps, double* E, int32_t K,
                       int32_t* nonfinite, hipStream_t st) {
    const int64_t waves = (int64_t)n_fields * nsteps;
    if (waves > 0)
        hipLaunchKernelGGL(k_esum, dim3((unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64))),
                           dim3(kBlock), 0, st, partial, d_fields, n_fields, nblk_total, k0,
                           nsteps, reinterpret_cast<double2*>(E), K, nonfinite);
    return hipGetLastError();
}

hipError_t launch_tables(const StepArgs& a, int32_t nsteps, hipStream_t st) {
    const int64_t n = (int64_t)nsteps * a.T;
    if (n > 0) hipLaunchKernelGGL(k_tables, dim3(grid_for(n)), dim3(kBlock), 0, st, a, nsteps);
    return hipGetLastError();
}

hipError_t launch_mfinal(int prec, const void* pop, const FieldDesc* h, int32_t n_fields,
                         void* M_out, int32_t nq, hipStream_t st) {
    int64_t off = 0;
    for (int f = 0; f < n_fields; ++f) {
        if (h[f].q < 0) continue;
        const int64_t ns = h[f].nsites, st2 = (int64_t)h[f].n[0] * h[f].n[1];
        if (prec == 1)
            hipLaunchKernelGGL(k_mfinal<float2>, dim3(grid_for(ns)), dim3(kBlock), 0, st,
                               static_cast<const float2*>(pop) + h[f].pop, ns, st2,
                               static_cast<float2*>(M_out) + off, nq);
        else
            hipLaunchKernelGGL(k_mfinal<double2>, dim3(grid_for(ns)), dim3(kBlock), 0, st,
                               static_cast<const double2*>(pop) + h[f].pop, ns, st2,
                               static_cast<double2*>(M_out) + off, nq);
        off += ns;
    }
    return hipGetLastError();
}

}  // namespace btl
