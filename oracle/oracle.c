/*
 * FP64 CPU oracle for the hybrid lattice Boltzmann Bloch-Torrey scheme
 * (Naughton, Tennyson, Georgiadis, arXiv:1907.00908).
 *
 * TEST INFRASTRUCTURE.  This file is the slow, plain reference that the HIP
 * path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may call it.  It shares no code with the
 * HIP library.
 *
 * It follows the paper's own formulation: per time step t^k
 *   1. zeroth moment M = sum_i g_i                      (Eq. M'summation)
 *      signal E_k = mean of M over the domain             (Sec. 2.1)
 *   2. BGK collision  ghat_i = g_i - (g_i - w_i M)/tau     (Eqs. collision_LBM,
 *      g_eq, tau_def)
 *   3. buffer rows at n = -1 and n = N filled from the post-collision values
 *      (modified periodic BC, Eq. collision_BC; mirroring BC, Sec. 2.4.4)
 *   4. streaming gbar_i(x + e_i) = ghat_i(x)             (Eq. streaming_LBM)
 *      with the half-link membrane condition on links that join two
 *      different compartments, in place of streaming  (Eqs. B5, P_def,
 *      permeability_BC)
 *   5. reaction g_i = g'_i exp(-i gamma (x.G0) f(t^k) dt) exp(-dt/T2)
 *                                                  (Eqs. reaction_LBM, delta_phi)
 * and after the last step the signal E_K and the magnetization M.
 *
 * With scheme = 1 the routine runs the classical LBM instead (Appendix A,
 * Eq. A12): no reaction split; the collision carries the reaction term,
 *   ghat_i = g_i - (g_i - w_i M)/tau + dt w_i R M,
 *   R(x, t^k) = -i gamma (x.G0) f(t^k) - 1/T2,
 * and the boundary and membrane rules are unchanged.
 *
 * With link positions given (link_delta != NULL) a membrane link uses the
 * theta = 0 form of the general membrane condition for a membrane at any
 * distance Delta_m along the link (Eqs. B2a_text/B2b_text with the
 * coefficients of Eqs. B4a-B4c and the Dirichlet/Neumann coefficients of
 * Eqs. c_n, c_d): for the population g'_i arriving at x across the link from
 * x - e_i, with ibar the opposite direction and Delta the distance from x to
 * the membrane,
 *   g'_i(x) = A_1 ghat_ibar(x) + A_2 ghat_ibar(x + e_i) + A_3 ghat_i(x)
 *           + B_1 ghat_i(x - e_i) + B_2 ghat_i(x - 2e_i) + B_3 ghat_ibar(x - e_i).
 * The two second nodes must belong to the compartments of their sides and,
 * with x - e_i, lie in the same tile of the lattice as x (no outer face in
 * the stencil); otherwise the link falls back to the half-link rule.
 *
 * With membrane normals given as well (link_normal != NULL) a membrane link
 * takes the general condition for a membrane at any angle (Sec. 2.4.2 and
 * Appendix B, theta != 0): on each side the Dirichlet and Neumann link
 * relations (Eqs. dirichlet_1/2, neumann_1/2 with the coefficients of Eqs.
 * c_d, c_n at the side's distance) give the value at the membrane and the
 * inflow flux along the link; the flux along each lattice direction
 * orthogonal to the link comes from the same two relations with the
 * coefficients for Delta_m = 0 on the lattice line through the membrane
 * point (Eqs. phi_1, phi_2: populations at the membrane point x' and at
 * x' + e_betabar); the normal inflow is their combination with the
 * direction cosines of the normal (two terms in 2D as printed, three in 3D),
 * and the permeability condition with flux continuity (Eqs. B1, B1.5)
 * closes the two sides' values.  The populations at the off-lattice points
 * are interpolated (quadratically) along the link direction from the three
 * nodes of the side's own compartment nearest to each point (a reading: the
 * paper does not say how they are obtained).
 * Stencils may reach through periodic faces (with the modified periodic
 * phase factor), not through mirroring faces or stencil tiles.  Where a
 * stencil node is missing the link takes the theta = 0 rule.
 *
 * With substeps = m > 1 the reaction of each step is taken as m sub-steps
 * of length dt' = dt/m (the reaction time step of Sec. 2.3, dt = m dt'),
 * each with its own waveform sample: f holds K*m samples, sub-step j of step
 * k multiplies by exp(-i gamma (x.G0) f[k m + j] dt') exp(-dt'/T2), and F
 * advances by f[k m + j] dt' per sub-step.  (Hybrid scheme only.)
 *
 * lattice = 1 runs the two-dimensional D2Q5 lattice of Sec. 2.2 instead
 * (Eq. omega_i: eps_D = 1/3, w_0 = 1/3, w_{1..4} = 1/6) on a single layer
 * (n2 = 1, no gradient along z); every rule above is unchanged.
 *
 * Lattice: D3Q7 with eps_D = 1/4, w_0 = 1/4, w_{+-x,+-y,+-z} = 1/8.  The
 * paper leaves the 3D weights implicit; eps_D = 1/4 is what its Fig. 11
 * caption requires (tau = 0.58 at D = 2, dt = 0.01, dx = 1), and the weights
 * extend the D2Q5 pattern w_0 = eps_D, w_i = eps_D/2 (Eq. omega_i) to 3D.
 *
 * Readings of the paper taken here:
 *  - Half-link condition: the second line of Eq. permeability_BC has its
 *    subscripts exchanged in print; the general form (Eq. B2b with the
 *    coefficients of Eq. B5) gives
 *        g'_alpha(x_e) = P/(1+P) ghat_alphabar(x_e) + 1/(1+P) ghat_alpha(x_i),
 *    i.e. the share 1/(1+P) of the population heading at the membrane
 *    crosses it and P/(1+P) is reflected back, on both sides.
 *  - A membrane sits on every link joining two different compartments; its
 *    permeability is looked up by the two phases (kappa = +inf: no membrane).
 *  - Modified periodic BC in 3D with an oblique gradient: one phase
 *    phi_a = L_a (gamma G0)_a F_k per axis, F_k = sum_{m<k} f_m dt
 *    (Eqs. modified_periodic_BC, periodic_phi, collision_BC).
 *  - Mirroring BC for a gradient normal to the face: the printed combined
 *    equation loses a complex conjugate on one line; composing Eqs.
 *    mirror_periodic_BC and mirror_periodic_BC2 gives
 *        ghat_i(x_m) = conj( ghat_ibar(x_n) exp(i theta) ),
 *        theta = gamma (x_n + x_m - 2 x_o).G0 F_k,  origin x_o = 0,
 *    and for a gradient parallel to the face ghat_i(x_m) = ghat_ibar(x_n).
 *    The buffer node lies one spacing beyond the face and has the geometry
 *    of the boundary node.  An oblique gradient on a mirrored axis is not
 *    defined by the paper; this routine rejects it (the Python wrapper runs
 *    such cases on the literally reflected and doubled domain instead).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 7
typedef double complex cplx;

static const int EX[QMAX][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                                {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const int OPP[QMAX] = {0, 2, 1, 4, 3, 6, 5};
/* D3Q7: eps_D = 1/4, w_0 = 1/4, w_i = 1/8 (reading above) */
static const double W7[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
/* D2Q5 (Eq. omega_i): eps_D = 1/3, w_0 = 1/3, w_{1..4} = 1/6; directions
   +-x, +-y are the first five of the table above */
static const double W5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};

enum { BC_PERIODIC = 0, BC_MIRROR = 1 };

/* direction i reflected in the plane normal to axis a */
static int reflect_dir(int i, int a) {
    if (i == 0) return 0;
    int ax = (i - 1) / 2;
    return ax == a ? OPP[i] : i;
}

/*
 * Coefficients A_1..A_3, B_1..B_3 of the general membrane condition for a
 * straight membrane normal to the link (theta = 0, Eqs. B4a, B4c) at
 * distance d (units of dx) from the receiving node; the other side's node is
 * at 1 - d.  Own-side Dirichlet/Neumann coefficients c_dj, c_nj (Eqs. c_d,
 * c_n) use d, the other side's (starred) use 1 - d.  kdt = kappa dt,
 * edx = eps_D dx.
 */
static void memb_coeffs(double d, double kdt, double edx, double A[3], double B[3]) {
    double cn[4], cd[4], cns[4], cds[4];
    for (int side = 0; side < 2; ++side) {
        const double D = side == 0 ? d : 1.0 - d;
        double *n_ = side == 0 ? cn : cns, *d_ = side == 0 ? cd : cds;
        const double h = 2.0 * D - 1.0, q = 2.0 * D + 1.0;
        n_[0] = 1.0;
        n_[1] = -h / q;
        n_[2] = h / q;
        n_[3] = 2.0 / q;
        d_[0] = 2.0 * (D - 1.0);
        d_[1] = -h * h / q;
        d_[2] = 2.0 * h / q;
        d_[3] = (3.0 - 2.0 * D) / q;
    }
    const double F = cd[3] * cds[3] * edx + (cd[3] * cns[3] + cn[3] * cds[3]) * kdt;
    for (int j = 0; j < 3; ++j) {
        A[j] = (cd[3] * cds[3] * cn[j] * edx + (cds[3] * cn[3] * cd[j] + cns[3] * cd[3] * cn[j]) * kdt) / F;
        B[j] = cd[3] * cn[3] * (cns[j] - cds[j]) * kdt / F;
    }
}

/* the coefficients above, for tests: out = {A_1, A_2, A_3, B_1, B_2, B_3} */
void oracle_memb_coeffs(double d, double kappa_dt, double epsd_dx, double *out) {
    memb_coeffs(d, kappa_dt, epsd_dx, out, out + 3);
}

/* pairwise sum of n complex values: rounding error O(log n) */
static cplx pairwise_sum(const cplx *v, long n) {
    if (n <= 8) {
        cplx s = 0;
        for (long i = 0; i < n; ++i) s += v[i];
        return s;
    }
    long h = n / 2;
    return pairwise_sum(v, h) + pairwise_sum(v + h, n - h);
}

/* Dirichlet and Neumann coefficients c_d1..c_d4, c_n1..c_n4 (Eqs. c_d, c_n)
   for a node at distance d from the membrane */
static void cdn(double d, double cd[4], double cn[4]) {
    const double q = 2.0 * d + 1.0, r = 2.0 * d - 1.0;
    cd[0] = 2.0 * (d - 1.0);
    cd[1] = -r * r / q;
    cd[2] = 2.0 * r / q;
    cd[3] = (3.0 - 2.0 * d) / q;
    cn[0] = 1.0;
    cn[1] = -r / q;
    cn[2] = r / q;
    cn[3] = 2.0 / q;
}

/* Geometry and state one side of a curved membrane link sees.  The side's
   node xs receives populations along e_s (direction ds) from the membrane
   at distance dist; ok(j) says whether node j belongs to the side's
   compartment and lies in its stencil tile. */
typedef struct {
    const cplx *gh;
    long PN, p0, p1;
    const uint32_t *comp;
    long n[3], tl[3], t0[3];   /* sizes, tile sizes, the side's tile origin */
    int wrap[3];               /* axis periodic over its whole length */
    double phi[3];             /* modified periodic phase L_a (gamma G0)_a F_k */
    uint32_t c;
    int lattice;
} side_ctx;

/* node j of the side (periodic axes wrap, with w the number of wraps) */
static int side_node(const side_ctx *sc, const long j[3], long jw[3], long w[3]) {
    for (int a = 0; a < 3; ++a) {
        jw[a] = j[a];
        w[a] = 0;
        if (sc->wrap[a]) {
            while (jw[a] < 0) { jw[a] += sc->n[a]; --w[a]; }
            while (jw[a] >= sc->n[a]) { jw[a] -= sc->n[a]; ++w[a]; }
        } else if (j[a] < sc->t0[a] || j[a] >= sc->t0[a] + sc->tl[a]) {
            return 0;
        }
    }
    return sc->comp[jw[0] + sc->n[0] * (jw[1] + sc->n[1] * jw[2])] == sc->c;
}

static int side_node_ok(const side_ctx *sc, const long j[3]) {
    long jw[3], w[3];
    return side_node(sc, j, jw, w);
}

/* post-collision population dir at node j; across a periodic face the
   modified periodic condition (Eq. collision_BC): the image of node j - N
   carries the factor exp(+i phi), of j + N exp(-i phi) */
static cplx side_val(const side_ctx *sc, int dir, const long j[3]) {
    long jw[3], w[3];
    side_node(sc, j, jw, w);
    cplx v = sc->gh[dir * sc->PN + ((jw[0] + 1) + sc->p0 * ((jw[1] + 1) + sc->p1 * (jw[2] + 1)))];
    for (int a = 0; a < 3; ++a)
        if (w[a] != 0) v *= cexp(-I * (double)w[a] * sc->phi[a]);
    return v;
}

/* population dir at the point base + t e, by quadratic (Lagrange)
   interpolation through the three nodes base + u e, u = -3 .. 3, of the
   side that lie nearest to the point (ties: the smaller u) */
static int side_interp(const side_ctx *sc, int dir, const long base[3], const int e[3],
                       double t, cplx *out) {
    int use[3], nu = 0;
    int taken[7] = {0};
    while (nu < 3) {
        int best = -100;
        for (int u = -3; u <= 3; ++u) {
            if (taken[u + 3]) continue;
            if (best == -100 || fabs(u - t) < fabs(best - t)) best = u;
        }
        if (best == -100) return 0;
        taken[best + 3] = 1;
        long j[3];
        for (int a = 0; a < 3; ++a) j[a] = base[a] + best * e[a];
        if (side_node_ok(sc, j)) use[nu++] = best;
    }
    cplx v = 0;
    for (int m = 0; m < 3; ++m) {
        double lw = 1.0;
        for (int l = 0; l < 3; ++l)
            if (l != m) lw *= (t - use[l]) / (double)(use[m] - use[l]);
        long j[3];
        for (int a = 0; a < 3; ++a) j[a] = base[a] + use[m] * e[a];
        v += lw * side_val(sc, dir, j);
    }
    *out = v;
    return 1;
}

/* One side: the inflow flux normal to the membrane as L + A m (m the side's
   value at the membrane), and D, the Dirichlet part of the arriving
   population (g' = D + c_d4 eps m).  nrm is the unit normal into the side.
   Returns 0 when a stencil node is missing. */
static int curved_side(const side_ctx *sc, const long xs[3], int ds, double dist,
                       const double nrm[3], double eps, double h, cplx *L, double *A,
                       cplx *Dp, double *cd4) {
    const int es[3] = {EX[ds][0], EX[ds][1], EX[ds][2]};
    const int dout = OPP[ds];
    long x2[3];
    for (int a = 0; a < 3; ++a) x2[a] = xs[a] + es[a];
    if (!side_node_ok(sc, xs) || !side_node_ok(sc, x2)) return 0;
    double cd[4], cn[4];
    cdn(dist, cd, cn);
    /* link relations (Eqs. dirichlet_1, neumann_1 of this side) */
    const cplx st[3] = {side_val(sc, dout, xs), side_val(sc, dout, x2), side_val(sc, ds, xs)};
    cplx Dl = 0, Nl = 0;
    for (int j = 0; j < 3; ++j) {
        Dl += cd[j] * st[j];
        Nl += cn[j] * st[j];
    }
    /* inflow flux along e_s: (D - N + c_d4 eps m) / (c_n4 h) */
    const int ax = (ds - 1) / 2;
    const double cth = fabs(nrm[ax]);
    *L = cth * (Dl - Nl) / (cn[3] * h);
    *A = cth * cd[3] * eps / (cn[3] * h);
    /* each orthogonal lattice direction with a normal component: the same
       relations at Delta_m = 0 on the line through the membrane point */
    double c0d[4], c0n[4];
    cdn(0.0, c0d, c0n);
    for (int b = 0; b < 3; ++b) {
        if (b == ax || (sc->lattice == 1 && b == 2)) continue;
        const double sb = fabs(nrm[b]);
        if (sb == 0.0) continue;
        const int sgn = nrm[b] > 0 ? 1 : -1;
        const int dbb = 1 + 2 * b + (sgn > 0 ? 0 : 1);   /* e_betabar: into the side */
        const int db = OPP[dbb];
        long base2[3];
        for (int a = 0; a < 3; ++a) base2[a] = xs[a] + (a == b ? sgn : 0);
        cplx b_p1, b_p2, bb_p1;
        if (!side_interp(sc, db, xs, es, -dist, &b_p1) ||
            !side_interp(sc, db, base2, es, -dist, &b_p2) ||
            !side_interp(sc, dbb, xs, es, -dist, &bb_p1))
            return 0;
        const cplx DN = (c0d[0] - c0n[0]) * b_p1 + (c0d[1] - c0n[1]) * b_p2 +
                        (c0d[2] - c0n[2]) * bb_p1;
        *L += sb * DN / (c0n[3] * h);
        *A += sb * c0d[3] * eps / (c0n[3] * h);
    }
    *Dp = Dl;
    *cd4 = cd[3];
    return 1;
}

/*
 * Run K steps of the scheme for one gradient direction.
 *
 * n[3]        sites per axis (x fastest), comp[n2][n1][n0] compartment ids
 * comp_phase  [n_comp] phase of each compartment
 * bc[3]       0 periodic (modified), 1 mirroring
 * off[3]      coordinate of node j is (j + off_a) * dx  (origin x_o = 0)
 * D, T2       [n_phase]; T2 may be +inf
 * kappa       [n_phase * n_phase] symmetric, um/ms; +inf = no membrane
 * f           [K * substeps] waveform samples, gG0[3] = gamma * G0 in
 *             rad/(um ms)
 * elo, ehi    the box [elo, ehi) over which the signal is averaged
 * link_delta  [3][n2][n1][n0] or NULL: for axis a, the distance (units of
 *             dx) from node j to the membrane on the link j -> j + e_a,
 *             0 < value < 1; read only on links joining two compartments
 * tile[3]     stencil tiles of the general membrane rule (NULL: whole axes)
 * link_normal [3][3][n2][n1][n0] or NULL (needs link_delta): for axis a,
 *             components c = 0..2 of a unit normal of the membrane on the
 *             link j -> j + e_a (either orientation)
 * E           out [K+1] complex (interleaved re, im)
 * M_out       out [n2][n1][n0] complex or NULL
 * returns 0, or -1 for invalid input, -2 for an unsupported case, -3 OOM
 */
int oracle_run(const int32_t n[3], const uint32_t *comp, const uint8_t *comp_phase,
               int32_t n_comp, int32_t n_phase, const int32_t bc[3],
               const double off[3], double dx, double dt, int32_t K,
               const double *D, const double *T2, const double *kappa,
               const double *f, const double gG0[3], const int32_t elo[3],
               const int32_t ehi[3], double *E, double *M_out, int32_t nthreads,
               int32_t scheme, const double *link_delta, const int32_t *tile,
               int32_t substeps, int32_t lattice, const double *link_normal) {
    const long n0 = n[0], n1 = n[1], n2 = n[2];
    if (n0 < 1 || n1 < 1 || n2 < 1 || dx <= 0 || dt <= 0 || K < 0) return -1;
    if (scheme != 0 && scheme != 1) return -1;
    if (substeps < 1 || (scheme == 1 && substeps != 1)) return -1;
    if (lattice != 0 && lattice != 1) return -1;
    if (link_normal && !link_delta) return -1;
    /* D2Q5 runs a single layer: n2 = 1, no gradient along z */
    if (lattice == 1 && (n[2] != 1 || gG0[2] != 0.0)) return -1;
    const int Q = lattice == 1 ? 5 : 7;
    const double *W = lattice == 1 ? W5 : W7;
    const double EPS_D = lattice == 1 ? 1.0 / 3.0 : 0.25;
    const int m_sub = substeps;
    const double dts = dt / m_sub;
    const long N = n0 * n1 * n2;
    for (int a = 0; a < 3; ++a) {
        if (bc[a] != BC_PERIODIC && bc[a] != BC_MIRROR) return -1;
        if (elo[a] < 0 || ehi[a] > n[a] || elo[a] >= ehi[a]) return -1;
        if (bc[a] == BC_MIRROR && gG0[a] != 0.0) {
            for (int b = 0; b < 3; ++b)
                if (b != a && gG0[b] != 0.0) return -2; /* oblique: not defined */
        }
    }
    for (long s = 0; s < N; ++s)
        if (comp[s] >= (uint32_t)n_comp) return -1;
    for (int c = 0; c < n_comp; ++c)
        if (comp_phase[c] >= n_phase) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

    for (int p = 0; p < n_phase; ++p)
        if (!(D[p] > 0) || !(T2[p] > 0)) return -1;
    for (int p = 0; p < n_phase * n_phase; ++p)
        if (!(kappa[p] >= 0)) return -1;
    long tl[3];
    for (int a = 0; a < 3; ++a) {
        tl[a] = tile ? tile[a] : n[a];
        if (tl[a] < 1 || n[a] % tl[a] != 0) return -1;
    }
    if (link_delta) /* every value the rule can read: links joining two compartments */
        for (int a = 0; a < 3; ++a)
            for (long s = 0; s < N; ++s) {
                long j[3] = {s % n0, (s / n0) % n1, s / (n0 * n1)};
                if (++j[a] == n[a]) {
                    if (bc[a] == BC_MIRROR) continue;  /* not a lattice link */
                    j[a] = 0;
                }
                if (comp[s] != comp[j[0] + n0 * (j[1] + n1 * j[2])] &&
                    !(link_delta[a * N + s] > 0.0 && link_delta[a * N + s] < 1.0))
                    return -1;
            }

    /* per-phase constants: tau (Eq. tau_def), T2 decay (Eq. reaction_LBM) */
    double *tau = malloc(sizeof(double) * n_phase);
    double *decay = malloc(sizeof(double) * n_phase);
    /* per phase-pair membrane split: reflected P/(1+P), transmitted 1/(1+P)
       with P = eps_D dx / (2 kappa dt) (Eqs. B5, P_def) */
    double *refl = malloc(sizeof(double) * n_phase * n_phase);
    double *trans = malloc(sizeof(double) * n_phase * n_phase);
    int *has_mem = malloc(sizeof(int) * n_phase * n_phase);
    for (int p = 0; p < n_phase; ++p) {
        tau[p] = 0.5 + dt * D[p] / (EPS_D * dx * dx);
        decay[p] = isinf(T2[p]) ? 1.0 : exp(-dt / T2[p]);
    }
    for (int p = 0; p < n_phase * n_phase; ++p) {
        double k = kappa[p];
        if (isinf(k)) { has_mem[p] = 0; refl[p] = 0; trans[p] = 1; continue; }
        has_mem[p] = 1;
        if (k == 0.0) { refl[p] = 1.0; trans[p] = 0.0; continue; }
        double P = EPS_D * dx / (2.0 * k * dt);
        refl[p] = P / (1.0 + P);
        trans[p] = 1.0 / (1.0 + P);
    }

    const long p0 = n0 + 2, p1 = n1 + 2, p2 = n2 + 2;
    const long PN = p0 * p1 * p2;
    cplx *g = malloc(sizeof(cplx) * Q * N);      /* g_i(x, t^k) */
    cplx *gh = malloc(sizeof(cplx) * Q * PN);    /* ghat_i with buffer rows */
    cplx *M = malloc(sizeof(cplx) * N);
    if (!g || !gh || !M || !tau || !decay || !refl || !trans || !has_mem) return -3;
    memset(gh, 0, sizeof(cplx) * Q * PN);
#define IDX(j0, j1, j2) ((j0) + n0 * ((j1) + n1 * (long)(j2)))
#define PIDX(j0, j1, j2) (((j0) + 1) + p0 * (((j1) + 1) + p1 * (long)((j2) + 1)))

    /* initial condition M = 1 + 0i (Sec. 2.1) as equilibrium populations */
    for (int i = 0; i < Q; ++i)
        for (long s = 0; s < N; ++s) g[i * N + s] = W[i];

    /* coordinate of node j on axis a */
#define COORD(a, j) (((double)(j) + off[a]) * dx)
    const long ecount = (long)(ehi[0] - elo[0]) * (ehi[1] - elo[1]) * (ehi[2] - elo[2]);
    cplx *Ebuf = malloc(sizeof(cplx) * ecount);
    double F = 0.0; /* F_k = sum_{m<k} f_m dt  (Eq. periodic_phi) */

    for (int k = 0; k <= K; ++k) {
        /* 1. zeroth moment and signal */
#pragma omp parallel for schedule(static)
        for (long s = 0; s < N; ++s) {
            cplx m = 0;
            for (int i = 0; i < Q; ++i) m += g[i * N + s];
            M[s] = m;
        }
        {
            long t = 0;
            for (long j2 = elo[2]; j2 < ehi[2]; ++j2)
                for (long j1 = elo[1]; j1 < ehi[1]; ++j1)
                    for (long j0 = elo[0]; j0 < ehi[0]; ++j0) Ebuf[t++] = M[IDX(j0, j1, j2)];
            cplx e = pairwise_sum(Ebuf, ecount) / (double)ecount;
            E[2 * k] = creal(e);
            E[2 * k + 1] = cimag(e);
        }
        if (k == K) break;

        /* 2. collision into the interior of the padded array */
#pragma omp parallel for schedule(static)
        for (long j2 = 0; j2 < n2; ++j2)
            for (long j1 = 0; j1 < n1; ++j1)
                for (long j0 = 0; j0 < n0; ++j0) {
                    long s = IDX(j0, j1, j2);
                    int p = comp_phase[comp[s]];
                    cplx RM = 0;
                    if (scheme == 1) {
                        /* reaction term of the classical collision (Eq. A12) */
                        const double xg = gG0[0] * COORD(0, j0) + gG0[1] * COORD(1, j1)
                                        + gG0[2] * COORD(2, j2);
                        const double rdec = isinf(T2[p]) ? 0.0 : 1.0 / T2[p];
                        RM = (-I * xg * f[k] - rdec) * M[s];
                    }
                    for (int i = 0; i < Q; ++i) {
                        cplx gi = g[i * N + s];
                        gh[i * PN + PIDX(j0, j1, j2)] = gi - (gi - W[i] * M[s]) / tau[p]
                                                      + dt * W[i] * RM;
                    }
                }

        /* 3. buffer rows, one axis at a time */
        for (int a = 0; a < 3; ++a) {
            const long na = n[a];
            const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
            const long nb1 = n[b1], nb2 = n[b2];
            const double phi = (double)na * dx * gG0[a] * F;   /* phi(L_a, t^k) */
            const cplx wrap_lo = cexp(I * phi), wrap_hi = cexp(-I * phi);
            const int normal = (gG0[a] != 0.0);  /* gradient normal to face a */
#pragma omp parallel for schedule(static)
            for (long u2 = 0; u2 < nb2; ++u2)
                for (long u1 = 0; u1 < nb1; ++u1) {
                    long jl[3], jh[3], bl[3], bh[3];
                    jl[b1] = jh[b1] = bl[b1] = bh[b1] = u1;
                    jl[b2] = jh[b2] = bl[b2] = bh[b2] = u2;
                    bl[a] = -1;          /* buffer row below node 0 */
                    bh[a] = na;          /* buffer row above node N-1 */
                    for (int i = 0; i < Q; ++i) {
                        cplx vlo, vhi;
                        if (bc[a] == BC_PERIODIC) {
                            /* ghat(x_-1) = e^{+i phi} ghat(x_{N-1});
                               ghat(x_N) = e^{-i phi} ghat(x_0) */
                            jl[a] = na - 1;
                            jh[a] = 0;
                            vlo = wrap_lo * gh[i * PN + PIDX(jl[0], jl[1], jl[2])];
                            vhi = wrap_hi * gh[i * PN + PIDX(jh[0], jh[1], jh[2])];
                        } else {
                            const int ib = reflect_dir(i, a);
                            jl[a] = 0;
                            jh[a] = na - 1;
                            cplx sl = gh[ib * PN + PIDX(jl[0], jl[1], jl[2])];
                            cplx sh = gh[ib * PN + PIDX(jh[0], jh[1], jh[2])];
                            if (normal) {
                                /* conj(ghat_ibar(x_n) e^{i theta}),
                                   theta = gamma (x_n + x_m - 2 x_o).G0 F */
                                double th_lo = gG0[a] * (COORD(a, 0) + COORD(a, -1)) * F;
                                double th_hi = gG0[a] * (COORD(a, na - 1) + COORD(a, na)) * F;
                                vlo = conj(sl * cexp(I * th_lo));
                                vhi = conj(sh * cexp(I * th_hi));
                            } else {
                                vlo = sl;
                                vhi = sh;
                            }
                        }
                        gh[i * PN + PIDX(bl[0], bl[1], bl[2])] = vlo;
                        gh[i * PN + PIDX(bh[0], bh[1], bh[2])] = vhi;
                    }
                }
        }

        /* 4. streaming with membranes, then 5. reaction */

#pragma omp parallel for schedule(static)
        for (long j2 = 0; j2 < n2; ++j2)
            for (long j1 = 0; j1 < n1; ++j1)
                for (long j0 = 0; j0 < n0; ++j0) {
                    const long s = IDX(j0, j1, j2);
                    const long jj[3] = {j0, j1, j2};
                    const uint32_t cx = comp[s];
                    const int px = comp_phase[cx];
                    /* reaction factor: exp(-i gamma (x.G0) f_k dt) exp(-dt/T2) */
                    const double xg = gG0[0] * COORD(0, j0) + gG0[1] * COORD(1, j1)
                                    + gG0[2] * COORD(2, j2);
                    cplx react = 1.0;
                    if (scheme == 0) {
                        /* m reaction sub-steps of length dt/m; their decay
                           factors multiply to exp(-dt/T2) */
                        for (int j = 0; j < m_sub; ++j)
                            react *= cexp(-I * xg * f[(long)k * m_sub + j] * dts);
                        react *= decay[px];
                    }
                    for (int i = 0; i < Q; ++i) {
                        long src[3];
                        int crossed = -1;
                        for (int a = 0; a < 3; ++a) {
                            src[a] = jj[a] - EX[i][a];
                            if (src[a] < 0 || src[a] >= n[a]) crossed = a;
                        }
                        cplx gin = gh[i * PN + PIDX(src[0], src[1], src[2])];
                        /* compartment the streamed population comes from */
                        uint32_t cs;
                        if (crossed < 0) {
                            cs = comp[IDX(src[0], src[1], src[2])];
                        } else if (bc[crossed] == BC_PERIODIC) {
                            long w[3] = {src[0], src[1], src[2]};
                            w[crossed] = (w[crossed] + n[crossed]) % n[crossed];
                            cs = comp[IDX(w[0], w[1], w[2])];
                        } else {
                            cs = cx; /* mirror: buffer node has the boundary node's geometry */
                        }
                        cplx gp;
                        const int pair = px * n_phase + comp_phase[cs];
                        int general = 0;
                        if (link_normal && cs != cx && has_mem[pair] &&
                            (crossed < 0 || (bc[crossed] == BC_PERIODIC && tl[crossed] == n[crossed]))) {
                            const int ax = (i - 1) / 2, sg = EX[i][ax];
                            long sw[3] = {src[0], src[1], src[2]};   /* src, wrapped */
                            if (crossed >= 0) sw[crossed] = (sw[crossed] + n[crossed]) % n[crossed];
                            const long lower = sg > 0 ? IDX(sw[0], sw[1], sw[2]) : s;
                            const double dl = link_delta[ax * N + lower];
                            const double d = sg > 0 ? 1.0 - dl : dl;
                            double nv[3];
                            for (int c = 0; c < 3; ++c) nv[c] = link_normal[(ax * 3 + c) * N + lower];
                            /* the normal into x's side has a positive component along e_i */
                            const double o = nv[ax] * sg > 0 ? 1.0 : -1.0;
                            double nown[3], nfar[3];
                            for (int c = 0; c < 3; ++c) {
                                nown[c] = o * nv[c];
                                nfar[c] = -nown[c];
                            }
                            side_ctx own = {gh, PN, p0, p1, comp, {n0, n1, n2},
                                            {tl[0], tl[1], tl[2]},
                                            {j0 / tl[0] * tl[0], j1 / tl[1] * tl[1], j2 / tl[2] * tl[2]},
                                            {bc[0] == BC_PERIODIC && tl[0] == n0,
                                             bc[1] == BC_PERIODIC && tl[1] == n1,
                                             bc[2] == BC_PERIODIC && tl[2] == n2},
                                            {n0 * dx * gG0[0] * F, n1 * dx * gG0[1] * F,
                                             n2 * dx * gG0[2] * F},
                                            cx, lattice};
                            side_ctx far = own;
                            far.c = cs;
                            const double h = dt / dx;
                            cplx Lo, Lf, Do, Df;
                            double Ao, Af, cdo, cdf;
                            if (nv[ax] != 0.0 &&
                                curved_side(&own, jj, i, d, nown, EPS_D, h, &Lo, &Ao, &Do, &cdo) &&
                                curved_side(&far, src, OPP[i], 1.0 - d, nfar, EPS_D, h, &Lf, &Af,
                                            &Df, &cdf)) {
                                /* inflow into each side kappa (m_other - m_side) (Eqs. B1,
                                   B1.5): L_o + A_o m_o = kappa (m_f - m_o),
                                   L_f + A_f m_f = kappa (m_o - m_f) */
                                const double kap = kappa[pair];
                                cplx mo;
                                if (kap == 0.0) {
                                    mo = -Lo / Ao;
                                } else {
                                    const double det = Ao * Af + kap * (Ao + Af);
                                    mo = (-(Af + kap) * Lo - kap * Lf) / det;
                                }
                                gp = Do + cdo * EPS_D * mo;
                                general = 1;
                            }
                        }
                        if (!general && link_delta && cs != cx && has_mem[pair] && crossed < 0) {
                            /* stencil x - 2e_i .. x + e_i along axis ax, in x's tile */
                            const int ax = (i - 1) / 2, sg = EX[i][ax];
                            const long j = jj[ax], t0 = j / tl[ax] * tl[ax];
                            const long jm2 = j - 2 * sg, jp1 = j + sg;
                            if (jm2 >= t0 && jm2 < t0 + tl[ax] && jp1 >= t0 && jp1 < t0 + tl[ax] &&
                                src[ax] >= t0 && src[ax] < t0 + tl[ax]) {
                                long a2[3] = {j0, j1, j2}, a1[3] = {j0, j1, j2};
                                a2[ax] = jm2;
                                a1[ax] = jp1;
                                const long s2 = IDX(a2[0], a2[1], a2[2]);
                                const long s1 = IDX(a1[0], a1[1], a1[2]);
                                if (comp[s1] == cx && comp[s2] == cs) {
                                    /* distance from x to the membrane: the link
                                       value is measured from its lower node */
                                    const long lower = sg > 0 ? IDX(src[0], src[1], src[2]) : s;
                                    const double dl = link_delta[ax * N + lower];
                                    const double d = sg > 0 ? 1.0 - dl : dl;
                                    double A[3], B[3];
                                    memb_coeffs(d, kappa[pair] * dt, EPS_D * dx, A, B);
                                    const int ib = OPP[i];
                                    gp = A[0] * gh[ib * PN + PIDX(j0, j1, j2)]
                                       + A[1] * gh[ib * PN + PIDX(a1[0], a1[1], a1[2])]
                                       + A[2] * gh[i * PN + PIDX(j0, j1, j2)]
                                       + B[0] * gin
                                       + B[1] * gh[i * PN + PIDX(a2[0], a2[1], a2[2])]
                                       + B[2] * gh[ib * PN + PIDX(src[0], src[1], src[2])];
                                    general = 1;
                                }
                            }
                        }
                        if (general) {
                        } else if (cs != cx && has_mem[pair]) {
                            /* half-link membrane: transmitted share of the
                               incoming population plus reflected share of the
                               outgoing one at this node */
                            gp = trans[pair] * gin + refl[pair] * gh[OPP[i] * PN + PIDX(j0, j1, j2)];
                        } else {
                            gp = gin;
                        }
                        g[i * N + s] = gp * react;
                    }
                }
        for (int j = 0; j < m_sub; ++j) F += f[(long)k * m_sub + j] * dts;
    }
    if (M_out) {
        for (long s = 0; s < N; ++s) {
            M_out[2 * s] = creal(M[s]);
            M_out[2 * s + 1] = cimag(M[s]);
        }
    }
    free(g); free(gh); free(M); free(Ebuf);
    free(tau); free(decay); free(refl); free(trans); free(has_mem);
    return 0;
#undef IDX
#undef PIDX
#undef COORD
}

/* relaxation time of Eq. tau_def: D3Q7 (lattice 0, eps_D = 1/4) or D2Q5
   (lattice 1, eps_D = 1/3) */
double oracle_tau(double D, double dt, double dx, int32_t lattice) {
    const double eps = lattice == 1 ? 1.0 / 3.0 : 0.25;
    return 0.5 + dt * D / (eps * dx * dx);
}
