// Term lists of the general membrane condition for a membrane at an angle to
// the lattice links (Sec. 2.4.2 and Appendix B), built on the host.
//
// A membrane link joins node x (receiving population i, pulled from x - e_i)
// and x - e_i in another compartment; the membrane cuts it at distance delta
// from x.  Each side s of the membrane (x's, and the other one seen from
// x - e_i along -e_i) relates its stencil to its own value m_s at the
// membrane point and to the flux into it:
//   * along the link, with the Dirichlet and Neumann link relations and
//     their coefficients at the side's distance from the membrane (Eqs.
//     dirichlet_1/2, neumann_1/2 with Eqs. c_d, c_n): the Dirichlet relation
//     gives the arriving population as D_s + c_d4 eps m_s, and the
//     difference of the two relations gives the flux along the link;
//   * along each other lattice axis beta with a normal component, with the
//     same relations for Delta_m = 0 on the lattice line through the
//     membrane point (Eqs. phi_1, phi_2), whose populations at that point and
//     one spacing from it along e_betabar are interpolated along the link
//     direction (quadratic Lagrange interpolation through the three nodes of
//     the side's compartment nearest to the point).
// With the direction cosines of the normal the flux into side s normal to
// the membrane is L_s + A_s m_s, linear in the stencil (L_s) and in m_s.  The
// permeability condition with flux continuity (Eqs. B1, B1.5) asks for
// L_s + A_s m_s = kappa (m_t - m_s) on both sides s, t; the 2 x 2 system gives
// m_x, and the arriving population D_x + c_d4 eps m_x is a fixed linear
// combination of post-collision populations: the term list of the link.
// It depends on kappa, dt and the lattice (eps), so it is rebuilt whenever a
// forward's constants change.
#include "btl_curved.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <thread>

namespace btl {
namespace {

// lattice directions: 0 rest, 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z
constexpr int kDir[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                            {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
inline int reverse_dir(int d) { return (d & 1) ? d + 1 : d - 1; }

// Dirichlet (cd) and Neumann (cn) coefficients of the link relations of a
// node at distance delta from the membrane (Eqs. c_d, c_n), index 0..3 for
// c_1..c_4.
struct LinkRel {
    double cd[4], cn[4];
    explicit LinkRel(double delta) {
        const double den = 2.0 * delta + 1.0, m = 2.0 * delta - 1.0;
        cd[0] = 2.0 * delta - 2.0;
        cd[1] = -m * m / den;
        cd[2] = 2.0 * m / den;
        cd[3] = (3.0 - 2.0 * delta) / den;
        cn[0] = 1.0;
        cn[1] = -m / den;
        cn[2] = m / den;
        cn[3] = 2.0 / den;
    }
};

// a weighted post-collision population: direction q at node j (lattice
// coordinates, possibly beyond periodic faces)
struct Term {
    int32_t j[3];
    int32_t q;
    double w;
};

// A linear form over post-collision populations (at most 3 + 2 * 9 terms
// per side; two sides).
struct Form {
    Term t[48];
    int n = 0;
    void add(const int32_t j[3], int q, double w) {
        for (int k = 0; k < n; ++k)
            if (t[k].q == q && t[k].j[0] == j[0] && t[k].j[1] == j[1] && t[k].j[2] == j[2]) {
                t[k].w += w;
                return;
            }
        Term& e = t[n++];
        memcpy(e.j, j, sizeof(e.j));
        e.q = q;
        e.w = w;
    }
    void add_scaled(const Form& o, double c) {
        for (int k = 0; k < o.n; ++k) add(o.t[k].j, o.t[k].q, c * o.t[k].w);
    }
};

struct Ctx {
    const CurvedGeom& g;
    int nq;
    double eps, h;   // lattice eps_D; dt / dx
};

// node j belongs to compartment c (periodic axes wrap; no node lies beyond
// a mirroring face)
bool in_comp(const CurvedGeom& g, const int32_t j[3], uint32_t c) {
    int64_t w[3];
    for (int a = 0; a < 3; ++a) {
        int64_t v = j[a];
        if (v < 0 || v >= g.n[a]) {
            if (g.bc[a] != BTL_PERIODIC) return false;
            v %= g.n[a];
            if (v < 0) v += g.n[a];
        }
        w[a] = v;
    }
    return g.comp[(size_t)(w[0] + g.n[0] * (w[1] + (int64_t)g.n[1] * w[2]))] == c;
}

// Adds c times the population q at the point base + t e (|t| < 1), by
// quadratic interpolation through the three nodes base + u e (u = -3..3) of
// compartment c nearest to the point (equal distances: the smaller u first).
bool add_interp(const CurvedGeom& g, uint32_t c, int q, const int32_t base[3], const int e[3],
                double t, double coef, Form& f) {
    // candidates by distance to the point; insertion sort keeps equal
    // distances in ascending u
    int order[7] = {-3, -2, -1, 0, 1, 2, 3};
    for (int k = 1; k < 7; ++k) {
        const int u = order[k];
        int m = k;
        while (m > 0 && fabs(u - t) < fabs(order[m - 1] - t)) {
            order[m] = order[m - 1];
            --m;
        }
        order[m] = u;
    }
    int use[3], nu = 0;
    for (int k = 0; k < 7 && nu < 3; ++k) {
        int32_t j[3];
        for (int a = 0; a < 3; ++a) j[a] = base[a] + order[k] * e[a];
        if (in_comp(g, j, c)) use[nu++] = order[k];
    }
    if (nu < 3) return false;
    for (int m = 0; m < 3; ++m) {
        double lw = 1.0;
        for (int l = 0; l < 3; ++l)
            if (l != m) lw *= (t - use[l]) / (double)(use[m] - use[l]);
        int32_t j[3];
        for (int a = 0; a < 3; ++a) j[a] = base[a] + use[m] * e[a];
        f.add(j, q, coef * lw);
    }
    return true;
}

// One side of the membrane: node xs of compartment c receives along
// direction ds from the membrane at distance delta; nrm is the unit normal
// pointing into the side.  On success: the normal inflow is L + A m (m the
// side's value at the membrane) and the arriving population at xs is
// Dform + cd4 eps m.
struct Side {
    Form L, D;
    double A = 0.0, cd4 = 0.0;
};

bool side_relations(const Ctx& cx, uint32_t c, const int32_t xs[3], int ds, double delta,
                    const double nrm[3], Side& out) {
    const CurvedGeom& g = cx.g;
    const int* es = kDir[ds];
    const int ax = (ds - 1) / 2;
    const int dr = reverse_dir(ds);
    int32_t x2[3];
    for (int a = 0; a < 3; ++a) x2[a] = xs[a] + es[a];
    if (!in_comp(g, xs, c) || !in_comp(g, x2, c)) return false;
    // along the link: stencil ghat_dr(xs), ghat_dr(xs + e_s), ghat_ds(xs)
    const LinkRel r(delta);
    const double cth = fabs(nrm[ax]);
    const double fl = cth / (r.cn[3] * cx.h);
    out.D.add(xs, dr, r.cd[0]);
    out.D.add(x2, dr, r.cd[1]);
    out.D.add(xs, ds, r.cd[2]);
    out.L.add(xs, dr, fl * (r.cd[0] - r.cn[0]));
    out.L.add(x2, dr, fl * (r.cd[1] - r.cn[1]));
    out.L.add(xs, ds, fl * (r.cd[2] - r.cn[2]));
    out.A = fl * r.cd[3] * cx.eps;
    out.cd4 = r.cd[3];
    // across the link: the Delta_m = 0 relations on the line through the
    // membrane point along each other axis b with a normal component
    const LinkRel r0(0.0);
    for (int b = 0; b < 3; ++b) {
        if (b == ax || (cx.nq == 5 && b == 2)) continue;
        const double sb = fabs(nrm[b]);
        if (sb == 0.0) continue;
        const int sg = nrm[b] > 0.0 ? 1 : -1;
        const int d_in = 1 + 2 * b + (sg > 0 ? 0 : 1);   // e_betabar, into the side
        const int d_out = reverse_dir(d_in);
        int32_t xb[3];
        for (int a = 0; a < 3; ++a) xb[a] = xs[a] + (a == b ? sg : 0);
        const double fb = sb / (r0.cn[3] * cx.h);
        if (!add_interp(g, c, d_out, xs, es, -delta, fb * (r0.cd[0] - r0.cn[0]), out.L) ||
            !add_interp(g, c, d_out, xb, es, -delta, fb * (r0.cd[1] - r0.cn[1]), out.L) ||
            !add_interp(g, c, d_in, xs, es, -delta, fb * (r0.cd[2] - r0.cn[2]), out.L))
            return false;
        out.A += fb * r0.cd[3] * cx.eps;
    }
    return true;
}

}  // namespace

bool curved_collect(const btl_geom& g, CurvedGeom& out) {
    const int64_t n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], N = n0 * n1 * n2;
    for (int a = 0; a < 3; ++a) {
        out.n[a] = g.n[a];
        out.bc[a] = g.bc[a];
    }
    out.comp.assign(g.comp_id, g.comp_id + N);
    out.phase.resize((size_t)g.n_comp);
    for (int c = 0; c < g.n_comp; ++c) out.phase[c] = (uint8_t)g.comp_phase[c];
    out.links.clear();
    const float* ld = g.link_delta;
    const float* ln = g.link_normal;
    for (int64_t j2 = 0; j2 < n2; ++j2)
        for (int64_t j1 = 0; j1 < n1; ++j1)
            for (int64_t j0 = 0; j0 < n0; ++j0) {
                const int64_t s = j0 + n0 * (j1 + n1 * j2);
                for (int d = 1; d < 7; ++d) {
                    const int ax = (d - 1) / 2;
                    const int sg = kDir[d][ax];
                    int64_t src[3] = {j0, j1, j2};
                    src[ax] -= sg;
                    if (src[ax] < 0 || src[ax] >= g.n[ax]) {
                        if (g.bc[ax] != BTL_PERIODIC) continue;   // a node's own image
                        src[ax] = (src[ax] + g.n[ax]) % g.n[ax];
                    }
                    const int64_t ss = src[0] + n0 * (src[1] + n1 * src[2]);
                    if (g.comp_id[ss] == g.comp_id[s]) continue;
                    // link values sit on the link's lower node
                    const int64_t lower = sg > 0 ? ss : s;
                    CurvedGeom::Link L;
                    L.s = s;
                    L.d = d;
                    const double dl = ld[ax * N + lower];
                    L.dist = sg > 0 ? 1.0 - dl : dl;
                    double nn = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        L.nrm[c] = ln[(ax * 3 + c) * N + lower];
                        if (!isfinite(L.nrm[c])) return false;
                        nn += L.nrm[c] * L.nrm[c];
                    }
                    if (nn == 0.0) return false;
                    out.links.push_back(L);
                }
            }
    return true;
}

namespace {

// The term lists of the links [l0, l1) of cg: per link that takes the
// condition its index-table position, its (first term, count) within
// `terms`, and its terms.
struct Chunk {
    std::vector<int64_t> pos;
    std::vector<int4> heads;
    std::vector<CvTerm> terms;
};

void terms_range(const CurvedGeom& cg, int nq, double dt, double dx, const double* kappa, int P,
                 size_t l0, size_t l1, Chunk& out) {
    std::vector<int4>& heads = out.heads;
    std::vector<CvTerm>& terms = out.terms;
    const Ctx cx{cg, nq, lattice_eps(nq), dt / dx};
    const int64_t n0 = cg.n[0], n1 = cg.n[1];
    const int64_t N = n0 * n1 * cg.n[2];
    // the kernel's lattice: a single-layer D2Q5 geometry (n0, n1, 1) runs as
    // (n0, 1, n1), its y axis in the z slots (site order unchanged)
    const int kax[3] = {0, nq == 5 ? 2 : 1, nq == 5 ? 1 : 2};
    const int64_t kn0 = n0, kn1 = nq == 5 ? 1 : n1;
    const int64_t ps = kn0 * kn1, zs = (int64_t)nq * ps;
    auto pop_index = [&](const int64_t j[3]) {   // geometry coordinates, in range
        int64_t k[3];
        for (int a = 0; a < 3; ++a) k[kax[a]] = j[a];
        return k[0] + kn0 * k[1] + zs * k[2];
    };
    for (size_t li = l0; li < l1; ++li) {
        const CurvedGeom::Link& lk = cg.links[li];
        const int d = lk.d;
        if (nq == 5 && d > 4) continue;
        const int64_t s = lk.s;
        const int32_t x[3] = {(int32_t)(s % n0), (int32_t)((s / n0) % n1), (int32_t)(s / (n0 * n1))};
        const int ax = (d - 1) / 2;
        const int sg = kDir[d][ax];
        if (lk.nrm[ax] == 0.0) continue;   // membrane along the link: the other rules
        int32_t src[3] = {x[0], x[1], x[2]};
        src[ax] -= sg;
        const uint32_t c_own = cg.comp[(size_t)s];
        int64_t sw[3] = {src[0], src[1], src[2]};
        sw[ax] = (sw[ax] + cg.n[ax]) % cg.n[ax];
        const uint32_t c_far = cg.comp[(size_t)(sw[0] + n0 * (sw[1] + n1 * sw[2]))];
        const double kap = kappa[cg.phase[c_own] * P + cg.phase[c_far]];
        if (isinf(kap)) continue;   // no membrane between these phases
        // unit normal into x's side (positive along e_d) and into the other
        const double o = lk.nrm[ax] * sg > 0.0 ? 1.0 : -1.0;
        double n_own[3], n_far[3];
        for (int a = 0; a < 3; ++a) {
            n_own[a] = o * lk.nrm[a];
            n_far[a] = -n_own[a];
        }
        Side so, sf;
        if (!side_relations(cx, c_own, x, d, lk.dist, n_own, so) ||
            !side_relations(cx, c_far, src, reverse_dir(d), 1.0 - lk.dist, n_far, sf))
            continue;
        // L_o + A_o m_o = kappa (m_f - m_o), L_f + A_f m_f = kappa (m_o - m_f)
        double wo, wf;   // m_o = wo L_o + wf L_f
        if (kap == 0.0) {
            wo = -1.0 / so.A;
            wf = 0.0;
        } else {
            const double det = so.A * sf.A + kap * (so.A + sf.A);
            wo = -(sf.A + kap) / det;
            wf = -kap / det;
        }
        Form g;
        g.add_scaled(so.D, 1.0);
        const double cm = so.cd4 * cx.eps;
        g.add_scaled(so.L, cm * wo);
        if (wf != 0.0) g.add_scaled(sf.L, cm * wf);
        // kernel offsets relative to x and periodic-face counts
        const int64_t xj[3] = {x[0], x[1], x[2]};
        const int64_t base = pop_index(xj);
        const int32_t first = (int32_t)terms.size();
        bool ok = true;
        for (int k = 0; k < g.n && ok; ++k) {
            const Term& t = g.t[k];
            if (t.w == 0.0) continue;
            int64_t jw[3];
            int32_t wrap = 0;
            for (int a = 0; a < 3; ++a) {
                int64_t v = t.j[a];
                int wn = 0;
                while (v < 0) {
                    v += cg.n[a];
                    --wn;
                }
                while (v >= cg.n[a]) {
                    v -= cg.n[a];
                    ++wn;
                }
                jw[a] = v;
                if (wn < -3 || wn > 3) ok = false;
                const int face = 2 * kax[a] + (wn > 0 ? 1 : 0);
                wrap |= (wn < 0 ? -wn : wn) << (2 * face);
            }
            // every node lies inside the field (a guard: wrapped coordinates)
            const int64_t at = t.q * ps + pop_index(jw);
            if (at < 0 || at >= (int64_t)nq * N) ok = false;
            CvTerm ct;
            ct.w = t.w;
            ct.off = (int32_t)(at - base);
            ct.wrap = wrap;
            terms.push_back(ct);
        }
        if (!ok) {
            terms.resize((size_t)first);
            continue;
        }
        out.pos.push_back((d - 1) * N + s);
        heads.push_back(make_int4(first, (int32_t)terms.size() - first, (int32_t)base, d));
    }
}

}  // namespace

bool curved_terms(const CurvedGeom& cg, int nq, double dt, double dx, const double* kappa,
                  int P, int32_t* idx, std::vector<int4>& heads, std::vector<CvTerm>& terms) {
    // links are independent: chunks on up to 16 host threads, joined in order
    const size_t L = cg.links.size();
    size_t T = std::min<size_t>(16, std::max(1u, std::thread::hardware_concurrency()));
    if (L < 16384) T = 1;
    std::vector<Chunk> ch(T);
    std::vector<std::thread> th;
    for (size_t t = 1; t < T; ++t)
        th.emplace_back(terms_range, std::cref(cg), nq, dt, dx, kappa, P, L * t / T,
                        L * (t + 1) / T, std::ref(ch[t]));
    terms_range(cg, nq, dt, dx, kappa, P, 0, L / T, ch[0]);
    for (std::thread& x : th) x.join();
    // place the chunks one after another (each copied by its own thread)
    std::vector<size_t> h0(T + 1, heads.size()), t0(T + 1, terms.size());
    for (size_t t = 0; t < T; ++t) {
        h0[t + 1] = h0[t] + ch[t].heads.size();
        t0[t + 1] = t0[t] + ch[t].terms.size();
    }
    if (h0[T] > (size_t)INT32_MAX || t0[T] > (size_t)INT32_MAX) return false;
    heads.resize(h0[T]);
    terms.resize(t0[T]);
    auto place = [&](size_t t) {
        Chunk& c = ch[t];
        for (size_t k = 0; k < c.heads.size(); ++k) {
            idx[c.pos[k]] = (int32_t)(h0[t] + k);
            heads[h0[t] + k] = make_int4((int32_t)t0[t] + c.heads[k].x, c.heads[k].y,
                                         c.heads[k].z, c.heads[k].w);
        }
        std::copy(c.terms.begin(), c.terms.end(), terms.begin() + t0[t]);
        c = Chunk();
    };
    th.clear();
    for (size_t t = 1; t < T; ++t) th.emplace_back(place, t);
    place(0);
    for (std::thread& x : th) x.join();
    return true;
}

}  // namespace btl
