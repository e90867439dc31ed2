// Host runtime and C ABI of libbtlbm (declared in include/btlbm.h).
//
// The runtime validates inputs, turns the per-phase material parameters into
// the FP64 constants of one step (1/tau, T2 decay, membrane transmission),
// builds the field table (one field per q-sample plus reflected image fields
// where a mirrored face sees an oblique gradient), and enqueues one step
// launch per time step on the caller's stream.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/btlbm.h"
#include "btl_internal.h"

using namespace btl;

namespace {


struct GeomHost {
    int32_t n[3];
    int32_t bc[3];
    int64_t nsites;
    int64_t words_off;   // offset into the concatenated site-word array
    int64_t gm_off = -1; // offset into the membrane-position tables, -1: none
};

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t cap = 0;      // elements
    hipError_t ensure(size_t n) {
        if (n <= cap) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipMalloc(&p, n * sizeof(T));
        if (e == hipSuccess) cap = n;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

std::string g_create_error;

constexpr int kGraphMinSteps = 16;   // forwards this long run from a cached hipGraph
constexpr int kXcdMinBlocks = 2048;  // grids above this use the XCD-contiguous order

// Everything a captured forward depends on besides the contents of its
// buffers; a forward replays the cached graph only when this matches.
struct GraphKey {
    int32_t prec, K, Q, n_fields, nblk, shape, T, ckpt, scheme, nq, xcd;
    uint64_t fields;     // hash of the per-field values the launches take by value
    const void* ptr[16];
};

// FNV-1a over the field-table entries that the captured launches take as
// kernel arguments rather than read from the device table: the init
// launches' range, plane stride and q-sample of every field, the geometry
// (site words, membrane positions) behind it, and for the classical scheme
// the gradient terms of its initial reaction.  Two calls that agree in
// every other key entry but differ here (a permuted ragged batch, another
// gradient under the classical scheme) must not share a graph.
uint64_t field_hash(const std::vector<FieldDesc>& fl, bool classical) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    };
    for (const FieldDesc& d : fl) {
        mix(&d.pop, sizeof(d.pop));
        mix(&d.words, sizeof(d.words));
        mix(&d.gm, sizeof(d.gm));
        mix(d.n, sizeof(d.n));
        mix(&d.nsites, sizeof(d.nsites));
        mix(&d.q, sizeof(d.q));
        if (classical) {
            mix(d.c, sizeof(d.c));
            mix(&d.cu, sizeof(d.cu));
        }
    }
    return h;
}

}  // namespace

struct btl_sim {
    int prec = BTL_F32;
    int scheme = BTL_HYBRID;
    int substeps = 1;            // reaction sub-steps per step (waveform samples per step)
    int grad_g = 0;              // 1: taped forwards plan fields for the gamma G0 gradient
    int nq = 7;                  // lattice: 7 (D3Q7) or 5 (D2Q5 on single-layer geometries)
    int device = 0;
    double dx = 1.0;
    int32_t n_phase = 1;
    std::vector<GeomHost> geoms;
    DevBuf<uint32_t> words;
    DevBuf<float> gm;            // [6][nsites] per geometry with membrane positions
    DevBuf<char> pop[2];
    DevBuf<FieldDesc> fields;
    DevBuf<int32_t> blk_field;
    DevBuf<double> steps;        // fdt [K] then Fk [K+1]
    DevBuf<double> consts;       // w [P], decay [P], trans [P*P], T2 [P], kappa [P*P], dt/T2 [P]
    DevBuf<double2> partial;     // per-wave signal partials of kTabSteps steps
    DevBuf<double2> tab;         // [kTabSteps][T] per-step phase tables
    DevBuf<int32_t> tab_field;   // [T]
    std::vector<FieldDesc> h_fields;
    // launch geometry of the adjoint steps (the forward's tile shape with
    // its own z-column length)
    DevBuf<FieldDesc> adj_fields;
    DevBuf<int32_t> adj_blk;
    DevBuf<double> adj_gmeta;      // [fields][kGMeta] for the gamma G0 gradient
    // pinned staging for the per-call tables, two slots so that a call can
    // be prepared while the previous one's uploads are still queued
    char* stage[2] = {nullptr, nullptr};
    size_t stage_cap[2] = {0, 0};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_used[2] = {false, false};
    int stage_slot = 0;
    // cached forward graph
    hipGraphExec_t graph_exec = nullptr;
    GraphKey graph_key;
    hipStream_t cap_stream = nullptr;
    DevBuf<double> E_int;
    int tile_shape = -1;        // -1: pick per call from the geometry sizes
    int xcd = -1;               // workgroup order: -1 by grid size, 0 plain, 1 XCD-contiguous
    int zc = 0;                 // sites per thread along z; 0: whole column
    // inputs of the last forward call (the autotuner replays them)
    struct SimLastT {
        bool valid = false;
        double dt = 0;
        std::vector<double> D, T2, kappa, gG0, f;
        std::vector<int32_t> q_geom;
    } last;
    DevBuf<double> tune_E;
    using SimLast = SimLastT;
    // adjoint tape of the last forward that asked for one
    struct Tape {
        bool valid = false;
        int32_t K = 0, C = 0, Q = 0, T = 0, n_fields = 0, nblk = 0, shape = 0, sub = 1, xcd = 0;
        int32_t nblk_adj = 0;      // workgroups of one adjoint step (adj_fields)
        int32_t nq = 7;            // lattice of the taped forward
        bool g_ok = false;         // the field set supports the gamma G0 gradient
        double dt = 0;
        int64_t state_elems = 0;   // V elements of one full state (all fields)
    } tape;
    DevBuf<char> ckpt;             // [ceil(K/C)] states: ghat^{mC}
    DevBuf<char> seg;              // [C] states of the segment being reversed
    DevBuf<char> lam[2];
    DevBuf<double2> tab_b;         // [C+1][T] phase tables of a segment
    DevBuf<double> gpart;
    DevBuf<double> gfield;
    std::string err;
};

// The lattice as the kernels see it.  A single-layer D2Q5 geometry
// (n0, n1, 1) is run as (n0, 1, n1): its rows along y become the columns
// that one thread walks (the memory order of sites is the same), the y
// faces and gradient component move to the z slots, and the kernel maps its
// planes 3 and 4 to the z pulls.  D3Q7 geometries are unchanged.
static GeomHost kernel_geom(const GeomHost& g, int nq) {
    GeomHost k = g;
    if (nq == 5) {
        k.n[1] = 1;
        k.n[2] = g.n[1];
        k.bc[1] = BTL_PERIODIC;
        k.bc[2] = g.bc[1];
    }
    return k;
}
static void kernel_grad(const double* G, int nq, double* out) {
    out[0] = G[0];
    out[1] = nq == 5 ? 0.0 : G[1];
    out[2] = nq == 5 ? G[1] : G[2];
}

// Tile shape with the fewest idle lanes over the geometries of a call
// (ties go to the wider x extent: longer contiguous rows per wavefront).
// Single-layer lattices always take 256 x 1 (their tiles are one row).
static int pick_shape(const std::vector<GeomHost>& gs, const int32_t* q_geom, int Q, int nq) {
    if (nq == 5) return kTile256x1;
    int best = kTile128x2;
    int64_t best_waste = -1;
    for (int oi = 0; oi < kShapeCount3D; ++oi) {
        const int sh = kShapes3D[oi];
        int64_t waste = 0;
        for (int q = 0; q < Q; ++q) {
            const GeomHost& g = gs[q_geom[q]];
            int32_t t0, t1;
            tile_grid(sh, g.n[0], g.n[1], &t0, &t1);
            waste += ((int64_t)t0 * t1 * kBlock - (int64_t)g.n[0] * g.n[1]) * g.n[2];
        }
        if (best_waste < 0 || waste < best_waste) {
            best = sh;
            best_waste = waste;
        }
    }
    return best;
}

static btl_status fail(btl_sim* s, btl_status st, const std::string& msg) {
    if (s)
        s->err = msg;
    else
        g_create_error = msg;
    return st;
}

static btl_status hip_fail(btl_sim* s, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(s, e == hipErrorOutOfMemory ? BTL_E_NOMEM : BTL_E_HIP, m);
}

// Site word: bits 0-3 the phase, bit 4 + (d-1) set when the pull link of
// direction d (from node x - e_d into x) joins two different compartments,
// and bits 10 + 3(d-1) .. +2 the phase of that neighbour.  Links through a
// mirror face join a node with its own image: never a membrane.
static void build_words(const btl_geom& g, std::vector<uint32_t>& out) {
    const int64_t n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    static const int ex[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                                 {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    out.resize((size_t)(n0 * n1 * n2));
    for (int64_t j2 = 0; j2 < n2; ++j2)
        for (int64_t j1 = 0; j1 < n1; ++j1)
            for (int64_t j0 = 0; j0 < n0; ++j0) {
                const int64_t s = j0 + n0 * (j1 + n1 * j2);
                const uint32_t c = g.comp_id[s];
                uint32_t w = g.comp_phase[c];
                const int64_t jj[3] = {j0, j1, j2};
                for (int d = 1; d < 7; ++d) {
                    int64_t src[3];
                    bool mirror = false;
                    for (int a = 0; a < 3; ++a) {
                        src[a] = jj[a] - ex[d][a];
                        if (src[a] < 0 || src[a] >= g.n[a]) {
                            if (g.bc[a] == BTL_MIRROR)
                                mirror = true;
                            else
                                src[a] = (src[a] + g.n[a]) % g.n[a];
                        }
                    }
                    if (mirror) continue;
                    const uint32_t cs = g.comp_id[src[0] + n0 * (src[1] + n1 * src[2])];
                    if (cs != c) {
                        w |= 1u << (4 + d - 1);
                        w |= (uint32_t)g.comp_phase[cs] << (10 + 3 * (d - 1));
                    }
                }
                out[(size_t)s] = w;
            }
}

// Membrane-position table of one geometry for the general membrane
// condition: for the pull link of direction d into site x (from x - e_d),
// entry [(d-1)*nsites + x] is 0 when the link keeps the half-link rule, v > 0
// when the membrane lies at distance v from x and v < 0 when it lies at
// distance 1 + v (the link's value measured from its lower node x - e_d).
// The general rule needs the stencil x - 2e_d .. x + e_d inside the lattice
// (no outer face), x + e_d in x's compartment and x - 2e_d in that of
// x - e_d.  Returns false when a membrane link's value is not in (0, 1).
static bool build_gm(const btl_geom& g, std::vector<float>& out) {
    const int64_t n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], N = n0 * n1 * n2;
    const int64_t st[3] = {1, n0, n0 * n1};
    const float* ld = g.link_delta;
    out.assign((size_t)(6 * N), 0.0f);
    for (int64_t j2 = 0; j2 < n2; ++j2)
        for (int64_t j1 = 0; j1 < n1; ++j1)
            for (int64_t j0 = 0; j0 < n0; ++j0) {
                const int64_t s = j0 + n0 * (j1 + n1 * j2);
                const int64_t jj[3] = {j0, j1, j2};
                const uint32_t c = g.comp_id[s];
                for (int a = 0; a < 3; ++a) {
                    // every value a membrane link can be read from
                    const bool last = jj[a] == g.n[a] - 1;
                    if (last && g.bc[a] == BTL_MIRROR) continue;
                    const int64_t up = last ? s - (g.n[a] - 1) * st[a] : s + st[a];
                    if (g.comp_id[up] != c) {
                        const float v = ld[a * N + s];
                        if (!(v > 0.0f && v < 1.0f)) return false;
                    }
                }
                for (int d = 1; d < 7; ++d) {
                    const int a = (d - 1) / 2;
                    const int sg = (d & 1) ? 1 : -1;        // e_d = sg e_a
                    const int64_t j = jj[a];
                    if (j - 2 * sg < 0 || j - 2 * sg >= g.n[a] || j + sg < 0 || j + sg >= g.n[a])
                        continue;
                    const int64_t sm1 = s - sg * st[a], sm2 = s - 2 * sg * st[a], sp1 = s + sg * st[a];
                    const uint32_t cs = g.comp_id[sm1];
                    if (cs == c || g.comp_id[sp1] != c || g.comp_id[sm2] != cs) continue;
                    out[(size_t)((d - 1) * N + s)] = sg > 0 ? -ld[a * N + sm1] : ld[a * N + s];
                }
            }
    return true;
}

extern "C" btl_status btl_create(const btl_geom* geoms, int32_t n_geom, int32_t prec,
                                 btl_sim** out) {
    if (!out) return fail(nullptr, BTL_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!geoms || n_geom < 1) return fail(nullptr, BTL_E_INVAL, "need at least one geometry");
    if (prec != BTL_F32 && prec != BTL_F64) return fail(nullptr, BTL_E_INVAL, "prec must be BTL_F32 or BTL_F64");
    const double dx = geoms[0].dx;
    const int32_t P = geoms[0].n_phase;
    if (!(dx > 0) || !isfinite(dx)) return fail(nullptr, BTL_E_INVAL, "dx must be finite and > 0");
    if (P < 1 || P > 8) return fail(nullptr, BTL_E_INVAL, "n_phase must be in 1..8");
    for (int g = 0; g < n_geom; ++g) {
        const btl_geom& G = geoms[g];
        if (G.dx != dx || G.n_phase != P)
            return fail(nullptr, BTL_E_INVAL, "all geometries must share dx and n_phase");
        int64_t ns = 1;
        for (int a = 0; a < 3; ++a) {
            if (G.n[a] < (a == 2 ? 1 : 2))
                return fail(nullptr, BTL_E_INVAL, "x and y need >= 2 sites, z >= 1");
            if (G.bc[a] != BTL_PERIODIC && G.bc[a] != BTL_MIRROR)
                return fail(nullptr, BTL_E_INVAL, "bc must be BTL_PERIODIC or BTL_MIRROR");
            ns *= G.n[a];
        }
        if (ns > (int64_t)INT32_MAX / 8) return fail(nullptr, BTL_E_INVAL, "geometry too large (sites)");
        if (G.n_comp < 1 || !G.comp_id || !G.comp_phase)
            return fail(nullptr, BTL_E_INVAL, "comp_id/comp_phase missing");
        for (int c = 0; c < G.n_comp; ++c)
            if (G.comp_phase[c] >= P) return fail(nullptr, BTL_E_INVAL, "comp_phase value >= n_phase");
        for (int64_t s = 0; s < ns; ++s)
            if (G.comp_id[s] >= (uint32_t)G.n_comp)
                return fail(nullptr, BTL_E_INVAL, "comp_id value >= n_comp");
    }
    btl_sim* s = new btl_sim();
    s->prec = prec;
    s->dx = dx;
    s->n_phase = P;
    (void)hipGetDevice(&s->device);
    std::vector<uint32_t> all, one;
    std::vector<float> gm_all, gm_one;
    for (int g = 0; g < n_geom; ++g) {
        GeomHost h;
        for (int a = 0; a < 3; ++a) {
            h.n[a] = geoms[g].n[a];
            h.bc[a] = geoms[g].bc[a];
        }
        h.nsites = (int64_t)h.n[0] * h.n[1] * h.n[2];
        h.words_off = (int64_t)all.size();
        build_words(geoms[g], one);
        all.insert(all.end(), one.begin(), one.end());
        if (geoms[g].link_delta) {
            if (!build_gm(geoms[g], gm_one)) {
                btl_destroy(s);
                return fail(nullptr, BTL_E_INVAL, "link_delta must be in (0, 1) on membrane links");
            }
            h.gm_off = (int64_t)gm_all.size();
            gm_all.insert(gm_all.end(), gm_one.begin(), gm_one.end());
        }
        s->geoms.push_back(h);
    }
    hipError_t e = s->words.ensure(all.size());
    if (e == hipSuccess)
        e = hipMemcpy(s->words.p, all.data(), all.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !gm_all.empty()) {
        e = s->gm.ensure(gm_all.size());
        if (e == hipSuccess)
            e = hipMemcpy(s->gm.p, gm_all.data(), gm_all.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        btl_status st = hip_fail(nullptr, e, "uploading site words");
        btl_destroy(s);
        return st;
    }
    *out = s;
    return BTL_OK;
}

// Field table of one q-sample.  A mirrored axis whose gradient component is
// non-zero makes the reflected medium depend on the sign of that component,
// so the q-sample carries one field per sign pattern sigma over those axes
// (sigma_a = 1: the copy reflected in axis a).  When every axis with a
// non-zero component is mirrored, the copy reflected in all of them is the
// complex conjugate of the primary (times a uniform phase), which halves the
// set: only patterns with sigma_{a*} = 0 (a* the first such axis) are kept.
// That symmetry needs the reaction as an exact phase factor; the classical
// scheme (reaction term inside the collision) keeps every pattern.
struct QFields {
    std::vector<int> sigma;   // canonical sign patterns, sigma[0] = 0 (primary)
    int amask = 0;
    bool conj_pair = false;
};

// full: the set a gradient with respect to gamma G0 needs, valid for every
// nearby G and not only for this one: every mirrored axis counts as carrying
// a component, and the conjugate pairing is kept only when every axis is
// mirrored (a periodic axis with a zero component would break it).  An axis
// one site long (the single layer of the D2Q5 lattice) has no links and no
// gradient component, and does not count.
static QFields plan_fields(const GeomHost& g, const double* G, bool classical, bool full = false) {
    QFields r;
    bool all_mirrored = true;
    int astar = -1;
    for (int a = 0; a < 3; ++a) {
        if (full) {
            if (g.n[a] == 1) continue;   // no links along it (the single layer)
            if (g.bc[a] == BTL_MIRROR) {
                r.amask |= 1 << a;
                if (astar < 0) astar = a;
            } else {
                all_mirrored = false;
            }
            continue;
        }
        if (G[a] == 0.0) continue;
        if (g.bc[a] == BTL_MIRROR) {
            r.amask |= 1 << a;
            if (astar < 0) astar = a;
        } else {
            all_mirrored = false;
        }
    }
    r.conj_pair = (r.amask != 0) && all_mirrored && !classical;
    for (int sg = 0; sg < 8; ++sg) {
        if ((sg & ~r.amask) != 0) continue;
        if (r.conj_pair && ((sg >> astar) & 1)) continue;
        r.sigma.push_back(sg);
    }
    return r;
}

static btl_status forward_impl(btl_sim* s, double dt, int32_t K, const double* D,
                               const double* T2, const double* kappa, int32_t Q,
                               const int32_t* q_geom, const double* gG0, const double* f,
                               double* E, void* M_final, int32_t ckpt_every, void* stream) {
    if (!s) return BTL_E_INVAL;
    if (!(dt > 0) || !isfinite(dt)) return fail(s, BTL_E_INVAL, "dt must be finite and > 0");
    if (K < 0) return fail(s, BTL_E_INVAL, "K must be >= 0");
    if (Q < 1) return fail(s, BTL_E_INVAL, "Q must be >= 1");
    if (!D || !T2 || !kappa || !q_geom || !gG0 || (K > 0 && !f) || !E)
        return fail(s, BTL_E_INVAL, "NULL argument");
    if (ckpt_every < 0) return fail(s, BTL_E_INVAL, "ckpt_every must be >= 0");
    const int32_t P = s->n_phase;
    for (int p = 0; p < P; ++p) {
        if (!(D[p] > 0) || !isfinite(D[p])) return fail(s, BTL_E_INVAL, "D must be finite and > 0");
        if (!(T2[p] > 0)) return fail(s, BTL_E_INVAL, "T2 must be > 0");
    }
    for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) {
            const double k = kappa[a * P + b];
            if (!(k >= 0)) return fail(s, BTL_E_INVAL, "kappa must be >= 0");
            if (k != kappa[b * P + a]) return fail(s, BTL_E_INVAL, "kappa must be symmetric");
        }
    const int32_t msub = s->substeps;
    const int32_t nq = s->nq;
    const double eps = lattice_eps(nq);
    for (int q = 0; q < Q; ++q) {
        if (q_geom[q] < 0 || q_geom[q] >= (int)s->geoms.size())
            return fail(s, BTL_E_INVAL, "q_geom out of range");
        for (int a = 0; a < 3; ++a)
            if (!isfinite(gG0[3 * q + a])) return fail(s, BTL_E_INVAL, "gG0 must be finite");
    }
    if (nq == 5)
        for (int q = 0; q < Q; ++q)
            if (s->geoms[q_geom[q]].n[2] != 1 || gG0[3 * q + 2] != 0.0)
                return fail(s, BTL_E_INVAL, "D2Q5 needs single-layer geometries (n[2] = 1) "
                                             "and no gradient along z");
    if (msub > 1 && s->scheme == BTL_CLASSICAL)
        return fail(s, BTL_E_UNSUPPORTED, "reaction sub-steps need the hybrid scheme");
    for (int64_t k = 0; k < (int64_t)K * msub; ++k)
        if (!isfinite(f[k])) return fail(s, BTL_E_INVAL, "f must be finite");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double dx = s->dx;

    // per-phase and per-pair constants (FP64)
    std::vector<double> consts(2 * P + P * P + P + P * P + P + P * P);
    for (int p = 0; p < P; ++p) {
        const double tau = 0.5 + dt * D[p] / (eps * dx * dx);
        consts[p] = 1.0 / tau;
        consts[P + p] = isinf(T2[p]) ? 1.0 : exp(-dt / T2[p]);
    }
    for (int i = 0; i < P * P; ++i) {
        const double k = kappa[i];
        double t;
        if (isinf(k))
            t = 1.0;
        else if (k == 0.0)
            t = 0.0;
        else {
            const double Pm = eps * dx / (2.0 * k * dt);
            t = 1.0 / (1.0 + Pm);
        }
        consts[2 * P + i] = t;
    }
    for (int p = 0; p < P; ++p) consts[2 * P + P * P + p] = T2[p];
    for (int i = 0; i < P * P; ++i) consts[3 * P + P * P + i] = kappa[i];
    for (int p = 0; p < P; ++p) consts[3 * P + 2 * P * P + p] = isinf(T2[p]) ? 0.0 : dt / T2[p];
    for (int i = 0; i < P * P; ++i) consts[4 * P + 2 * P * P + i] = kappa[i] * dt;
    bool uses_gm = false;
    for (int q = 0; q < Q; ++q) uses_gm |= s->geoms[q_geom[q]].gm_off >= 0;
    const bool classical = s->scheme == BTL_CLASSICAL;
    // per-step waveform tables: f_k dt and F_k.  With m reaction sub-steps
    // of dt' = dt/m (Sec. 2.3) the reaction of step k is the product of m
    // exact phase factors, i.e. one factor with the summed angle, so f_k dt
    // becomes sum_j f[k m + j] dt'.
    std::vector<double> steps((size_t)K + (size_t)K + 1);
    {
        const double dts = dt / msub;
        double F = 0.0;
        for (int k = 0; k < K; ++k) {
            double a = 0.0;
            for (int j = 0; j < msub; ++j) a += f[(size_t)k * msub + j] * dts;
            steps[k] = a;
            steps[(size_t)K + k] = F;
            F += a;
        }
        steps[(size_t)2 * K] = F;
    }

    // launch shape
    int shape = s->tile_shape >= 0 ? s->tile_shape : pick_shape(s->geoms, q_geom, Q, nq);
    if ((nq == 5) != (shape == kTile256x1)) shape = pick_shape(s->geoms, q_geom, Q, nq);
    int ZC = s->zc;
    if (ZC <= 0) {
        ZC = 1;
        for (int q = 0; q < Q; ++q) ZC = std::max(ZC, kernel_geom(s->geoms[q_geom[q]], nq).n[2]);
    }
    ZC = std::min(ZC, kMaxZc);

    // field table
    std::vector<FieldDesc>& fl = s->h_fields;
    fl.clear();
    bool g_complete = true;   // every q-sample's field set is the full one
    // per field: owning q-sample, s_b, sigma_b and d beta_f / d G_b (kGMeta)
    std::vector<double> gmeta;
    int64_t pop_elems = 0;
    int32_t nblk_total = 0;
    for (int q = 0; q < Q; ++q) {
        const GeomHost g = kernel_geom(s->geoms[q_geom[q]], nq);
        double G[3];
        kernel_grad(gG0 + 3 * q, nq, G);
        const bool full = s->grad_g && ckpt_every > 0 && K > 0;
        QFields qf = plan_fields(g, G, s->scheme == BTL_CLASSICAL, full);
        {
            const QFields qa = plan_fields(g, G, s->scheme == BTL_CLASSICAL, true);
            if (!(qa.amask == qf.amask && qa.conj_pair == qf.conj_pair && qa.sigma == qf.sigma))
                g_complete = false;
        }
        const int base = (int)fl.size();
        auto slot_of = [&](int sg, int* cj) {
            for (size_t i = 0; i < qf.sigma.size(); ++i)
                if (qf.sigma[i] == sg) {
                    *cj = 0;
                    return base + (int)i;
                }
            const int sb = sg ^ qf.amask;
            for (size_t i = 0; i < qf.sigma.size(); ++i)
                if (qf.sigma[i] == sb) {
                    *cj = 1;
                    return base + (int)i;
                }
            *cj = -1;
            return -1;
        };
        double gsum = 0.0;
        for (int a = 0; a < 3; ++a) gsum += G[a];
        for (size_t fi = 0; fi < qf.sigma.size(); ++fi) {
            FieldDesc d;
            memset(&d, 0, sizeof(d));
            const int sg = qf.sigma[fi];
            d.pop = pop_elems;
            d.words = g.words_off;
            for (int a = 0; a < 3; ++a) d.n[a] = g.n[a];
            d.nsites = (int32_t)g.nsites;
            d.blk0 = nblk_total;
            d.zc = ZC;
            tile_grid(shape, g.n[0], g.n[1], &d.tiles[0], &d.tiles[1]);
            d.tiles[2] = (g.n[2] + ZC - 1) / ZC;
            d.nblk = d.tiles[0] * d.tiles[1] * d.tiles[2];
            d.q = fi == 0 ? q : -1;
            d.gm = g.gm_off;
            d.cu = 0.0;
            for (int a = 0; a < 3; ++a) {
                const int sig = (sg >> a) & 1;
                d.c[a] = G[a] * dx * (sig ? -1.0 : 1.0);
                if (sig) d.cu -= dx * G[a];
            }
            fl.push_back(d);
            {
                double gm[kGMeta] = {0.0};
                gm[0] = q;
                for (int a = 0; a < 3; ++a) {
                    const int sig = (sg >> a) & 1;
                    gm[1 + a] = sig ? -1.0 : 1.0;
                    gm[4 + a] = sig;
                }
                gmeta.insert(gmeta.end(), gm, gm + kGMeta);
            }
            pop_elems += (int64_t)nq * g.nsites;
            nblk_total += d.nblk;
        }
        // faces (needs all slots of this q allocated)
        for (size_t fi = 0; fi < qf.sigma.size(); ++fi) {
            FieldDesc& d = fl[base + fi];
            const int sg = qf.sigma[fi];
            for (int a = 0; a < 3; ++a) {
                const double La = g.n[a] * dx;
                if (g.bc[a] == BTL_PERIODIC) {
                    // ghat(x_-1) = e^{+i phi} ghat(x_{N-1}), ghat(x_N) = e^{-i phi} ghat(x_0)
                    d.face_kind[2 * a] = d.face_kind[2 * a + 1] = kFacePeriodic;
                    d.face_pop[2 * a] = d.face_pop[2 * a + 1] = d.pop;
                    d.beta[2 * a] = La * G[a];
                    d.beta[2 * a + 1] = -La * G[a];
                    double* gm = &gmeta[(size_t)(base + fi) * kGMeta + 7];
                    gm[3 * (2 * a) + a] = La;
                    gm[3 * (2 * a + 1) + a] = -La;
                } else {
                    const int sa = ((sg >> a) & 1) ? -1 : 1;
                    const int sp = (qf.amask >> a) & 1 ? (sg ^ (1 << a)) : sg;
                    int cj = 0;
                    const int slot = slot_of(sp, &cj);
                    const double gam = cj ? dx * gsum : 0.0;
                    const int kind = kFaceMirror | (cj ? kFaceConj : 0);
                    d.face_kind[2 * a] = d.face_kind[2 * a + 1] = kind;
                    d.face_pop[2 * a] = d.face_pop[2 * a + 1] = fl[slot].pop;
                    d.beta[2 * a] = gam;
                    d.beta[2 * a + 1] = -sa * 2.0 * La * G[a] + gam;
                    double* gm = &gmeta[(size_t)(base + fi) * kGMeta + 7];
                    for (int b = 0; b < 3; ++b) {
                        gm[3 * (2 * a) + b] = cj ? dx : 0.0;
                        gm[3 * (2 * a + 1) + b] = (cj ? dx : 0.0) + (b == a ? -sa * 2.0 * La : 0.0);
                    }
                }
            }
        }
        // adjoint pull through each face: periodic faces read the same field
        // at the wrapped node with the forward factor of the opposite face;
        // mirror faces read the partner field (the forward source of that
        // face, an involution) with that partner's factor and conjugation
        for (size_t fi = 0; fi < qf.sigma.size(); ++fi) {
            FieldDesc& d = fl[base + fi];
            for (int f = 0; f < 6; ++f) {
                if ((d.face_kind[f] & kFaceMirror) == 0) {
                    d.adj_kind[f] = kFacePeriodic;
                    d.adj_pop[f] = d.pop;
                    d.adj_fac[f] = -1 - (f ^ 1);          // own table, resolved below
                } else {
                    int partner = -1;
                    for (size_t pj = 0; pj < qf.sigma.size(); ++pj)
                        if (fl[base + pj].pop == d.face_pop[f]) partner = base + (int)pj;
                    d.adj_kind[f] = fl[partner].face_kind[f];
                    d.adj_pop[f] = fl[partner].pop;
                    d.adj_fac[f] = -1000 - (partner * 6 + f);  // partner table, resolved below
                }
            }
        }
    }
    const int32_t n_fields = (int32_t)fl.size();
    // the kernels address a field's reads with 32-bit element offsets from
    // its own base: every plane it reads must lie within +-2^31 elements
    for (int i = 0; i < n_fields; ++i) {
        int64_t lo = 0, hi = (int64_t)nq * fl[i].nsites;
        for (int f = 0; f < 6; ++f) {
            lo = std::min(lo, fl[i].face_pop[f] - fl[i].pop);
            hi = std::max(hi, fl[i].face_pop[f] - fl[i].pop + (int64_t)nq * fl[i].nsites);
            lo = std::min(lo, fl[i].adj_pop[f] - fl[i].pop);
            hi = std::max(hi, fl[i].adj_pop[f] - fl[i].pop + (int64_t)nq * fl[i].nsites);
        }
        if (lo < -(int64_t)INT32_MAX || hi > (int64_t)INT32_MAX)
            return fail(s, BTL_E_UNSUPPORTED, "geometry too large for the image fields of one q-sample");
    }
    // phase tables: per field [n0 + n1 + n2 + 6] entries
    int32_t T = 0;
    for (int i = 0; i < n_fields; ++i) {
        fl[i].tab = T;
        T += fl[i].n[0] + fl[i].n[1] + fl[i].n[2] + 6;
    }
    for (int i = 0; i < n_fields; ++i)
        for (int f = 0; f < 6; ++f) {
            const int32_t v = fl[i].adj_fac[f];
            if (v <= -1000) {
                const int partner = (-1000 - v) / 6, pf = (-1000 - v) % 6;
                fl[i].adj_fac[f] = fl[partner].tab + fl[partner].n[0] + fl[partner].n[1] +
                                   fl[partner].n[2] + pf;
            } else {
                fl[i].adj_fac[f] = fl[i].tab + fl[i].n[0] + fl[i].n[1] + fl[i].n[2] + (-1 - v);
            }
        }
    std::vector<int32_t> tabf(T);
    for (int i = 0; i < n_fields; ++i)
        for (int e = 0; e < fl[i].n[0] + fl[i].n[1] + fl[i].n[2] + 6; ++e) tabf[fl[i].tab + e] = i;
    std::vector<int32_t> blk(nblk_total);
    for (int i = 0; i < n_fields; ++i)
        for (int b = 0; b < fl[i].nblk; ++b) blk[fl[i].blk0 + b] = i;
    // With a tape, the launch geometry of the adjoint steps: the same tile
    // shape, whole z columns when all workgroups are resident at once (cut
    // into as many pieces as still fit at once when that leaves SIMDs with
    // room), otherwise columns cut so that the grid runs in about eight rounds
    // (BTLBM_ADJ_ZC sets the length).  The adjoint carries four values along
    // the column and loads in two phases per site; on the benchmark workload
    // it measured faster on whole columns than on the short chunks the
    // forward step often prefers, but a grid slightly larger than one round
    // of resident workgroups leaves most of the chip idle in its second.
    const bool taping = ckpt_every > 0 && K > 0;
    std::vector<FieldDesc> afl;
    std::vector<int32_t> ablk;
    int32_t nblk_adj = 0;
    if (taping) {
        const char* ez = getenv("BTLBM_ADJ_ZC");
        int zc_adj = ez ? std::max(0, atoi(ez)) : 0;
        if (!ez) {
            // resident workgroups: 1024 SIMDs x (4 waves FP32, 2 FP64) / 4 waves each
            const int64_t cap = s->prec == BTL_F32 ? 1024 : 512;
            int64_t whole = 0;
            int32_t nz = 1;
            for (const FieldDesc& d : fl) {
                whole += (int64_t)d.tiles[0] * d.tiles[1];
                nz = std::max(nz, d.n[2]);
            }
            if (whole > cap) {
                const int64_t split = (8 * cap + whole - 1) / whole;
                zc_adj = std::max<int>(8, (int)((nz + split - 1) / split));
            } else if (2 * whole <= cap) {
                // cut the columns so that the grid still fits at once but
                // fills the SIMDs (512 whole-column workgroups would leave
                // two waves per SIMD)
                const int64_t split = cap / whole;
                zc_adj = (int)((nz + split - 1) / split);
            }
        }
        afl = fl;
        for (FieldDesc& d : afl) {
            const int32_t zc = zc_adj > 0 ? std::min(zc_adj, d.n[2]) : d.n[2];
            d.zc = zc;
            d.tiles[2] = (d.n[2] + zc - 1) / zc;
            d.nblk = d.tiles[0] * d.tiles[1] * d.tiles[2];
            d.blk0 = nblk_adj;
            nblk_adj += d.nblk;
        }
        ablk.resize(nblk_adj);
        for (int i = 0; i < n_fields; ++i)
            for (int b = 0; b < afl[i].nblk; ++b) ablk[afl[i].blk0 + b] = i;
    }

    const size_t esz = s->prec == BTL_F32 ? sizeof(float2) : sizeof(double2);
    hipError_t e;
    if ((e = s->pop[0].ensure((size_t)pop_elems * esz)) != hipSuccess ||
        (e = s->pop[1].ensure((size_t)pop_elems * esz)) != hipSuccess)
        return hip_fail(s, e, "allocating populations");
    if ((e = s->fields.ensure(n_fields)) != hipSuccess ||
        (e = s->blk_field.ensure(nblk_total)) != hipSuccess ||
        (e = s->steps.ensure(steps.size())) != hipSuccess ||
        (e = s->consts.ensure(consts.size())) != hipSuccess ||
        (e = s->partial.ensure((size_t)kTabSteps * nblk_total * (kBlock / 64))) != hipSuccess ||
        (e = s->tab.ensure((size_t)kTabSteps * T)) != hipSuccess ||
        (e = s->tab_field.ensure(T)) != hipSuccess ||
        (taping && ((e = s->adj_fields.ensure(n_fields)) != hipSuccess ||
                    (e = s->adj_blk.ensure(nblk_adj)) != hipSuccess ||
                    (e = s->adj_gmeta.ensure((size_t)n_fields * kGMeta)) != hipSuccess)))
        return hip_fail(s, e, "allocating tables");
    // stage all tables in pinned memory and upload asynchronously
    const size_t b_fields = (size_t)n_fields * sizeof(FieldDesc);
    const size_t b_blk = (size_t)nblk_total * sizeof(int32_t);
    const size_t b_steps = steps.size() * sizeof(double);
    const size_t b_consts = consts.size() * sizeof(double);
    const size_t b_tabf = (size_t)T * sizeof(int32_t);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_blk = al(b_fields), o_steps = o_blk + al(b_blk), o_consts = o_steps + al(b_steps);
    const size_t o_tabf = o_consts + al(b_consts);
    const size_t b_afl = taping ? b_fields : 0, b_ablk = (size_t)nblk_adj * sizeof(int32_t);
    const size_t b_agm = taping ? (size_t)n_fields * kGMeta * sizeof(double) : 0;
    const size_t o_afl = o_tabf + al(b_tabf), o_ablk = o_afl + al(b_afl);
    const size_t o_agm = o_ablk + al(b_ablk);
    const size_t total = o_agm + al(b_agm);
    const int slot = s->stage_slot;
    if (!s->stage_ev[slot] && (e = hipEventCreateWithFlags(&s->stage_ev[slot], hipEventDisableTiming)) != hipSuccess)
        return hip_fail(s, e, "creating event");
    if (s->stage_used[slot] && (e = hipEventSynchronize(s->stage_ev[slot])) != hipSuccess)
        return hip_fail(s, e, "waiting for staging slot");
    if (s->stage_cap[slot] < total) {
        if (s->stage[slot]) (void)hipHostFree(s->stage[slot]);
        s->stage[slot] = nullptr;
        s->stage_cap[slot] = 0;
        if ((e = hipHostMalloc((void**)&s->stage[slot], total, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(s, e, "allocating pinned staging");
        s->stage_cap[slot] = total;
    }
    char* stg = s->stage[slot];
    memcpy(stg, fl.data(), b_fields);
    memcpy(stg + o_blk, blk.data(), b_blk);
    memcpy(stg + o_steps, steps.data(), b_steps);
    memcpy(stg + o_consts, consts.data(), b_consts);
    memcpy(stg + o_tabf, tabf.data(), b_tabf);
    if (taping) {
        memcpy(stg + o_afl, afl.data(), b_afl);
        memcpy(stg + o_ablk, ablk.data(), b_ablk);
        memcpy(stg + o_agm, gmeta.data(), b_agm);
    }
    if ((e = hipMemcpyAsync(s->fields.p, stg, b_fields, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(s->blk_field.p, stg + o_blk, b_blk, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(s->steps.p, stg + o_steps, b_steps, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(s->consts.p, stg + o_consts, b_consts, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(s->tab_field.p, stg + o_tabf, b_tabf, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (taping &&
         ((e = hipMemcpyAsync(s->adj_fields.p, stg + o_afl, b_afl, hipMemcpyHostToDevice, st)) != hipSuccess ||
          (e = hipMemcpyAsync(s->adj_blk.p, stg + o_ablk, b_ablk, hipMemcpyHostToDevice, st)) != hipSuccess ||
          (e = hipMemcpyAsync(s->adj_gmeta.p, stg + o_agm, b_agm, hipMemcpyHostToDevice, st)) != hipSuccess)) ||
        (e = hipEventRecord(s->stage_ev[slot], st)) != hipSuccess)
        return hip_fail(s, e, "uploading tables");
    s->stage_used[slot] = true;
    s->stage_slot ^= 1;

    s->tape.valid = false;
    // XCD-contiguous workgroup order pays off when the grid runs in several
    // waves (tiles that share edge rows then meet in one XCD's L2); grids
    // that fit on the chip at once keep the plain order.  The autotuner
    // measures both.
    const int xcd_on = s->xcd >= 0 ? s->xcd : (nblk_total > kXcdMinBlocks ? 1 : 0);
    const size_t state_bytes = (size_t)pop_elems * esz;
    if (ckpt_every > 0 && K > 0) {
        if (P > kAdjMaxPhase) return fail(s, BTL_E_UNSUPPORTED, "the adjoint supports n_phase <= 4");
        if (classical) return fail(s, BTL_E_UNSUPPORTED, "the adjoint supports the hybrid scheme only");
        if (uses_gm)
            return fail(s, BTL_E_UNSUPPORTED, "the adjoint supports the half-link membrane rule only");
        const int32_t C = std::min(ckpt_every, K);
        const int32_t nck = (K + C - 1) / C;
        if ((e = s->ckpt.ensure((size_t)nck * state_bytes)) != hipSuccess)
            return hip_fail(s, e, "allocating checkpoints");
        s->tape.K = K;
        s->tape.C = C;
        s->tape.Q = Q;
        s->tape.T = T;
        s->tape.n_fields = n_fields;
        s->tape.nblk = nblk_total;
        s->tape.nblk_adj = nblk_adj;
        s->tape.g_ok = g_complete;
        s->tape.shape = shape;
        s->tape.dt = dt;
        s->tape.sub = msub;
        s->tape.xcd = xcd_on;
        s->tape.state_elems = pop_elems;
        s->tape.nq = nq;
    }
    // Everything a forward enqueues after the uploads: init, one table
    // launch per kTabSteps steps, one step launch per step, checkpoint
    // copies.  Replayed from a cached hipGraph when the call has the same
    // shape and buffers as the previous one.
    auto enqueue = [&](hipStream_t q, double* Eptr) -> btl_status {
        hipError_t err;
        if ((err = launch_init(s->prec, s->pop[0].p, pop_elems, s->fields.p, n_fields, fl.data(),
                               Eptr, Q, K, nq, q)) != hipSuccess)
            return hip_fail(s, err, "init launch");
        if (classical && K > 0 &&
            (err = launch_init_classical(s->prec, s->pop[0].p, fl.data(), n_fields, s->words.p,
                                         s->steps.p, s->consts.p + 3 * P + 2 * P * P, nq, q)) !=
                hipSuccess)
            return hip_fail(s, err, "init launch");
        if (ckpt_every > 0 && K > 0 &&
            (err = hipMemcpyAsync(s->ckpt.p, s->pop[0].p, state_bytes, hipMemcpyDeviceToDevice, q)) !=
                hipSuccess)
            return hip_fail(s, err, "checkpoint copy");
        StepArgs a;
        memset(&a, 0, sizeof(a));
        a.words = s->words.p;
        a.fields = s->fields.p;
        a.blk_field = s->blk_field.p;
        a.fdt = s->steps.p;
        a.Fk = s->steps.p + K;
        a.w = s->consts.p;
        a.decay = s->consts.p + P;
        a.trans = s->consts.p + 2 * P;
        a.rdt = s->consts.p + 3 * P + 2 * P * P;
        a.gm = uses_gm ? s->gm.p : nullptr;
        a.kdt = s->consts.p + 4 * P + 2 * P * P;
        a.edx = eps * dx;
        a.nq = nq;
        a.xcd = xcd_on;
        a.classical = classical ? 1 : 0;
        a.partial = s->partial.p;
        a.n_phase = P;
        a.K = K;
        a.tab_field = s->tab_field.p;
        a.T = T;
        for (int k = 0; k < K; ++k) {
            if (k % kTabSteps == 0) {
                a.k = k;
                a.tab = s->tab.p;
                if ((err = launch_tables(a, std::min(kTabSteps, K - k), q)) != hipSuccess)
                    return hip_fail(s, err, "table launch");
            }
            a.tab = s->tab.p + (size_t)(k % kTabSteps) * T;
            a.src = s->pop[k & 1].p;
            a.dst = s->pop[(k + 1) & 1].p;
            a.k = k;
            if ((err = launch_step(s->prec, shape, a, nblk_total, q)) != hipSuccess)
                return hip_fail(s, err, "step launch");
            if ((k + 1) % kTabSteps == 0 || k + 1 == K) {
                const int32_t k0 = k - k % kTabSteps;
                if ((err = launch_esum(s->partial.p, s->fields.p, n_fields, nblk_total, k0,
                                       k + 1 - k0, Eptr, K, q)) != hipSuccess)
                    return hip_fail(s, err, "signal launch");
            }
            if (ckpt_every > 0 && (k + 1) % s->tape.C == 0 && k + 1 < K) {
                const size_t m = (size_t)(k + 1) / s->tape.C;
                if ((err = hipMemcpyAsync(s->ckpt.p + m * state_bytes, s->pop[(k + 1) & 1].p,
                                          state_bytes, hipMemcpyDeviceToDevice, q)) != hipSuccess)
                    return hip_fail(s, err, "checkpoint copy");
            }
        }
        return BTL_OK;
    };
    const bool use_graph = K >= kGraphMinSteps && getenv("BTLBM_NO_GRAPH") == nullptr;
    if (!use_graph) {
        const btl_status rc = enqueue(st, E);
        if (rc != BTL_OK) return rc;
    } else {
        const size_t ebytes = (size_t)Q * (K + 1) * 2 * sizeof(double);
        if ((e = s->E_int.ensure((size_t)Q * (K + 1) * 2)) != hipSuccess)
            return hip_fail(s, e, "allocating signal buffer");
        GraphKey key;
        memset(&key, 0, sizeof(key));
        key.prec = s->prec;
        key.K = K;
        key.Q = Q;
        key.n_fields = n_fields;
        key.nblk = nblk_total;
        key.shape = shape;
        key.T = T;
        key.ckpt = ckpt_every;
        key.scheme = s->scheme;
        key.nq = nq;
        key.xcd = xcd_on;
        key.fields = field_hash(fl, classical);
        const void* ptrs[] = {s->pop[0].p, s->pop[1].p, s->fields.p, s->blk_field.p, s->steps.p,
                              s->consts.p, s->partial.p, s->tab.p, s->tab_field.p,
                              s->E_int.p, s->ckpt.p, s->words.p};
        static_assert(sizeof(ptrs) / sizeof(ptrs[0]) <= sizeof(key.ptr) / sizeof(key.ptr[0]),
                      "graph key too small");
        for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) key.ptr[i] = ptrs[i];
        if (!(s->graph_exec && memcmp(&key, &s->graph_key, sizeof(key)) == 0)) {
            if (s->graph_exec) {
                (void)hipGraphExecDestroy(s->graph_exec);
                s->graph_exec = nullptr;
            }
            if (!s->cap_stream &&
                (e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(s, e, "creating capture stream");
            if ((e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return hip_fail(s, e, "begin capture");
            const btl_status rc = enqueue(s->cap_stream, s->E_int.p);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(s->cap_stream, &graph);
            if (rc != BTL_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (ec != hipSuccess) return hip_fail(s, ec, "end capture");
            e = hipGraphInstantiate(&s->graph_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                s->graph_exec = nullptr;
                return hip_fail(s, e, "graph instantiate");
            }
            s->graph_key = key;
        }
        if ((e = hipGraphLaunch(s->graph_exec, st)) != hipSuccess) return hip_fail(s, e, "graph launch");
        if ((e = hipMemcpyAsync(E, s->E_int.p, ebytes, hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return hip_fail(s, e, "signal copy");
    }
    if (ckpt_every > 0 && K > 0) s->tape.valid = true;
    if (M_final) {
        if ((e = launch_mfinal(s->prec, s->pop[K & 1].p, fl.data(), n_fields, M_final, nq, st)) !=
            hipSuccess)
            return hip_fail(s, e, "final magnetization launch");
    }
    return BTL_OK;
}

// Fields of one q-sample: 2^(k-1) or 2^k image fields, see plan_fields.
static int64_t q_state_elems(const btl_sim* s, int32_t g, const double* G) {
    const GeomHost gh = kernel_geom(s->geoms[g], s->nq);
    double Gk[3];
    kernel_grad(G, s->nq, Gk);
    return (int64_t)plan_fields(gh, Gk, s->scheme == BTL_CLASSICAL).sigma.size() * s->nq * gh.nsites;
}

extern "C" btl_status btl_forward(btl_sim* s, double dt, int32_t K, const double* D,
                                  const double* T2, const double* kappa, int32_t Q,
                                  const int32_t* q_geom, const double* gG0, const double* f,
                                  double* E, void* M_final, int32_t ckpt_every, void* stream) {
    if (!s) return BTL_E_INVAL;
    if (Q < 1 || !q_geom || !gG0) return forward_impl(s, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E,
                                                      M_final, ckpt_every, stream);
    for (int q = 0; q < Q; ++q)
        if (q_geom[q] < 0 || q_geom[q] >= (int)s->geoms.size())
            return fail(s, BTL_E_INVAL, "q_geom out of range");
    if (D && T2 && kappa && (K == 0 || f)) {
        const int32_t P = s->n_phase;
        s->last.valid = true;
        s->last.dt = dt;
        s->last.D.assign(D, D + P);
        s->last.T2.assign(T2, T2 + P);
        s->last.kappa.assign(kappa, kappa + P * P);
        s->last.gG0.assign(gG0, gG0 + 3 * Q);
        s->last.f.assign(f, f + (size_t)K * s->substeps);
        s->last.q_geom.assign(q_geom, q_geom + Q);
    }
    // q-waves: when the two population copies of all q-samples do not fit
    // in device memory, run consecutive subsets of the q-samples
    const size_t esz = s->prec == BTL_F32 ? sizeof(float2) : sizeof(double2);
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    const size_t have = free_b + s->pop[0].cap + s->pop[1].cap;
    double budget = 0.85 * (double)have;
    // BTLBM_MEM_BUDGET (bytes) lowers the budget, to exercise q-waves on
    // small problems
    if (const char* v = getenv("BTLBM_MEM_BUDGET")) budget = std::min(budget, atof(v));
    double need = 0.0;
    for (int q = 0; q < Q; ++q) need += 2.0 * (double)q_state_elems(s, q_geom[q], gG0 + 3 * q) * esz;
    if (need <= budget || ckpt_every > 0)
        return forward_impl(s, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E, M_final, ckpt_every,
                            stream);
    int32_t q0 = 0;
    int64_t m_off = 0;
    while (q0 < Q) {
        double acc = 0.0;
        int32_t q1 = q0;
        while (q1 < Q) {
            const double b = 2.0 * (double)q_state_elems(s, q_geom[q1], gG0 + 3 * q1) * esz;
            if (q1 > q0 && acc + b > budget) break;
            acc += b;
            ++q1;
        }
        if (acc > budget)
            return fail(s, BTL_E_NOMEM, "one q-sample does not fit in device memory");
        void* Mw = M_final ? static_cast<char*>(M_final) + m_off * esz : nullptr;
        const btl_status rc =
            forward_impl(s, dt, K, D, T2, kappa, q1 - q0, q_geom + q0, gG0 + 3 * q0, f,
                         E + (size_t)q0 * (K + 1) * 2, Mw, 0, stream);
        if (rc != BTL_OK) return rc;
        for (int q = q0; q < q1; ++q) m_off += s->geoms[q_geom[q]].nsites;
        q0 = q1;
    }
    return BTL_OK;
}

extern "C" btl_status btl_backward(btl_sim* s, const double* dL_dE, double* dD, double* dT2,
                                   double* dkappa, double* df, double* dgG0, void* stream) {
    if (!s) return BTL_E_INVAL;
    if (!s->tape.valid) return fail(s, BTL_E_INVAL, "no adjoint tape: run btl_forward with ckpt_every > 0");
    if (!dL_dE) return fail(s, BTL_E_INVAL, "dL_dE is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const btl_sim::Tape& tp = s->tape;
    const int32_t K = tp.K, C = tp.C, T = tp.T, P = s->n_phase, nf = tp.n_fields;
    if (dgG0 && !tp.g_ok)
        return fail(s, BTL_E_UNSUPPORTED,
                    "dgG0 needs btl_set_grad_gG0(s, 1) before the taped forward (a mirrored axis "
                    "without a gradient component, or the conjugate pairing next to a periodic "
                    "axis, has no image fields to differentiate)");
    const int NG = 2 * P + P * P + 2 + (dgG0 ? kNGGrad : 0);
    const size_t esz = s->prec == BTL_F32 ? sizeof(float2) : sizeof(double2);
    const size_t state_bytes = (size_t)tp.state_elems * esz;
    hipError_t e;
    const int32_t nblk_adj = tp.nblk_adj;
    if ((e = s->seg.ensure((size_t)C * state_bytes)) != hipSuccess ||
        (e = s->lam[0].ensure(state_bytes)) != hipSuccess ||
        (e = s->lam[1].ensure(state_bytes)) != hipSuccess ||
        (e = s->tab_b.ensure((size_t)(C + 1) * T)) != hipSuccess ||
        (e = s->gpart.ensure((size_t)C * nblk_adj * NG)) != hipSuccess ||
        (e = s->gfield.ensure((size_t)K * nf * NG)) != hipSuccess)
        return hip_fail(s, e, "allocating adjoint buffers");

    StepArgs fa;   // forward recompute
    memset(&fa, 0, sizeof(fa));
    fa.words = s->words.p;
    fa.fields = s->fields.p;
    fa.blk_field = s->blk_field.p;
    fa.fdt = s->steps.p;
    fa.Fk = s->steps.p + K;
    fa.w = s->consts.p;
    fa.decay = s->consts.p + P;
    fa.trans = s->consts.p + 2 * P;
    fa.partial = s->partial.p;
    fa.n_phase = P;
    fa.K = K;
    fa.tab_field = s->tab_field.p;
    fa.T = T;
    fa.nq = tp.nq;
    fa.xcd = tp.xcd;

    AdjArgs aa;
    memset(&aa, 0, sizeof(aa));
    aa.words = s->words.p;
    aa.fields = s->adj_fields.p;
    aa.blk_field = s->adj_blk.p;
    aa.w = s->consts.p;
    aa.decay = s->consts.p + P;
    aa.trans = s->consts.p + 2 * P;
    aa.dLdE = reinterpret_cast<const double2*>(dL_dE);
    aa.gpart = s->gpart.p;
    aa.dt = tp.dt;
    aa.xcd = nblk_adj > kXcdMinBlocks ? 1 : 0;
    aa.n_phase = P;
    aa.K = K;
    aa.ng = NG;
    aa.gradg = dgG0 ? 1 : 0;
    aa.nq = tp.nq;

    const int32_t nseg = (K + C - 1) / C;
    int lam_cur = 0;      // buffer holding Lambda^k on entry to adjoint step k
    for (int32_t m = nseg - 1; m >= 0; --m) {
        const int32_t k0 = m * C, k1 = std::min(K, k0 + C);
        // phase tables of steps k0 .. k1 (the last only when k1 < K)
        fa.k = k0;
        fa.tab = s->tab_b.p;
        if ((e = launch_tables(fa, (k1 - k0) + (k1 < K ? 1 : 0), st)) != hipSuccess)
            return hip_fail(s, e, "adjoint table launch");
        // recompute ghat^{k0+1} .. ghat^{k1-1} from the checkpoint
        const char* ck = s->ckpt.p + (size_t)m * state_bytes;
        if ((e = hipMemcpyAsync(s->seg.p, ck, state_bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return hip_fail(s, e, "segment copy");
        for (int32_t k = k0; k < k1 - 1; ++k) {
            fa.k = k;
            fa.tab = s->tab_b.p + (size_t)(k - k0) * T;
            fa.src = s->seg.p + (size_t)(k - k0) * state_bytes;
            fa.dst = s->seg.p + (size_t)(k - k0 + 1) * state_bytes;
            if ((e = launch_step(s->prec, tp.shape, fa, tp.nblk, st)) != hipSuccess)
                return hip_fail(s, e, "recompute launch");
        }
        // reverse sweep over the segment
        for (int32_t k = k1; k > k0; --k) {
            aa.k = k;
            aa.top = (k == K) ? 1 : 0;
            aa.lam_in = aa.top ? nullptr : s->lam[lam_cur].p;
            aa.lam_out = s->lam[lam_cur ^ 1].p;
            aa.fwd = s->seg.p + (size_t)(k - 1 - k0) * state_bytes;
            aa.tab_prev = s->tab_b.p + (size_t)(k - 1 - k0) * T;
            aa.tab_cur = aa.top ? aa.tab_prev : s->tab_b.p + (size_t)(k - k0) * T;
            aa.slot = k - 1 - k0;
            if ((e = launch_adj(s->prec, tp.shape, aa, nblk_adj, st)) != hipSuccess)
                return hip_fail(s, e, "adjoint launch");
            lam_cur ^= 1;
        }
        // per-step, per-field sums of this segment: gfield[k0 .. k1 - 1]
        if ((e = launch_adj_gsum(s->gpart.p, s->adj_fields.p, nf, nblk_adj, NG, k0, k1 - k0,
                                 s->gfield.p, st)) != hipSuccess)
            return hip_fail(s, e, "adjoint sum launch");
    }
    if ((e = launch_adj_final(s->gfield.p, K, nf, P, tp.dt, s->dx, s->consts.p,
                              s->consts.p + 2 * P + P * P, s->consts.p + 3 * P + P * P, dD, dT2,
                              dkappa, df, tp.sub, NG, s->adj_gmeta.p, s->steps.p,
                              s->steps.p + K, tp.Q, dgG0, lattice_eps(tp.nq),
                              tp.nq == 5 ? 1 : 0, st)) != hipSuccess)
        return hip_fail(s, e, "adjoint final launch");
    return BTL_OK;
}

extern "C" btl_status btl_autotune(btl_sim* s, int32_t Q, int32_t K_probe, void* stream) {
    if (!s) return BTL_E_INVAL;
    // fixed launch shape for measurements: BTLBM_TILE (0..5, see TileShape), BTLBM_ZC,
    // BTLBM_XCD (0 plain, 1 XCD-contiguous workgroup order); BTLBM_VERBOSE
    // prints the choice
    const char* et = getenv("BTLBM_TILE");
    const char* ez = getenv("BTLBM_ZC");
    const char* ex = getenv("BTLBM_XCD");
    if (ex) s->xcd = atoi(ex) ? 1 : 0;
    if (et || ez) {
        if (et) s->tile_shape = std::max(0, std::min(kTileCount - 1, atoi(et)));
        if (s->nq == 5) s->tile_shape = kTile256x1;
        else if (s->tile_shape == kTile256x1) s->tile_shape = kTile128x2;
        if (ez) s->zc = std::max(0, std::min(kMaxZc, atoi(ez)));
        return BTL_OK;
    }
    if (!s->last.valid) return fail(s, BTL_E_INVAL, "btl_autotune replays the last btl_forward: call it first");
    if (K_probe < 1) return fail(s, BTL_E_INVAL, "K_probe must be >= 1");
    const btl_sim::SimLast& L = s->last;
    const int32_t Qr = std::min<int32_t>(Q > 0 ? Q : (int32_t)L.q_geom.size(), (int32_t)L.q_geom.size());
    std::vector<double> f((size_t)K_probe * s->substeps);
    for (size_t k = 0; k < f.size(); ++k) f[k] = L.f.empty() ? 1.0 : L.f[k % L.f.size()];
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = s->tune_E.ensure((size_t)Qr * (K_probe + 1) * 2)) != hipSuccess)
        return hip_fail(s, e, "autotune buffer");
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        return hip_fail(s, e, "autotune events");
    int nz_max = 1;
    for (int q = 0; q < Qr; ++q)
        nz_max = std::max(nz_max, kernel_geom(s->geoms[L.q_geom[q]], s->nq).n[2]);
    // z-column lengths: whole columns, halves, thirds, quarters, and short
    // columns for small lattices that need more workgroups
    std::vector<int> zcs = {0};
    for (int div : {2, 3, 4}) zcs.push_back((nz_max + div - 1) / div);
    for (int z : {1, 2, 4, 8, 16}) zcs.push_back(z);
    std::sort(zcs.begin(), zcs.end());
    zcs.erase(std::unique(zcs.begin(), zcs.end()), zcs.end());
    zcs.erase(std::remove_if(zcs.begin(), zcs.end(), [&](int z) { return z >= nz_max; }), zcs.end());
    const btl_sim::SimLast saved = L;
    // one warm forward of the probe in the current launch configuration,
    // then the fastest of kTuneReps timed ones (single timings of a few
    // milliseconds are noisy at the percent level)
    constexpr int kTuneReps = 3;
    // a candidate whose first timing is kTuneCut times the best so far is not
    // timed again: it cannot win by noise, and most candidates are like that
    constexpr float kTuneCut = 1.15f;
    float best = -1.0f;
    auto time_probe = [&](float* best_ms) -> btl_status {
        *best_ms = -1.0f;
        for (int r = 0; r <= kTuneReps; ++r) {
            if (r > 1 && best > 0.0f && *best_ms > kTuneCut * best) break;
            if (r > 0) (void)hipEventRecord(e0, st);
            const btl_status rr = btl_forward(s, saved.dt, K_probe, saved.D.data(), saved.T2.data(),
                                              saved.kappa.data(), Qr, saved.q_geom.data(),
                                              saved.gG0.data(), f.data(), s->tune_E.p, nullptr, 0,
                                              stream);
            if (rr != BTL_OK) return rr;
            if (r == 0) continue;
            (void)hipEventRecord(e1, st);
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(s, e, "autotune timing");
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (*best_ms < 0.0f || ms < *best_ms) *best_ms = ms;
        }
        return BTL_OK;
    };
    int best_shape = -1, best_zc = 0, best_xcd = 0;
    btl_status rc = BTL_OK;
    std::vector<int> shapes;
    if (s->nq == 5)
        shapes.push_back(kTile256x1);
    else
        shapes.assign(kShapes3D, kShapes3D + kShapeCount3D);
    // shape, z-column length and workgroup order are searched jointly: the
    // best column length differs between the two orders
    for (int sh : shapes) {
        for (int zc : zcs) {
            for (int xo = 0; xo < 2 && rc == BTL_OK; ++xo) {
                s->tile_shape = sh;
                s->zc = zc;
                s->xcd = xo;
                float ms = 0.0f;
                if ((rc = time_probe(&ms)) != BTL_OK) break;
                if (best < 0.0f || ms < best) {
                    best = ms;
                    best_shape = sh;
                    best_zc = zc;
                    best_xcd = xo;
                }
            }
            if (rc != BTL_OK) break;
        }
        if (rc != BTL_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->last = saved;
    if (rc != BTL_OK) {
        s->tile_shape = -1;
        s->zc = 0;
        s->xcd = -1;
        return rc;
    }
    s->tile_shape = best_shape;
    s->zc = best_zc;
    s->xcd = best_xcd;
    if (getenv("BTLBM_VERBOSE"))
        fprintf(stderr, "btlbm autotune: tile shape %d, z-column %d, xcd order %d (%.3f ms per probe)\n",
                best_shape, best_zc, best_xcd, best);
    return BTL_OK;
}

extern "C" btl_status btl_get_launch(const btl_sim* s, int32_t* tile_shape, int32_t* zc,
                                     int32_t* xcd) {
    if (!s || !tile_shape || !zc || !xcd) return BTL_E_INVAL;
    *tile_shape = s->tile_shape;
    *zc = s->zc;
    *xcd = s->xcd;
    return BTL_OK;
}

extern "C" btl_status btl_set_lattice(btl_sim* s, int32_t lattice) {
    if (!s) return BTL_E_INVAL;
    if (lattice != BTL_D3Q7 && lattice != BTL_D2Q5)
        return fail(s, BTL_E_INVAL, "lattice must be BTL_D3Q7 or BTL_D2Q5");
    s->nq = lattice == BTL_D2Q5 ? 5 : 7;
    s->tape.valid = false;
    s->last.valid = false;
    return BTL_OK;
}

extern "C" btl_status btl_set_grad_gG0(btl_sim* s, int32_t on) {
    if (!s) return BTL_E_INVAL;
    if (on != 0 && on != 1) return fail(s, BTL_E_INVAL, "btl_set_grad_gG0 takes 0 or 1");
    s->grad_g = on;
    return BTL_OK;
}

extern "C" btl_status btl_set_substeps(btl_sim* s, int32_t m) {
    if (!s) return BTL_E_INVAL;
    if (m < 1 || m > 65536) return fail(s, BTL_E_INVAL, "substeps must be in 1..65536");
    s->substeps = m;
    s->last.valid = false;
    return BTL_OK;
}

extern "C" btl_status btl_set_scheme(btl_sim* s, int32_t scheme) {
    if (!s) return BTL_E_INVAL;
    if (scheme != BTL_HYBRID && scheme != BTL_CLASSICAL)
        return fail(s, BTL_E_INVAL, "scheme must be BTL_HYBRID or BTL_CLASSICAL");
    s->scheme = scheme;
    s->tape.valid = false;
    return BTL_OK;
}

extern "C" void btl_destroy(btl_sim* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    s->words.release();
    s->gm.release();
    s->pop[0].release();
    s->pop[1].release();
    s->fields.release();
    s->blk_field.release();
    s->adj_fields.release();
    s->adj_blk.release();
    s->adj_gmeta.release();
    s->steps.release();
    s->consts.release();
    s->partial.release();
    s->tune_E.release();
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    s->E_int.release();
    s->ckpt.release();
    s->seg.release();
    s->lam[0].release();
    s->lam[1].release();
    s->tab_b.release();
    s->gpart.release();
    s->gfield.release();
    s->tab.release();
    s->tab_field.release();
    for (int i = 0; i < 2; ++i) {
        if (s->stage[i]) (void)hipHostFree(s->stage[i]);
        if (s->stage_ev[i]) (void)hipEventDestroy(s->stage_ev[i]);
    }
    delete s;
}

extern "C" const char* btl_last_error(const btl_sim* s) {
    return s ? s->err.c_str() : g_create_error.c_str();
}
