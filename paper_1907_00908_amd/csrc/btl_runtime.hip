// Host runtime and C ABI of libbtlbm (declared in include/btlbm.h).
//
// The runtime validates inputs, turns the per-phase material parameters into
// the FP64 constants of one step (1/tau, T2 decay, membrane transmission),
// builds the field table (one field per q-sample plus reflected image fields
// where a mirrored face sees an oblique gradient), and enqueues one step
// launch per time step on the caller's stream.
//
// A call is first planned on the host (CallPlan: field and workgroup tables,
// per-step waveform sums, constants), then given device buffers (CallBufs:
// the simulator's own allocations, or the fixed device scratch of
// btl_forward_noalloc), then its tables are uploaded and its launches
// enqueued.  Reverse sweeps that do not fit a uniform checkpoint tape replay
// the forward from t = 0 per group of q-samples with a binomial
// checkpointing schedule (plan_reversal).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/btlbm.h"
#include "btl_curved.h"
#include "btl_internal.h"

using namespace btl;

// Device scratch of btl_forward_noalloc, for callers that cannot allocate:
// populations, signal partials, phase tables and the call's small tables all
// live here.  Each device holds its own copy for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress returns
// for that device (scratch_address), never through the array's name.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device (looked up once per device).
hipError_t scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

struct GeomHost {
    int32_t n[3];
    int32_t bc[3];
    int64_t nsites;
    int64_t words_off;   // offset into the concatenated site-word array
    int64_t gm_off = -1; // offset into the membrane-position tables, -1: none
    int64_t cv_off = -1; // offset into the curved-link index tables, -1: none
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
    size_t bytes() const { return cap * sizeof(T); }
};

std::string g_create_error;

constexpr int kGraphMinSteps = 16;   // forwards this long run from a cached hipGraph
constexpr int kGraphSlots = 4;       // cached forward graphs per simulator
constexpr int kXcdMinBlocks = 2048;  // grids above this use the XCD-contiguous order
constexpr size_t kStageInit = (size_t)1 << 20;   // pinned staging per slot at creation

// Everything a captured forward depends on besides the contents of its
// buffers; a forward replays a cached graph only when this matches.
struct GraphKey {
    int32_t prec, K, Q, n_fields, nblk, shape, T, ckpt, scheme, nq, xcd;
    uint64_t fields;     // hash of the per-field values the launches take by value
    const void* ptr[20];
};

struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    GraphKey key;
    uint64_t used = 0;   // last use (least recently used slot is replaced)
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
        mix(&d.cv, sizeof(d.cv));
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

// Settings that shape a call besides its arguments (the btl_set_* calls and
// the autotuner's choice).  A taped forward keeps a copy, so that a reverse
// sweep replays it exactly.
struct Settings {
    int scheme = BTL_HYBRID;
    int msub = 1;          // reaction sub-steps per step
    int nq = 7;            // 7 (D3Q7) or 5 (D2Q5 on single-layer geometries)
    int grad_g = 0;        // taped forwards plan the full field set (gamma G0 gradient)
    int tile_shape = -1;   // forward launch: -1 chosen per call
    int zc = 0;            //   sites per thread along z, 0 whole columns
    int xcd = -1;          //   workgroup order, -1 by grid size
    int adj_zc = -1;       // adjoint launch: -1 automatic, 0 whole columns, > 0 sites
    int adj_xcd = -1;      //   workgroup order, -1 by grid size
};

// Autotuner results of this process, by device and workload shape: a later
// simulator with the same shape takes the launch without timing it again.
struct TuneEntry {
    std::string key;
    int shape, zc, xcd;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune_cache;

}  // namespace

struct btl_sim {
    int prec = BTL_F32;
    Settings set;
    int use_graphs = 1;          // forwards of >= kGraphMinSteps steps replay cached graphs
    int64_t mem_limit = 0;       // btl_set_memory_budget (0: none)
    int device = 0;
    double dx = 1.0;
    int32_t n_phase = 1;
    std::vector<GeomHost> geoms;
    DevBuf<uint32_t> words;
    DevBuf<float> gm;            // [6][nsites] per geometry with membrane positions
    // membranes at an angle (link_normal): the membrane links of each such
    // geometry, and the term tables of the constants in cv_key
    std::vector<CurvedGeom> curved;
    DevBuf<uint8_t> cvm;         // [nsites] per curved geometry: its curved links (bit d-1)
    DevBuf<int4> cvh;            // (first term, count, site element, direction) per link
    DevBuf<CvTerm> cvt;
    std::vector<double> cv_key;  // (lattice, dt, kappa) the tables hold, empty: none
    size_t cvm_elems = 0;
    int32_t cv_max_links = 0;    // most membrane links of one curved geometry (k_links grid)
    DevBuf<char> pop[2];
    DevBuf<FieldDesc> fields;
    DevBuf<int2> blk_field;
    DevBuf<double> steps;        // fdt [K] then Fk [K+1]
    DevBuf<double> consts;       // w [P], decay [P], trans [P*P], T2 [P], kappa [P*P], dt/T2 [P], kappa dt [P*P]
    DevBuf<double2> partial;     // per-wave signal partials of kTabSteps steps
    DevBuf<double2> tab;         // [kTabSteps][T] per-step phase tables
    DevBuf<int32_t> tab_field;   // [T]
    // launch geometry of the adjoint steps (the forward's tile shape with
    // its own z-column length)
    DevBuf<FieldDesc> adj_fields;
    DevBuf<int2> adj_blk;
    DevBuf<double> adj_gmeta;    // [fields][kGMeta] for the gamma G0 gradient
    // pinned staging for the per-call tables, two slots so that a call can
    // be prepared while the previous one's uploads are still queued
    char* stage[2] = {nullptr, nullptr};
    size_t stage_cap[2] = {0, 0};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_used[2] = {false, false};
    int stage_slot = 0;
    // non-finite report: host-visible flag the signal and gradient kernels set
    int32_t* nf_host = nullptr;
    int32_t* nf_dev = nullptr;
    char* scratch = nullptr;     // this device's copy of `scratch`
    // cached forward graphs
    GraphSlot graphs[kGraphSlots];
    uint64_t graph_clock = 0;
    hipStream_t cap_stream = nullptr;
    DevBuf<double> E_int;
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
        bool deferred = false;     // no states kept: btl_backward replays from t = 0
        Settings set;              // settings of the taped forward
        int32_t K = 0, C = 0, Q = 0, T = 0, n_fields = 0, nblk = 0, shape = 0, sub = 1, xcd = 0;
        int32_t nblk_adj = 0;      // workgroups of one adjoint step (adj_fields)
        int32_t nq = 7;            // lattice of the taped forward
        bool g_ok = false;         // the field set supports the gamma G0 gradient
        double dt = 0;
        int64_t state_elems = 0;   // V elements of one full state (all fields)
        // inputs of a deferred tape
        std::vector<double> D, T2, kappa, gG0, f;
        std::vector<int32_t> q_geom;
    } tape;
    DevBuf<char> ckpt;             // uniform tape: [ceil(K/C)] states ghat^{mC}; deferred: snapshots
    DevBuf<char> seg;              // [C] states of the segment being reversed
    DevBuf<char> lam[2];
    DevBuf<double2> tab_b;         // phase tables of a segment
    DevBuf<double> gpart;
    DevBuf<double> gfield;
    // statistics of the last reverse sweep (btl_get_backward_stats)
    int64_t stat_fwd_steps = 0;    // forward steps run by the reverse sweep
    int32_t stat_waves = 0;        // groups of q-samples reversed one after another
    int32_t stat_snapshots = 0;    // states kept per group (binomial schedule), 0: uniform tape
    // events around each segment's run of adjoint steps (uniform tape), read
    // by btl_get_backward_timing; created on first use and reused
    std::vector<hipEvent_t> tev;
    int32_t tev_used = 0;          // events recorded by the last backward (pairs)
    int32_t tev_steps = 0;         // adjoint steps they bracket
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
        if (geoms[g].link_normal && !geoms[g].link_delta) {
            btl_destroy(s);
            return fail(nullptr, BTL_E_INVAL, "link_normal needs link_delta");
        }
        if (geoms[g].link_delta) {
            if (!build_gm(geoms[g], gm_one)) {
                btl_destroy(s);
                return fail(nullptr, BTL_E_INVAL, "link_delta must be in (0, 1) on membrane links");
            }
            h.gm_off = (int64_t)gm_all.size();
            gm_all.insert(gm_all.end(), gm_one.begin(), gm_one.end());
        }
        if (geoms[g].link_normal) {
            CurvedGeom cg;
            if (!curved_collect(geoms[g], cg)) {
                btl_destroy(s);
                return fail(nullptr, BTL_E_INVAL,
                            "link_normal must be a finite non-zero vector on membrane links");
            }
            h.cv_off = cg.cv_off = (int64_t)s->cvm_elems;
            s->cvm_elems += (size_t)h.nsites;
            s->cv_max_links = std::max<int32_t>(s->cv_max_links, (int32_t)cg.links.size());
            s->curved.push_back(std::move(cg));
        }
        s->geoms.push_back(h);
    }
    const char* what = "uploading site words";
    hipError_t e = s->words.ensure(all.size());
    if (e == hipSuccess)
        e = hipMemcpy(s->words.p, all.data(), all.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !gm_all.empty()) {
        e = s->gm.ensure(gm_all.size());
        if (e == hipSuccess)
            e = hipMemcpy(s->gm.p, gm_all.data(), gm_all.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    // set-up that later calls rely on without allocating: the non-finite
    // flag (pinned, mapped into the device's address space), the pinned
    // staging slots and their events, and this device's scratch address
    if (e == hipSuccess) {
        what = "allocating the non-finite flag";
        e = hipHostMalloc((void**)&s->nf_host, sizeof(int32_t),
                          hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess) {
            *s->nf_host = 0;
            e = hipHostGetDevicePointer((void**)&s->nf_dev, s->nf_host, 0);
        }
    }
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        what = "allocating pinned staging";
        e = hipHostMalloc((void**)&s->stage[i], kStageInit, hipHostMallocDefault);
        if (e == hipSuccess) {
            s->stage_cap[i] = kStageInit;
            e = hipEventCreateWithFlags(&s->stage_ev[i], hipEventDisableTiming);
        }
    }
    if (e == hipSuccess) {
        what = "looking up the device scratch";
        void* p = nullptr;
        e = scratch_address(s->device, &p);
        s->scratch = static_cast<char*>(p);
    }
    if (e != hipSuccess) {
        btl_status st = hip_fail(nullptr, e, what);
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


// Everything a call computes on the host before touching the device.
struct CallPlan {
    int32_t K = 0, Q = 0, P = 0, nq = 7, msub = 1;
    double dt = 0.0;
    bool classical = false, uses_gm = false, uses_cv = false, taping = false, g_complete = true;
    int shape = 0, xcd_on = 0, order = 0;   // order: 2 = fields interleaved per block
    int32_t n_fields = 0, nblk_total = 0, nblk_adj = 0, T = 0;
    int64_t pop_elems = 0;       // V elements of one state (all fields of the call)
    std::vector<double> consts, steps, gmeta;
    std::vector<FieldDesc> fl, afl;
    std::vector<int2> blk, ablk;
    std::vector<int32_t> tabf;
};

// Checks of a forward's arguments that need no device call.
static btl_status validate_inputs(btl_sim* s, const Settings& cs, double dt, int32_t K,
                                  const double* D, const double* T2, const double* kappa,
                                  int32_t Q, const int32_t* q_geom, const double* gG0,
                                  const double* f, const double* E) {
    if (!(dt > 0) || !isfinite(dt)) return fail(s, BTL_E_INVAL, "dt must be finite and > 0");
    if (K < 0) return fail(s, BTL_E_INVAL, "K must be >= 0");
    if (Q < 1) return fail(s, BTL_E_INVAL, "Q must be >= 1");
    if (!D || !T2 || !kappa || !q_geom || !gG0 || (K > 0 && !f) || !E)
        return fail(s, BTL_E_INVAL, "NULL argument");
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
    for (int q = 0; q < Q; ++q) {
        if (q_geom[q] < 0 || q_geom[q] >= (int)s->geoms.size())
            return fail(s, BTL_E_INVAL, "q_geom out of range");
        for (int a = 0; a < 3; ++a)
            if (!isfinite(gG0[3 * q + a])) return fail(s, BTL_E_INVAL, "gG0 must be finite");
    }
    if (cs.nq == 5)
        for (int q = 0; q < Q; ++q)
            if (s->geoms[q_geom[q]].n[2] != 1 || gG0[3 * q + 2] != 0.0)
                return fail(s, BTL_E_INVAL, "D2Q5 needs single-layer geometries (n[2] = 1) "
                                             "and no gradient along z");
    if (cs.msub > 1 && cs.scheme == BTL_CLASSICAL)
        return fail(s, BTL_E_UNSUPPORTED, "reaction sub-steps need the hybrid scheme");
    for (int64_t k = 0; k < (int64_t)K * cs.msub; ++k)
        if (!isfinite(f[k])) return fail(s, BTL_E_INVAL, "f must be finite");
    return BTL_OK;
}

// The adjoint covers the hybrid scheme with half-link membranes and at most
// kAdjMaxPhase phases.
static btl_status adjoint_supported(btl_sim* s, const Settings& cs, int32_t Q,
                                    const int32_t* q_geom) {
    if (s->n_phase > kAdjMaxPhase) return fail(s, BTL_E_UNSUPPORTED, "the adjoint supports n_phase <= 4");
    if (cs.scheme == BTL_CLASSICAL)
        return fail(s, BTL_E_UNSUPPORTED, "the adjoint supports the hybrid scheme only");
    for (int q = 0; q < Q; ++q)
        if (s->geoms[q_geom[q]].gm_off >= 0)
            return fail(s, BTL_E_UNSUPPORTED, "the adjoint supports the half-link membrane rule only");
    return BTL_OK;
}

// Plan one call (validated inputs): per-phase constants, waveform sums,
// launch shape, field table (with image fields and face couplings), phase
// table layout, workgroup tables and, when taping, the adjoint's launch
// geometry and the gamma G0 metadata.
static btl_status make_plan(btl_sim* s, const Settings& cs, double dt, int32_t K,
                            const double* D, const double* T2, const double* kappa, int32_t Q,
                            const int32_t* q_geom, const double* gG0, const double* f,
                            bool taping, CallPlan& p) {
    const int32_t P = s->n_phase;
    const int32_t msub = cs.msub;
    const int32_t nq = cs.nq;
    const double eps = lattice_eps(nq);
    const double dx = s->dx;
    p = CallPlan();
    p.K = K;
    p.Q = Q;
    p.P = P;
    p.nq = nq;
    p.msub = msub;
    p.dt = dt;
    p.classical = cs.scheme == BTL_CLASSICAL;
    p.taping = taping && K > 0;

    // per-phase and per-pair constants (FP64)
    std::vector<double>& consts = p.consts;
    consts.assign(2 * P + P * P + P + P * P + P + P * P, 0.0);
    for (int ph = 0; ph < P; ++ph) {
        const double tau = 0.5 + dt * D[ph] / (eps * dx * dx);
        consts[ph] = 1.0 / tau;
        consts[P + ph] = isinf(T2[ph]) ? 1.0 : exp(-dt / T2[ph]);
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
    for (int ph = 0; ph < P; ++ph) consts[2 * P + P * P + ph] = T2[ph];
    for (int i = 0; i < P * P; ++i) consts[3 * P + P * P + i] = kappa[i];
    for (int ph = 0; ph < P; ++ph) consts[3 * P + 2 * P * P + ph] = isinf(T2[ph]) ? 0.0 : dt / T2[ph];
    for (int i = 0; i < P * P; ++i) consts[4 * P + 2 * P * P + i] = kappa[i] * dt;
    for (int q = 0; q < Q; ++q) {
        p.uses_gm |= s->geoms[q_geom[q]].gm_off >= 0;
        p.uses_cv |= s->geoms[q_geom[q]].cv_off >= 0;
    }
    // per-step waveform tables: f_k dt and F_k.  With m reaction sub-steps
    // of dt' = dt/m (Sec. 2.3) the reaction of step k is the product of m
    // exact phase factors, i.e. one factor with the summed angle, so f_k dt
    // becomes sum_j f[k m + j] dt'.
    std::vector<double>& steps = p.steps;
    steps.assign((size_t)K + (size_t)K + 1, 0.0);
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
    int shape = cs.tile_shape >= 0 ? cs.tile_shape : pick_shape(s->geoms, q_geom, Q, nq);
    if ((nq == 5) != (shape == kTile256x1)) shape = pick_shape(s->geoms, q_geom, Q, nq);
    p.shape = shape;
    int ZC = cs.zc;
    if (ZC <= 0) {
        ZC = 1;
        for (int q = 0; q < Q; ++q) ZC = std::max(ZC, kernel_geom(s->geoms[q_geom[q]], nq).n[2]);
    }
    ZC = std::min(ZC, kMaxZc);

    // field table
    std::vector<FieldDesc>& fl = p.fl;
    std::vector<double>& gmeta = p.gmeta;   // per field: q-sample, s_b, sigma_b, d beta_f / d G_b
    int64_t pop_elems = 0;
    int32_t nblk_total = 0;
    for (int q = 0; q < Q; ++q) {
        const GeomHost g = kernel_geom(s->geoms[q_geom[q]], nq);
        double G[3];
        kernel_grad(gG0 + 3 * q, nq, G);
        const bool full = cs.grad_g && p.taping;
        QFields qf = plan_fields(g, G, p.classical, full);
        {
            const QFields qa = plan_fields(g, G, p.classical, true);
            if (!(qa.amask == qf.amask && qa.conj_pair == qf.conj_pair && qa.sigma == qf.sigma))
                p.g_complete = false;
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
            d.cv = g.cv_off;
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
            for (int fc = 0; fc < 6; ++fc) {
                if ((d.face_kind[fc] & kFaceMirror) == 0) {
                    d.adj_kind[fc] = kFacePeriodic;
                    d.adj_pop[fc] = d.pop;
                    d.adj_fac[fc] = -1 - (fc ^ 1);          // own table, resolved below
                } else {
                    int partner = -1;
                    for (size_t pj = 0; pj < qf.sigma.size(); ++pj)
                        if (fl[base + pj].pop == d.face_pop[fc]) partner = base + (int)pj;
                    d.adj_kind[fc] = fl[partner].face_kind[fc];
                    d.adj_pop[fc] = fl[partner].pop;
                    d.adj_fac[fc] = -1000 - (partner * 6 + fc);  // partner table, resolved below
                }
            }
        }
    }
    const int32_t n_fields = (int32_t)fl.size();
    // the kernels address a field's reads with 32-bit element offsets from
    // its own base: every plane it reads must lie within +-2^31 elements
    for (int i = 0; i < n_fields; ++i) {
        int64_t lo = 0, hi = (int64_t)nq * fl[i].nsites;
        for (int fc = 0; fc < 6; ++fc) {
            lo = std::min(lo, fl[i].face_pop[fc] - fl[i].pop);
            hi = std::max(hi, fl[i].face_pop[fc] - fl[i].pop + (int64_t)nq * fl[i].nsites);
            lo = std::min(lo, fl[i].adj_pop[fc] - fl[i].pop);
            hi = std::max(hi, fl[i].adj_pop[fc] - fl[i].pop + (int64_t)nq * fl[i].nsites);
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
        for (int fc = 0; fc < 6; ++fc) {
            const int32_t v = fl[i].adj_fac[fc];
            if (v <= -1000) {
                const int partner = (-1000 - v) / 6, pf = (-1000 - v) % 6;
                fl[i].adj_fac[fc] = fl[partner].tab + fl[partner].n[0] + fl[partner].n[1] +
                                    fl[partner].n[2] + pf;
            } else {
                fl[i].adj_fac[fc] = fl[i].tab + fl[i].n[0] + fl[i].n[1] + fl[i].n[2] + (-1 - v);
            }
        }
    p.tabf.assign(T, 0);
    for (int i = 0; i < n_fields; ++i)
        for (int e = 0; e < fl[i].n[0] + fl[i].n[1] + fl[i].n[2] + 6; ++e) p.tabf[fl[i].tab + e] = i;
    // workgroup order: field after field, or (order bit 1) the fields that
    // share a geometry and grid interleaved block by block, so that the
    // workgroups running together read one block's geometry tables (site
    // words, membrane positions and term lists, the same for every field of
    // the geometry) once instead of once per field
    const int32_t order = cs.xcd >= 0 ? cs.xcd : 0;
    p.order = order & 2;
    p.blk.clear();
    p.blk.reserve(nblk_total);
    if (order & 2) {
        std::vector<bool> done(n_fields, false);
        for (int i = 0; i < n_fields; ++i) {
            if (done[i]) continue;
            std::vector<int> grp;
            for (int j = i; j < n_fields; ++j)
                if (!done[j] && fl[j].words == fl[i].words && fl[j].nblk == fl[i].nblk &&
                    fl[j].tiles[0] == fl[i].tiles[0] && fl[j].tiles[1] == fl[i].tiles[1]) {
                    grp.push_back(j);
                    done[j] = true;
                }
            for (int b = 0; b < fl[i].nblk; ++b)
                for (int j : grp) p.blk.push_back(make_int2(j, b));
        }
    } else {
        for (int i = 0; i < n_fields; ++i)
            for (int b = 0; b < fl[i].nblk; ++b) p.blk.push_back(make_int2(i, b));
    }
    // With a tape, the launch geometry of the adjoint steps: the same tile
    // shape, whole z columns when all workgroups are resident at once (cut
    // into as many pieces as still fit at once when that leaves SIMDs with
    // room), otherwise columns cut so that the grid runs in about eight rounds
    // (btl_set_adjoint_launch fixes the length).  The adjoint carries four
    // values along the column and loads in two phases per site; on the
    // two-phase axon workload (128^3) it measured faster on whole columns
    // than on the short chunks the forward step often prefers, but a grid
    // slightly larger than one round of resident workgroups leaves most of
    // the chip idle in its second.
    if (p.taping) {
        int zc_adj = cs.adj_zc >= 0 ? cs.adj_zc : 0;
        if (cs.adj_zc < 0) {
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
        p.afl = fl;
        int32_t nblk_adj = 0;
        for (FieldDesc& d : p.afl) {
            const int32_t zc = zc_adj > 0 ? std::min(zc_adj, d.n[2]) : d.n[2];
            d.zc = zc;
            d.tiles[2] = (d.n[2] + zc - 1) / zc;
            d.nblk = d.tiles[0] * d.tiles[1] * d.tiles[2];
            d.blk0 = nblk_adj;
            nblk_adj += d.nblk;
        }
        p.ablk.clear();
        p.ablk.reserve(nblk_adj);
        for (int i = 0; i < n_fields; ++i)
            for (int b = 0; b < p.afl[i].nblk; ++b) p.ablk.push_back(make_int2(i, b));
        p.nblk_adj = nblk_adj;
    }
    p.n_fields = n_fields;
    p.nblk_total = nblk_total;
    p.T = T;
    p.pop_elems = pop_elems;
    // XCD-contiguous workgroup order pays off when the grid runs in several
    // waves (tiles that share edge rows then meet in one XCD's L2); grids
    // that fit on the chip at once keep the plain order.  The autotuner
    // measures both.
    p.xcd_on = cs.xcd >= 0 ? (cs.xcd & 1) : (nblk_total > kXcdMinBlocks ? 1 : 0);
    return BTL_OK;
}

static size_t state_elem_bytes(const btl_sim* s) {
    return s->prec == BTL_F32 ? sizeof(float2) : sizeof(double2);
}

// Elements of one state of a q-sample: 2^(k-1) or 2^k image fields (see
// plan_fields; full: the field set of a tape that supports the gamma G0
// gradient).
static int64_t q_state_elems(const btl_sim* s, const Settings& cs, int32_t g, const double* G,
                             bool full) {
    const GeomHost gh = kernel_geom(s->geoms[g], cs.nq);
    double Gk[3];
    kernel_grad(G, cs.nq, Gk);
    return (int64_t)plan_fields(gh, Gk, cs.scheme == BTL_CLASSICAL, full).sigma.size() * cs.nq *
           gh.nsites;
}

// Device bytes the population state of a call may take: 85 % of what the
// device has free plus what this simulator already holds for states, or the
// caller's limit (btl_set_memory_budget) when lower.
static double memory_budget(const btl_sim* s) {
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    const size_t held = s->pop[0].bytes() + s->pop[1].bytes() + s->ckpt.bytes() + s->seg.bytes() +
                        s->lam[0].bytes() + s->lam[1].bytes();
    double b = 0.85 * (double)(free_b + held);
    if (s->mem_limit > 0) b = std::min(b, (double)s->mem_limit);
    return b;
}

// Device buffers of one call.
struct CallBufs {
    char* pop[2] = {nullptr, nullptr};
    FieldDesc* fields = nullptr;
    int2* blk = nullptr;
    double* steps = nullptr;
    double* consts = nullptr;
    double2* partial = nullptr;
    double2* tab = nullptr;
    int32_t* tabf = nullptr;
    FieldDesc* afields = nullptr;
    int2* ablk = nullptr;
    double* agmeta = nullptr;
};

// The simulator's own buffers, grown to the plan's sizes.
static btl_status alloc_bufs(btl_sim* s, const CallPlan& p, CallBufs& b) {
    const size_t esz = state_elem_bytes(s);
    hipError_t e;
    if ((e = s->pop[0].ensure((size_t)p.pop_elems * esz)) != hipSuccess ||
        (e = s->pop[1].ensure((size_t)p.pop_elems * esz)) != hipSuccess)
        return hip_fail(s, e, "allocating populations");
    if ((e = s->fields.ensure(p.n_fields)) != hipSuccess ||
        (e = s->blk_field.ensure(p.nblk_total)) != hipSuccess ||
        (e = s->steps.ensure(p.steps.size())) != hipSuccess ||
        (e = s->consts.ensure(p.consts.size())) != hipSuccess ||
        (e = s->partial.ensure((size_t)kTabSteps * p.nblk_total * (kBlock / 64))) != hipSuccess ||
        (e = s->tab.ensure((size_t)kTabSteps * p.T)) != hipSuccess ||
        (e = s->tab_field.ensure(p.T)) != hipSuccess ||
        (p.taping && ((e = s->adj_fields.ensure(p.n_fields)) != hipSuccess ||
                      (e = s->adj_blk.ensure(p.nblk_adj)) != hipSuccess ||
                      (e = s->adj_gmeta.ensure((size_t)p.n_fields * kGMeta)) != hipSuccess)))
        return hip_fail(s, e, "allocating tables");
    b.pop[0] = s->pop[0].p;
    b.pop[1] = s->pop[1].p;
    b.fields = s->fields.p;
    b.blk = s->blk_field.p;
    b.steps = s->steps.p;
    b.consts = s->consts.p;
    b.partial = s->partial.p;
    b.tab = s->tab.p;
    b.tabf = s->tab_field.p;
    b.afields = s->adj_fields.p;
    b.ablk = s->adj_blk.p;
    b.agmeta = s->adj_gmeta.p;
    return BTL_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Bytes of device scratch a call without tape takes (populations first).
static size_t scratch_need(const btl_sim* s, const CallPlan& p) {
    const size_t esz = state_elem_bytes(s);
    return 2 * align256((size_t)p.pop_elems * esz) + align256(p.n_fields * sizeof(FieldDesc)) +
           align256(p.nblk_total * sizeof(int2)) + align256(p.steps.size() * sizeof(double)) +
           align256(p.consts.size() * sizeof(double)) +
           align256((size_t)kTabSteps * p.nblk_total * (kBlock / 64) * sizeof(double2)) +
           align256((size_t)kTabSteps * p.T * sizeof(double2)) + align256(p.T * sizeof(int32_t));
}

// Buffers of a call carved out of this device's scratch (no allocation).
static btl_status scratch_bufs(btl_sim* s, const CallPlan& p, CallBufs& b) {
    const size_t need = scratch_need(s, p);
    if (p.taping) return fail(s, BTL_E_INVAL, "btl_forward_noalloc keeps no adjoint tape");
    if (!s->scratch) return fail(s, BTL_E_HIP, "device scratch unavailable");
    if (need > kScratchBytes) {
        char msg[160];
        snprintf(msg, sizeof(msg), "btl_forward_noalloc: the call needs %zu bytes of device scratch, "
                 "the maximum is %zu", need, kScratchBytes);
        return fail(s, BTL_E_INVAL, msg);
    }
    const size_t esz = state_elem_bytes(s);
    char* c = s->scratch;
    auto take = [&c](size_t n) {
        char* r = c;
        c += align256(n);
        return r;
    };
    b.pop[0] = take((size_t)p.pop_elems * esz);
    b.pop[1] = take((size_t)p.pop_elems * esz);
    b.fields = reinterpret_cast<FieldDesc*>(take(p.n_fields * sizeof(FieldDesc)));
    b.blk = reinterpret_cast<int2*>(take(p.nblk_total * sizeof(int2)));
    b.steps = reinterpret_cast<double*>(take(p.steps.size() * sizeof(double)));
    b.consts = reinterpret_cast<double*>(take(p.consts.size() * sizeof(double)));
    b.partial = reinterpret_cast<double2*>(
        take((size_t)kTabSteps * p.nblk_total * (kBlock / 64) * sizeof(double2)));
    b.tab = reinterpret_cast<double2*>(take((size_t)kTabSteps * p.T * sizeof(double2)));
    b.tabf = reinterpret_cast<int32_t*>(take(p.T * sizeof(int32_t)));
    return BTL_OK;
}

// Pinned staging: wait until the slot's previous uploads have been read,
// grow it when allowed (grow = false: fail instead of allocating).
static btl_status stage_acquire(btl_sim* s, size_t total, bool grow, char** out) {
    const int slot = s->stage_slot;
    hipError_t e;
    if (s->stage_used[slot] && (e = hipEventSynchronize(s->stage_ev[slot])) != hipSuccess)
        return hip_fail(s, e, "waiting for staging slot");
    s->stage_used[slot] = false;
    if (s->stage_cap[slot] < total) {
        if (!grow) {
            char msg[160];
            snprintf(msg, sizeof(msg), "btl_forward_noalloc: the call's tables need %zu bytes of "
                     "staging, the simulator has %zu", total, s->stage_cap[slot]);
            return fail(s, BTL_E_INVAL, msg);
        }
        if (s->stage[slot]) (void)hipHostFree(s->stage[slot]);
        s->stage[slot] = nullptr;
        s->stage_cap[slot] = 0;
        if ((e = hipHostMalloc((void**)&s->stage[slot], total, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(s, e, "allocating pinned staging");
        s->stage_cap[slot] = total;
    }
    *out = s->stage[slot];
    return BTL_OK;
}

static btl_status stage_release(btl_sim* s, hipStream_t st) {
    const int slot = s->stage_slot;
    const hipError_t e = hipEventRecord(s->stage_ev[slot], st);
    if (e != hipSuccess) return hip_fail(s, e, "recording staging event");
    s->stage_used[slot] = true;
    s->stage_slot ^= 1;
    return BTL_OK;
}

// One asynchronous upload of several host arrays through a staging slot.
struct Upload {
    const void* src;
    void* dst;
    size_t bytes;
};
static btl_status upload(btl_sim* s, const std::vector<Upload>& ups, bool grow, hipStream_t st) {
    size_t total = 0;
    for (const Upload& u : ups) total += align256(u.bytes);
    char* stg = nullptr;
    btl_status rc = stage_acquire(s, total, grow, &stg);
    if (rc != BTL_OK) return rc;
    size_t off = 0;
    for (const Upload& u : ups) {
        if (u.bytes == 0) continue;
        memcpy(stg + off, u.src, u.bytes);
        const hipError_t e = hipMemcpyAsync(u.dst, stg + off, u.bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(s, e, "uploading tables");
        off += align256(u.bytes);
    }
    return stage_release(s, st);
}

static btl_status upload_plan(btl_sim* s, const CallPlan& p, const CallBufs& b, bool grow,
                              hipStream_t st) {
    std::vector<Upload> ups = {
        {p.fl.data(), b.fields, p.fl.size() * sizeof(FieldDesc)},
        {p.blk.data(), b.blk, p.blk.size() * sizeof(int2)},
        {p.steps.data(), b.steps, p.steps.size() * sizeof(double)},
        {p.consts.data(), b.consts, p.consts.size() * sizeof(double)},
        {p.tabf.data(), b.tabf, p.tabf.size() * sizeof(int32_t)}};
    if (p.taping) {
        ups.push_back({p.afl.data(), b.afields, p.afl.size() * sizeof(FieldDesc)});
        ups.push_back({p.ablk.data(), b.ablk, p.ablk.size() * sizeof(int2)});
        ups.push_back({p.gmeta.data(), b.agmeta, p.gmeta.size() * sizeof(double)});
    }
    return upload(s, ups, grow, st);
}

// Step arguments shared by every launch of a call (the per-step fields are
// set by the caller).
static StepArgs step_args(const btl_sim* s, const CallPlan& p, const CallBufs& b) {
    const int32_t P = p.P;
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.words = s->words.p;
    a.fields = b.fields;
    a.blk_field = b.blk;
    a.fdt = b.steps;
    a.Fk = b.steps + p.K;
    a.w = b.consts;
    a.decay = b.consts + P;
    a.trans = b.consts + 2 * P;
    a.rdt = b.consts + 3 * P + 2 * P * P;
    a.gm = p.uses_gm ? s->gm.p : nullptr;
    a.cvm = p.uses_cv ? s->cvm.p : nullptr;
    a.cvh = s->cvh.p;
    a.cvt = s->cvt.p;
    a.kdt = b.consts + 4 * P + 2 * P * P;
    a.edx = lattice_eps(p.nq) * s->dx;
    a.nq = p.nq;
    a.xcd = p.xcd_on;
    a.classical = p.classical ? 1 : 0;
    a.partial = b.partial;
    a.n_phase = P;
    a.K = p.K;
    a.tab_field = b.tabf;
    a.T = p.T;
    return a;
}

// Everything a forward enqueues after the uploads: init, one table launch
// per kTabSteps steps, one step launch per step, one signal launch per
// kTabSteps steps and, with a uniform tape, the checkpoint copies.
static btl_status enqueue_forward(btl_sim* s, const CallPlan& p, const CallBufs& b, hipStream_t q,
                                  double* Eptr, char* ckpt, int32_t C) {
    const size_t state_bytes = (size_t)p.pop_elems * state_elem_bytes(s);
    const int32_t K = p.K;
    hipError_t err;
    // without a tape, the classical scheme's initial collision or curved
    // links (whose pass reads the state), the first step starts from the
    // equilibrium constants and no initial state is written
    const bool fused = K > 0 && !ckpt && !p.classical && !p.uses_cv;
    if ((err = launch_init(s->prec, b.pop[0], p.pop_elems, b.fields, p.n_fields, p.fl.data(), Eptr,
                           p.Q, K, p.nq, q, !fused)) != hipSuccess)
        return hip_fail(s, err, "init launch");
    if (p.classical && K > 0 &&
        (err = launch_init_classical(s->prec, b.pop[0], p.fl.data(), p.n_fields, s->words.p,
                                     b.steps, b.consts + 3 * p.P + 2 * p.P * p.P, p.nq, q)) !=
            hipSuccess)
        return hip_fail(s, err, "init launch");
    if (ckpt && K > 0 &&
        (err = hipMemcpyAsync(ckpt, b.pop[0], state_bytes, hipMemcpyDeviceToDevice, q)) != hipSuccess)
        return hip_fail(s, err, "checkpoint copy");
    StepArgs a = step_args(s, p, b);
    for (int k = 0; k < K; ++k) {
        if (k % kTabSteps == 0) {
            a.k = k;
            a.tab = b.tab;
            if ((err = launch_tables(a, std::min(kTabSteps, K - k), q)) != hipSuccess)
                return hip_fail(s, err, "table launch");
        }
        a.tab = b.tab + (size_t)(k % kTabSteps) * p.T;
        a.src = b.pop[k & 1];
        a.dst = b.pop[(k + 1) & 1];
        a.k = k;
        a.first = fused && k == 0 ? 1 : 0;
        if (p.uses_cv &&
            (err = launch_links(s->prec, a, s->cv_max_links, p.n_fields, q)) != hipSuccess)
            return hip_fail(s, err, "membrane link launch");
        if ((err = launch_step(s->prec, p.shape, a, p.nblk_total, q)) != hipSuccess)
            return hip_fail(s, err, "step launch");
        if ((k + 1) % kTabSteps == 0 || k + 1 == K) {
            const int32_t k0 = k - k % kTabSteps;
            if ((err = launch_esum(b.partial, b.fields, p.n_fields, p.nblk_total, k0, k + 1 - k0,
                                   Eptr, K, s->nf_dev, q)) != hipSuccess)
                return hip_fail(s, err, "signal launch");
        }
        if (ckpt && (k + 1) % C == 0 && k + 1 < K) {
            const size_t m = (size_t)(k + 1) / C;
            if ((err = hipMemcpyAsync(ckpt + m * state_bytes, b.pop[(k + 1) & 1], state_bytes,
                                      hipMemcpyDeviceToDevice, q)) != hipSuccess)
                return hip_fail(s, err, "checkpoint copy");
        }
    }
    return BTL_OK;
}

// Run a planned, uploaded forward on stream st: eagerly, or (K >= 16 steps,
// graphs on) by replaying a cached hipGraph of the same launches.  The
// graph writes the signal into the simulator's own buffer, copied to E.
static btl_status run_forward(btl_sim* s, const CallPlan& p, const CallBufs& b, hipStream_t st,
                              double* E, char* ckpt, int32_t C) {
    const int32_t K = p.K, Q = p.Q;
    const bool use_graph = K >= kGraphMinSteps && s->use_graphs;
    if (!use_graph) return enqueue_forward(s, p, b, st, E, ckpt, C);
    hipError_t e;
    const size_t ebytes = (size_t)Q * (K + 1) * 2 * sizeof(double);
    if ((e = s->E_int.ensure((size_t)Q * (K + 1) * 2)) != hipSuccess)
        return hip_fail(s, e, "allocating signal buffer");
    GraphKey key;
    memset(&key, 0, sizeof(key));
    key.prec = s->prec;
    key.K = K;
    key.Q = Q;
    key.n_fields = p.n_fields;
    key.nblk = p.nblk_total;
    key.shape = p.shape;
    key.T = p.T;
    key.ckpt = ckpt ? C : 0;
    key.scheme = p.classical ? 1 : 0;
    key.nq = p.nq;
    key.xcd = p.xcd_on | p.order;
    key.fields = field_hash(p.fl, p.classical);
    const void* ptrs[] = {b.pop[0], b.pop[1], b.fields, b.blk, b.steps, b.consts, b.partial,
                          b.tab, b.tabf, s->E_int.p, ckpt, s->words.p, s->gm.p, s->nf_dev,
                          s->cvm.p, s->cvh.p, s->cvt.p};
    static_assert(sizeof(ptrs) / sizeof(ptrs[0]) <= sizeof(key.ptr) / sizeof(key.ptr[0]),
                  "graph key too small");
    for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) key.ptr[i] = ptrs[i];
    GraphSlot* hit = nullptr;
    for (GraphSlot& g : s->graphs)
        if (g.exec && memcmp(&key, &g.key, sizeof(key)) == 0) hit = &g;
    if (!hit) {
        // replace the least recently used slot
        hit = &s->graphs[0];
        for (GraphSlot& g : s->graphs)
            if (!g.exec || (hit->exec && g.used < hit->used)) hit = &g;
        if (hit->exec) {
            (void)hipGraphExecDestroy(hit->exec);
            hit->exec = nullptr;
        }
        if (!s->cap_stream &&
            (e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(s, e, "creating capture stream");
        if ((e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(s, e, "begin capture");
        const btl_status rc = enqueue_forward(s, p, b, s->cap_stream, s->E_int.p, ckpt, C);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(s->cap_stream, &graph);
        if (rc != BTL_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (ec != hipSuccess) return hip_fail(s, ec, "end capture");
        e = hipGraphInstantiate(&hit->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            hit->exec = nullptr;
            return hip_fail(s, e, "graph instantiate");
        }
        hit->key = key;
    }
    hit->used = ++s->graph_clock;
    if ((e = hipGraphLaunch(hit->exec, st)) != hipSuccess) return hip_fail(s, e, "graph launch");
    if ((e = hipMemcpyAsync(E, s->E_int.p, ebytes, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hip_fail(s, e, "signal copy");
    return BTL_OK;
}

static btl_status final_magnetization(btl_sim* s, const CallPlan& p, const CallBufs& b,
                                      void* M_final, hipStream_t st) {
    if (!M_final) return BTL_OK;
    const hipError_t e =
        launch_mfinal(s->prec, b.pop[p.K & 1], p.fl.data(), p.n_fields, M_final, p.nq, st);
    if (e != hipSuccess) return hip_fail(s, e, "final magnetization launch");
    return BTL_OK;
}

// One planned call on the simulator's buffers, with a uniform tape when
// C > 0 (the state every C steps, for btl_backward).
// Term tables of the membranes at an angle for this call's lattice, dt and
// permeabilities (built when these differ from the tables' constants).
// Work still queued on st may read the old tables: it finishes first.
// Without may_alloc the tables must fit the device buffers they have.
// The fields' ranges in the head table of the current build.
static void curved_ranges(const btl_sim* s, CallPlan& p) {
    for (FieldDesc& d : p.fl) {
        d.cv_h0 = d.cv_nh = 0;
        for (const CurvedGeom& cg : s->curved)
            if (d.cv >= 0 && cg.cv_off == d.cv) {
                d.cv_h0 = cg.h0;
                d.cv_nh = cg.nh;
            }
    }
}

static btl_status ensure_curved(btl_sim* s, CallPlan& p, const double* kappa, hipStream_t st,
                                bool may_alloc) {
    if (!p.uses_cv) return BTL_OK;
    std::vector<double> key = {(double)p.nq, p.dt};
    key.insert(key.end(), kappa, kappa + p.P * p.P);
    if (key.size() == s->cv_key.size() &&
        memcmp(key.data(), s->cv_key.data(), key.size() * sizeof(double)) == 0) {
        curved_ranges(s, p);
        return BTL_OK;
    }
    std::vector<uint8_t> mask(s->cvm_elems, 0);
    std::vector<int4> heads;
    std::vector<CvTerm> terms;
    for (CurvedGeom& cg : s->curved) {
        const size_t ns = cg.comp.size();
        std::vector<int32_t> idx(6 * ns, -1);
        cg.h0 = (int32_t)heads.size();
        if (!curved_terms(cg, p.nq, p.dt, s->dx, kappa, p.P, idx.data(), heads, terms))
            return fail(s, BTL_E_UNSUPPORTED, "more than 2^31 - 1 membrane terms");
        cg.nh = (int32_t)heads.size() - cg.h0;
        for (int d = 0; d < 6; ++d)
            for (size_t j = 0; j < ns; ++j)
                if (idx[d * ns + j] >= 0) mask[cg.cv_off + j] |= (uint8_t)(1u << d);
    }
    curved_ranges(s, p);
    if (heads.empty()) heads.push_back(make_int4(0, 0, 0, 0));
    if (terms.empty()) terms.push_back(CvTerm{0.0, 0, 0});
    if (!may_alloc && (mask.size() > s->cvm.cap || heads.size() > s->cvh.cap ||
                       terms.size() > s->cvt.cap))
        return fail(s, BTL_E_UNSUPPORTED,
                    "the membrane term tables for these constants need device memory: run "
                    "btl_forward with them first");
    s->cv_key.clear();
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = s->cvm.ensure(mask.size());
    if (e == hipSuccess) e = s->cvh.ensure(heads.size());
    if (e == hipSuccess) e = s->cvt.ensure(terms.size());
    if (e == hipSuccess)
        e = hipMemcpy(s->cvm.p, mask.data(), mask.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s->cvh.p, heads.data(), heads.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s->cvt.p, terms.data(), terms.size() * sizeof(CvTerm),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(s, e, "membrane term tables");
    s->cv_key = key;
    return BTL_OK;
}

static btl_status forward_call(btl_sim* s, const Settings& cs, double dt, int32_t K,
                               const double* D, const double* T2, const double* kappa, int32_t Q,
                               const int32_t* q_geom, const double* gG0, const double* f,
                               double* E, void* M_final, int32_t C, hipStream_t st) {
    CallPlan p;
    btl_status rc = make_plan(s, cs, dt, K, D, T2, kappa, Q, q_geom, gG0, f, C > 0, p);
    if (rc != BTL_OK) return rc;
    if ((rc = ensure_curved(s, p, kappa, st, true)) != BTL_OK) return rc;
    CallBufs b;
    if ((rc = alloc_bufs(s, p, b)) != BTL_OK) return rc;
    if ((rc = upload_plan(s, p, b, true, st)) != BTL_OK) return rc;
    char* ckpt = nullptr;
    if (p.taping) {
        C = std::min(C, K);
        const int32_t nck = (K + C - 1) / C;
        const size_t state_bytes = (size_t)p.pop_elems * state_elem_bytes(s);
        hipError_t e;
        if ((e = s->ckpt.ensure((size_t)nck * state_bytes)) != hipSuccess)
            return hip_fail(s, e, "allocating checkpoints");
        ckpt = s->ckpt.p;
        btl_sim::Tape& tp = s->tape;
        tp = btl_sim::Tape();
        tp.set = cs;
        tp.K = K;
        tp.C = C;
        tp.Q = Q;
        tp.T = p.T;
        tp.n_fields = p.n_fields;
        tp.nblk = p.nblk_total;
        tp.nblk_adj = p.nblk_adj;
        tp.g_ok = p.g_complete;
        tp.shape = p.shape;
        tp.dt = dt;
        tp.sub = p.msub;
        tp.xcd = p.xcd_on;
        tp.state_elems = p.pop_elems;
        tp.nq = p.nq;
    }
    if ((rc = run_forward(s, p, b, st, E, ckpt, C)) != BTL_OK) return rc;
    if (p.taping) s->tape.valid = true;
    return final_magnetization(s, p, b, M_final, st);
}

// Consecutive groups of q-samples ("q-waves") whose states fit the budget:
// per_q[q] bytes each, at most `budget` per group (at least one q-sample).
static std::vector<int32_t> wave_bounds(const std::vector<double>& per_q, double budget) {
    std::vector<int32_t> cut = {0};
    const int32_t Q = (int32_t)per_q.size();
    int32_t q0 = 0;
    while (q0 < Q) {
        double acc = 0.0;
        int32_t q1 = q0;
        while (q1 < Q && (q1 == q0 || acc + per_q[q1] <= budget)) acc += per_q[q1++];
        cut.push_back(q1);
        q0 = q1;
    }
    return cut;
}

// Free the population states, checkpoints and adjoint states of earlier
// calls, and the cached graphs that capture their addresses (the next call
// allocates what it needs).
static void drop_states(btl_sim* s) {
    for (GraphSlot& g : s->graphs)
        if (g.exec) {
            (void)hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
        }
    s->seg.release();
    s->ckpt.release();
    s->pop[0].release();
    s->pop[1].release();
    s->lam[0].release();
    s->lam[1].release();
}

// Report (and clear) a non-finite value left by earlier work on the device.
static btl_status take_nonfinite(btl_sim* s) {
    if (s->nf_host && __atomic_load_n(s->nf_host, __ATOMIC_ACQUIRE) != 0) {
        __atomic_store_n(s->nf_host, 0, __ATOMIC_RELEASE);
        return fail(s, BTL_E_NONFINITE,
                    "a non-finite signal or gradient was produced by earlier work of this "
                    "simulator (reported once)");
    }
    return BTL_OK;
}

// Forward without the non-finite check (btl_forward and the autotuner's
// probes): q-waves when the states exceed the budget; a taped forward keeps
// a uniform tape when it fits, otherwise a deferred one (btl_backward then
// replays the forward from t = 0 with binomial checkpointing).
static btl_status forward_entry(btl_sim* s, double dt, int32_t K, const double* D,
                                const double* T2, const double* kappa, int32_t Q,
                                const int32_t* q_geom, const double* gG0, const double* f,
                                double* E, void* M_final, int32_t ckpt_every, void* stream) {
    if (!s) return BTL_E_INVAL;
    const Settings cs = s->set;
    if (ckpt_every < 0) return fail(s, BTL_E_INVAL, "ckpt_every must be >= 0");
    btl_status rc = validate_inputs(s, cs, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E);
    if (rc != BTL_OK) return rc;
    const int32_t P = s->n_phase;
    s->last.valid = true;
    s->last.dt = dt;
    s->last.D.assign(D, D + P);
    s->last.T2.assign(T2, T2 + P);
    s->last.kappa.assign(kappa, kappa + P * P);
    s->last.gG0.assign(gG0, gG0 + 3 * Q);
    s->last.f.assign(f, f + (size_t)K * cs.msub);
    s->last.q_geom.assign(q_geom, q_geom + Q);
    s->tape.valid = false;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool taping = ckpt_every > 0 && K > 0;
    if (taping && (rc = adjoint_supported(s, cs, Q, q_geom)) != BTL_OK) return rc;
    const size_t esz = state_elem_bytes(s);
    const double budget = memory_budget(s);
    const bool full = taping && cs.grad_g;
    std::vector<double> per_q(Q);
    double S = 0.0;   // one state of all q-samples, bytes
    for (int q = 0; q < Q; ++q) {
        per_q[q] = (double)q_state_elems(s, cs, q_geom[q], gG0 + 3 * q, full) * esz;
        S += per_q[q];
    }
    if (taping) {
        const int32_t C = std::min(ckpt_every, K);
        const int32_t nck = (K + C - 1) / C;
        // checkpoints + segment + two adjoint states + two forward states
        if ((double)(nck + C + 4) * S <= budget)
            return forward_call(s, cs, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E, M_final, C, st);
    } else if (2.0 * S <= budget) {
        return forward_call(s, cs, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E, M_final, 0, st);
    }
    // q-waves (no tape kept on the device)
    for (double& v : per_q) v *= 2.0;
    const std::vector<int32_t> cut = wave_bounds(per_q, budget);
    int64_t m_off = 0;
    for (size_t w = 0; w + 1 < cut.size(); ++w) {
        const int32_t q0 = cut[w], q1 = cut[w + 1];
        if (per_q[q0] > budget && q1 == q0 + 1)
            return fail(s, BTL_E_NOMEM, "one q-sample does not fit in device memory");
        void* Mw = M_final ? static_cast<char*>(M_final) + m_off * esz : nullptr;
        rc = forward_call(s, cs, dt, K, D, T2, kappa, q1 - q0, q_geom + q0, gG0 + 3 * q0, f,
                          E + (size_t)q0 * (K + 1) * 2, Mw, 0, st);
        if (rc != BTL_OK) return rc;
        for (int q = q0; q < q1; ++q) m_off += s->geoms[q_geom[q]].nsites;
    }
    if (taping) {
        // deferred tape: the inputs are all a reverse sweep needs, since the
        // initial state is the equilibrium at M = 1
        btl_sim::Tape& tp = s->tape;
        tp = btl_sim::Tape();
        tp.deferred = true;
        tp.set = cs;
        tp.K = K;
        tp.C = std::min(ckpt_every, K);
        tp.Q = Q;
        tp.dt = dt;
        tp.sub = cs.msub;
        tp.nq = cs.nq;
        tp.D.assign(D, D + P);
        tp.T2.assign(T2, T2 + P);
        tp.kappa.assign(kappa, kappa + P * P);
        tp.gG0.assign(gG0, gG0 + 3 * Q);
        tp.f.assign(f, f + (size_t)K * cs.msub);
        tp.q_geom.assign(q_geom, q_geom + Q);
        CallPlan pg;   // the field set the reverse sweep will plan (gamma G0 support)
        if ((rc = make_plan(s, cs, dt, K, D, T2, kappa, Q, q_geom, gG0, f, true, pg)) != BTL_OK)
            return rc;
        tp.g_ok = pg.g_complete;
        tp.n_fields = pg.n_fields;
        tp.valid = true;
    }
    return BTL_OK;
}

extern "C" btl_status btl_forward(btl_sim* s, double dt, int32_t K, const double* D,
                                  const double* T2, const double* kappa, int32_t Q,
                                  const int32_t* q_geom, const double* gG0, const double* f,
                                  double* E, void* M_final, int32_t ckpt_every, void* stream) {
    if (!s) return BTL_E_INVAL;
    const btl_status rc = take_nonfinite(s);
    if (rc != BTL_OK) return rc;
    return forward_entry(s, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E, M_final, ckpt_every,
                         stream);
}

extern "C" btl_status btl_forward_noalloc(btl_sim* s, double dt, int32_t K, const double* D,
                                          const double* T2, const double* kappa, int32_t Q,
                                          const int32_t* q_geom, const double* gG0,
                                          const double* f, double* E, void* M_final,
                                          void* stream) {
    if (!s) return BTL_E_INVAL;
    btl_status rc = take_nonfinite(s);
    if (rc != BTL_OK) return rc;
    const Settings cs = s->set;
    if ((rc = validate_inputs(s, cs, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E)) != BTL_OK)
        return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    CallPlan p;
    if ((rc = make_plan(s, cs, dt, K, D, T2, kappa, Q, q_geom, gG0, f, false, p)) != BTL_OK)
        return rc;
    if ((rc = ensure_curved(s, p, kappa, st, false)) != BTL_OK) return rc;
    CallBufs b;
    if ((rc = scratch_bufs(s, p, b)) != BTL_OK) return rc;
    if ((rc = upload_plan(s, p, b, false, st)) != BTL_OK) return rc;
    if ((rc = enqueue_forward(s, p, b, st, E, nullptr, 0)) != BTL_OK) return rc;
    return final_magnetization(s, p, b, M_final, st);
}

extern "C" btl_status btl_synchronize(btl_sim* s, void* stream) {
    if (!s) return BTL_E_INVAL;
    const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(s, e, "stream synchronize");
    return take_nonfinite(s);
}

// C(n, k), or cap + 1 when it exceeds cap (no overflow for n <= 2^31).
static int64_t binom_cap(int64_t n, int64_t k, int64_t cap) {
    if (k < 0 || k > n) return 0;
    k = std::min(k, n - k);
    int64_t v = 1;
    for (int64_t i = 1; i <= k; ++i) {
        // v = C(n - k + i, i) grows with i: stop as soon as it passes cap
        v = v * (n - k + i) / i;
        if (v > cap) return cap + 1;
    }
    return v;
}

// One action of a reversal schedule.  Advance: forward steps k0 .. k1 - 1
// from the state at k0 in slot src into slot dst (-1: the work buffers).
// Adjoint: adjoint step k1 from the state at k1 - 1 in slot src (-1: the
// work buffer the last advance wrote).
struct RevAction {
    int kind;   // 0 advance, 1 adjoint step
    int32_t k0, k1;
    int src, dst;
};

// Reversal by binomial checkpointing (Griewank's schedule): the adjoint
// steps b, b - 1, .., a + 1, with the state at a kept in slot sa and the
// slots in `free` available.  With s slots in all (sa included) and
// repetition number t (forward steps taken at most t times each), at most
// beta(s, t) = C(s + t, t) steps can be reversed, and
// beta(s, t) = beta(s, t - 1) + beta(s - 1, t): a first new checkpoint j
// steps beyond a leaves the steps after it to s - 1 slots at the same t
// (j >= l - beta(s - 1, t)) and the steps before it to s slots at t - 1
// (j <= beta(s, t - 1)).  Within that range j = beta(s, t - 2) gives the
// least recomputation, t l - C(s + t, t - 1) forward steps in all for l
// steps (the minimum for s slots).
static void plan_reversal(int32_t a, int32_t b, int sa, std::vector<int>& free,
                          std::vector<RevAction>& out) {
    const int32_t l = b - a;
    if (l == 1) {
        out.push_back({1, a, b, sa, sa});
        return;
    }
    if (free.empty()) {
        // only the state at a: advance from it afresh for every step
        for (int32_t k = b; k > a; --k) {
            if (k - 1 > a) {
                out.push_back({0, a, k - 1, sa, -1});
                out.push_back({1, k - 1, k, -1, -1});
            } else {
                out.push_back({1, a, k, sa, sa});
            }
        }
        return;
    }
    const int64_t s = (int64_t)free.size() + 1;
    int64_t t = 1;
    while (binom_cap(s + t, t, l) < l) ++t;
    const int64_t lo = std::max<int64_t>(1, l - binom_cap(s - 1 + t, t, l));
    const int64_t hi = std::min<int64_t>(l - 1, binom_cap(s + t - 1, t - 1, l));
    const int64_t pref = t >= 2 ? binom_cap(s + t - 2, t - 2, l) : 1;
    const int32_t m = a + (int32_t)std::max(lo, std::min(hi, pref));
    const int slot = free.back();
    free.pop_back();
    out.push_back({0, a, m, sa, slot});
    plan_reversal(m, b, slot, free, out);
    free.push_back(slot);
    plan_reversal(a, m, sa, free, out);
}

static AdjArgs adj_args(const btl_sim* s, const Settings& cs, const FieldDesc* afields,
                        const int2* ablk, const double* consts, int32_t nblk_adj,
                        const double* dL_dE, double dt, int32_t K, int NG, bool gradg, int nq) {
    const int32_t P = s->n_phase;
    AdjArgs aa;
    memset(&aa, 0, sizeof(aa));
    aa.words = s->words.p;
    aa.fields = afields;
    aa.blk_field = ablk;
    aa.w = consts;
    aa.decay = consts + P;
    aa.trans = consts + 2 * P;
    aa.dLdE = reinterpret_cast<const double2*>(dL_dE);
    aa.gpart = s->gpart.p;
    aa.dt = dt;
    aa.xcd = cs.adj_xcd >= 0 ? cs.adj_xcd : (nblk_adj > kXcdMinBlocks ? 1 : 0);
    aa.n_phase = P;
    aa.K = K;
    aa.ng = NG;
    aa.gradg = gradg ? 1 : 0;
    aa.nq = nq;
    return aa;
}

static btl_status final_gradients(btl_sim* s, const double* gfield, int32_t K, int32_t nf,
                                  int NG, double dt, int32_t sub, int32_t Q, int nq,
                                  const double* gmeta, double* dD, double* dT2, double* dkappa,
                                  double* df, double* dgG0, hipStream_t st) {
    const int32_t P = s->n_phase;
    const hipError_t e = launch_adj_final(
        gfield, K, nf, P, dt, s->dx, s->consts.p, s->consts.p + 2 * P + P * P,
        s->consts.p + 3 * P + P * P, dD, dT2, dkappa, df, sub, NG, gmeta, s->steps.p,
        s->steps.p + K, Q, dgG0, lattice_eps(nq), nq == 5 ? 1 : 0, s->nf_dev, st);
    if (e != hipSuccess) return hip_fail(s, e, "adjoint final launch");
    return BTL_OK;
}

// Reverse sweep over a uniform tape: per segment (last first), recompute the
// segment's states from its checkpoint, then run its adjoint steps.
static btl_status backward_uniform(btl_sim* s, const double* dL_dE, double* dD, double* dT2,
                                   double* dkappa, double* df, double* dgG0, hipStream_t st) {
    const btl_sim::Tape& tp = s->tape;
    const int32_t K = tp.K, C = tp.C, T = tp.T, P = s->n_phase, nf = tp.n_fields;
    const int NG = 2 * P + P * P + 2 + (dgG0 ? kNGGrad : 0);
    const size_t state_bytes = (size_t)tp.state_elems * state_elem_bytes(s);
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
    AdjArgs aa = adj_args(s, tp.set, s->adj_fields.p, s->adj_blk.p, s->consts.p, nblk_adj, dL_dE,
                          tp.dt, K, NG, dgG0 != nullptr, tp.nq);

    const int32_t nseg = (K + C - 1) / C;
    int lam_cur = 0;      // buffer holding Lambda^k on entry to adjoint step k
    int64_t nfwd = 0;
    s->tev_used = 0;
    s->tev_steps = 0;
    while ((int32_t)s->tev.size() < 2 * nseg) {
        hipEvent_t ev;
        if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(s, e, "timing events");
        s->tev.push_back(ev);
    }
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
            ++nfwd;
        }
        // reverse sweep over the segment, bracketed by timing events (each
        // after an empty launch, so that the interval holds the adjoint
        // launches alone)
        if ((e = launch_mark(st)) != hipSuccess ||
            (e = hipEventRecord(s->tev[s->tev_used], st)) != hipSuccess)
            return hip_fail(s, e, "timing event");
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
        if ((e = launch_mark(st)) != hipSuccess ||
            (e = hipEventRecord(s->tev[s->tev_used + 1], st)) != hipSuccess)
            return hip_fail(s, e, "timing event");
        s->tev_used += 2;
        s->tev_steps += k1 - k0;
        // per-step, per-field sums of this segment: gfield[k0 .. k1 - 1]
        if ((e = launch_adj_gsum(s->gpart.p, s->adj_fields.p, nf, nblk_adj, NG, k0, k1 - k0,
                                 s->gfield.p, 0, nf, st)) != hipSuccess)
            return hip_fail(s, e, "adjoint sum launch");
    }
    s->stat_fwd_steps = nfwd;
    s->stat_waves = 1;
    s->stat_snapshots = 0;
    return final_gradients(s, s->gfield.p, K, nf, NG, tp.dt, tp.sub, tp.Q, tp.nq,
                           s->adj_gmeta.p, dD, dT2, dkappa, df, dgG0, st);
}

// Reverse sweep of a deferred tape: the q-samples in groups whose states fit
// the memory budget, each group replayed from t = 0 (the equilibrium at
// M = 1) under a binomial checkpointing schedule with as many snapshot
// slots as fit.  Per-step, per-field sums go to one record spanning every
// group in the order of a single batch, so the final gradients are formed
// exactly as after a uniform tape.
static btl_status backward_deferred(btl_sim* s, const double* dL_dE, double* dD, double* dT2,
                                    double* dkappa, double* df, double* dgG0, hipStream_t st) {
    const btl_sim::Tape tp = s->tape;   // copy: planning below must not alias the record
    const Settings& cs = tp.set;
    const int32_t K = tp.K, Q = tp.Q, P = s->n_phase;
    const int NG = 2 * P + P * P + 2 + (dgG0 ? kNGGrad : 0);
    const size_t esz = state_elem_bytes(s);
    btl_status rc;
    hipError_t e;
    CallPlan G;
    if ((rc = make_plan(s, cs, tp.dt, K, tp.D.data(), tp.T2.data(), tp.kappa.data(), Q,
                        tp.q_geom.data(), tp.gG0.data(), tp.f.data(), true, G)) != BTL_OK)
        return rc;
    const int32_t nfT = G.n_fields;
    std::vector<double> per_q(Q, 0.0);
    for (int32_t i = 0; i < nfT; ++i)
        per_q[(int)G.gmeta[(size_t)i * kGMeta]] += (double)G.nq * G.fl[i].nsites * esz;
    // drop the states and graphs of earlier calls: the sweep sizes its own
    drop_states(s);
    const double B = memory_budget(s);
    // groups sized for a repetition number of at most two where possible
    // (beta(s, 2) >= K), each q-sample on its own otherwise
    int64_t s_target = 1;
    while (s_target < K && binom_cap(s_target + 2, 2, K) < K) ++s_target;
    std::vector<double> need(per_q);
    for (double& v : need) v *= (double)(s_target + 4);
    const std::vector<int32_t> cut = wave_bounds(need, B);
    if ((e = s->gfield.ensure((size_t)K * nfT * NG)) != hipSuccess)
        return hip_fail(s, e, "allocating adjoint buffers");
    int32_t f0 = 0;
    int64_t nfwd = 0;
    int32_t min_slots = INT32_MAX;
    for (size_t w = 0; w + 1 < cut.size(); ++w) {
        const int32_t q0 = cut[w], q1 = cut[w + 1], Qw = q1 - q0;
        CallPlan W;
        if ((rc = make_plan(s, cs, tp.dt, K, tp.D.data(), tp.T2.data(), tp.kappa.data(), Qw,
                            tp.q_geom.data() + q0, tp.gG0.data() + 3 * q0, tp.f.data(), true,
                            W)) != BTL_OK)
            return rc;
        const size_t Sw = (size_t)W.pop_elems * esz;
        int64_t slots = (int64_t)(B / (double)Sw) - 4;   // two work and two adjoint states
        if (slots < 1)
            return fail(s, BTL_E_NOMEM, "the reverse sweep of one q-sample does not fit in device memory");
        slots = std::min<int64_t>(slots, K);
        min_slots = std::min<int32_t>(min_slots, (int32_t)slots);
        CallBufs b;
        if ((rc = alloc_bufs(s, W, b)) != BTL_OK) return rc;
        if ((rc = upload_plan(s, W, b, true, st)) != BTL_OK) return rc;
        const int32_t T = W.T, nblk_adj = W.nblk_adj;
        if ((e = s->ckpt.ensure((size_t)slots * Sw)) != hipSuccess ||
            (e = s->lam[0].ensure(Sw)) != hipSuccess || (e = s->lam[1].ensure(Sw)) != hipSuccess ||
            (e = s->tab_b.ensure((size_t)(kTabSteps + 2) * T)) != hipSuccess ||
            (e = s->gpart.ensure((size_t)nblk_adj * NG)) != hipSuccess)
            return hip_fail(s, e, "allocating adjoint buffers");
        auto slot_ptr = [&](int i) { return s->ckpt.p + (size_t)i * Sw; };
        // the state at t = 0 in slot 0
        if ((e = launch_init(s->prec, slot_ptr(0), W.pop_elems, b.fields, W.n_fields, W.fl.data(),
                             nullptr, Qw, K, W.nq, st)) != hipSuccess)
            return hip_fail(s, e, "init launch");
        std::vector<int> free;
        for (int i = (int)slots - 1; i >= 1; --i) free.push_back(i);
        std::vector<RevAction> acts;
        plan_reversal(0, K, 0, free, acts);
        StepArgs fa = step_args(s, W, b);
        double2* tab_adj = s->tab_b.p + (size_t)kTabSteps * T;
        AdjArgs aa = adj_args(s, cs, b.afields, b.ablk, b.consts, nblk_adj,
                              dL_dE + (size_t)q0 * (K + 1) * 2, tp.dt, K, NG, dgG0 != nullptr,
                              W.nq);
        const char* last_work = nullptr;
        int lam_cur = 0;
        // BTLBM_VERBOSE: a line per group and every 2000 adjoint steps as
        // they are enqueued (launches block once the queue is full, so this
        // follows the device within the queue's depth)
        const bool verbose = getenv("BTLBM_VERBOSE") != nullptr;
        if (verbose)
            fprintf(stderr, "btlbm reverse sweep: group %zu of %zu, %d q-samples, %lld kept states, "
                    "%zu actions\n", w + 1, cut.size() - 1, Qw, (long long)slots, acts.size());
        for (const RevAction& act : acts) {
            if (act.kind == 0) {
                const char* cur = slot_ptr(act.src);
                for (int32_t k = act.k0; k < act.k1; ++k) {
                    const int32_t j = k - act.k0;
                    if (j % kTabSteps == 0) {
                        fa.k = k;
                        fa.tab = s->tab_b.p;
                        if ((e = launch_tables(fa, std::min(kTabSteps, act.k1 - k), st)) != hipSuccess)
                            return hip_fail(s, e, "table launch");
                    }
                    char* dst = (k == act.k1 - 1 && act.dst >= 0) ? slot_ptr(act.dst) : b.pop[j & 1];
                    fa.k = k;
                    fa.tab = s->tab_b.p + (size_t)(j % kTabSteps) * T;
                    fa.src = cur;
                    fa.dst = dst;
                    if ((e = launch_step(s->prec, W.shape, fa, W.nblk_total, st)) != hipSuccess)
                        return hip_fail(s, e, "recompute launch");
                    cur = dst;
                    ++nfwd;
                }
                if (act.dst < 0) last_work = cur;
            } else {
                const int32_t k = act.k1;
                fa.k = k - 1;
                fa.tab = tab_adj;
                if ((e = launch_tables(fa, k < K ? 2 : 1, st)) != hipSuccess)
                    return hip_fail(s, e, "adjoint table launch");
                aa.k = k;
                aa.top = (k == K) ? 1 : 0;
                aa.lam_in = aa.top ? nullptr : s->lam[lam_cur].p;
                aa.lam_out = s->lam[lam_cur ^ 1].p;
                aa.fwd = act.src >= 0 ? slot_ptr(act.src) : last_work;
                aa.tab_prev = tab_adj;
                aa.tab_cur = aa.top ? tab_adj : tab_adj + T;
                aa.slot = 0;
                if ((e = launch_adj(s->prec, W.shape, aa, nblk_adj, st)) != hipSuccess)
                    return hip_fail(s, e, "adjoint launch");
                lam_cur ^= 1;
                if ((e = launch_adj_gsum(s->gpart.p, b.afields, W.n_fields, nblk_adj, NG, k - 1, 1,
                                         s->gfield.p, f0, nfT, st)) != hipSuccess)
                    return hip_fail(s, e, "adjoint sum launch");
                if (verbose && (K - k + 1) % 2000 == 0)
                    fprintf(stderr, "btlbm reverse sweep: %d of %d adjoint steps enqueued, %lld forward "
                            "steps\n", K - k + 1, K, (long long)nfwd);
            }
        }
        f0 += W.n_fields;
    }
    if ((e = s->adj_gmeta.ensure(G.gmeta.size())) != hipSuccess)
        return hip_fail(s, e, "allocating tables");
    if ((rc = upload(s, {{G.gmeta.data(), s->adj_gmeta.p, G.gmeta.size() * sizeof(double)}}, true,
                     st)) != BTL_OK)
        return rc;
    s->stat_fwd_steps = nfwd;
    s->stat_waves = (int32_t)cut.size() - 1;
    s->stat_snapshots = min_slots;
    s->tev_used = 0;          // adjoint steps interleave with recomputes: not timed
    s->tev_steps = 0;
    return final_gradients(s, s->gfield.p, K, nfT, NG, tp.dt, tp.sub, Q, tp.nq, s->adj_gmeta.p,
                           dD, dT2, dkappa, df, dgG0, st);
}

extern "C" btl_status btl_backward(btl_sim* s, const double* dL_dE, double* dD, double* dT2,
                                   double* dkappa, double* df, double* dgG0, void* stream) {
    if (!s) return BTL_E_INVAL;
    btl_status rc = take_nonfinite(s);
    if (rc != BTL_OK) return rc;
    if (!s->tape.valid) return fail(s, BTL_E_INVAL, "no adjoint tape: run btl_forward with ckpt_every > 0");
    if (!dL_dE) return fail(s, BTL_E_INVAL, "dL_dE is NULL");
    if (dgG0 && !s->tape.g_ok)
        return fail(s, BTL_E_UNSUPPORTED,
                    "dgG0 needs btl_set_grad_gG0(s, 1) before the taped forward (a mirrored axis "
                    "without a gradient component, or the conjugate pairing next to a periodic "
                    "axis, has no image fields to differentiate)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->tape.deferred) return backward_deferred(s, dL_dE, dD, dT2, dkappa, df, dgG0, st);
    return backward_uniform(s, dL_dE, dD, dT2, dkappa, df, dgG0, st);
}

extern "C" btl_status btl_get_backward_stats(const btl_sim* s, int64_t* fwd_steps, int32_t* groups,
                                             int32_t* snapshots) {
    if (!s || !fwd_steps || !groups || !snapshots) return BTL_E_INVAL;
    *fwd_steps = s->stat_fwd_steps;
    *groups = s->stat_waves;
    *snapshots = s->stat_snapshots;
    return BTL_OK;
}

extern "C" btl_status btl_get_backward_timing(btl_sim* s, double* ms_adjoint,
                                              int64_t* adjoint_steps) {
    if (!s || !ms_adjoint || !adjoint_steps) return BTL_E_INVAL;
    if (s->tev_used == 0)
        return fail(s, BTL_E_INVAL, "no timed reverse sweep: the last btl_backward replayed a "
                                    "deferred tape, or none ran");
    hipError_t e = hipEventSynchronize(s->tev[s->tev_used - 1]);
    if (e != hipSuccess) return hip_fail(s, e, "timing events");
    double ms = 0.0;
    for (int32_t i = 0; i < s->tev_used; i += 2) {
        float t = 0.0f;
        if ((e = hipEventElapsedTime(&t, s->tev[i], s->tev[i + 1])) != hipSuccess)
            return hip_fail(s, e, "timing events");
        ms += t;
    }
    *ms_adjoint = ms;
    *adjoint_steps = s->tev_steps;
    return BTL_OK;
}

// Autotuner cache key: device, storage precision, lattice, scheme, and per
// q-sample the kernel geometry, the field count and whether it carries
// membrane positions (what decides the grid and the kernel variant).
static std::string tune_key(const btl_sim* s, const CallPlan& p) {
    hipDeviceProp_t prop;
    memset(&prop, 0, sizeof(prop));
    (void)hipGetDeviceProperties(&prop, s->device);
    std::string k = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
    k += "/p" + std::to_string(s->prec) + "/n" + std::to_string(p.nq) + "/c" +
         std::to_string(p.classical ? 1 : 0);
    for (const FieldDesc& d : p.fl)
        k += "/" + std::to_string(d.n[0]) + "x" + std::to_string(d.n[1]) + "x" +
             std::to_string(d.n[2]) + (d.gm >= 0 ? "g" : "") + (d.cv >= 0 ? "c" : "");
    return k;
}

extern "C" btl_status btl_autotune(btl_sim* s, int32_t Q, int32_t K_probe, void* stream) {
    if (!s) return BTL_E_INVAL;
    btl_status rc = take_nonfinite(s);
    if (rc != BTL_OK) return rc;
    if (!s->last.valid) return fail(s, BTL_E_INVAL, "btl_autotune replays the last btl_forward: call it first");
    if (K_probe < 1) return fail(s, BTL_E_INVAL, "K_probe must be >= 1");
    const btl_sim::SimLast saved = s->last;
    int32_t Qr = std::min<int32_t>(Q > 0 ? Q : (int32_t)saved.q_geom.size(),
                                   (int32_t)saved.q_geom.size());
    // the probe covers at most one q-wave: a batch whose states exceed the
    // budget runs wave after wave in one launch shape, and probes of a part
    // of a wave rank the shapes differently (32 q-samples of a 128-sample
    // wave put the wave's fastest shape 8 % behind)
    if (Qr > 0) {
        const size_t esz = state_elem_bytes(s);
        std::vector<double> per_q(Qr);
        for (int32_t q = 0; q < Qr; ++q)
            per_q[q] = 2.0 * (double)q_state_elems(s, s->set, saved.q_geom[q],
                                                   saved.gG0.data() + 3 * q, false) * esz;
        Qr = wave_bounds(per_q, memory_budget(s))[1];
    }
    std::vector<double> f((size_t)K_probe * s->set.msub);
    for (size_t k = 0; k < f.size(); ++k) f[k] = saved.f.empty() ? 1.0 : saved.f[k % saved.f.size()];
    // a launch this process already chose for the same shape of workload
    std::string key;
    bool shared_geom = false, geom_tables = false;
    {
        Settings cs = s->set;
        cs.tile_shape = -1;
        cs.zc = 0;
        cs.xcd = -1;
        CallPlan p;
        if ((rc = make_plan(s, cs, saved.dt, K_probe, saved.D.data(), saved.T2.data(),
                            saved.kappa.data(), Qr, saved.q_geom.data(), saved.gG0.data(),
                            f.data(), false, p)) != BTL_OK)
            return rc;
        key = tune_key(s, p);
        // fields sharing a geometry (several q-samples, or image fields):
        // the field-interleaved orders are candidates too
        for (int i = 0; i < p.n_fields && !shared_geom; ++i)
            for (int j = i + 1; j < p.n_fields; ++j)
                if (p.fl[j].words == p.fl[i].words) {
                    shared_geom = true;
                    break;
                }
        geom_tables = p.uses_gm || p.uses_cv;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const TuneEntry& t : g_tune_cache)
            if (t.key == key) {
                s->set.tile_shape = t.shape;
                s->set.zc = t.zc;
                s->set.xcd = t.xcd;
                return BTL_OK;
            }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = s->tune_E.ensure((size_t)Qr * (K_probe + 1) * 2)) != hipSuccess)
        return hip_fail(s, e, "autotune buffer");
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        return hip_fail(s, e, "autotune events");
    int nz_max = 1;
    for (int q = 0; q < Qr; ++q)
        nz_max = std::max(nz_max, kernel_geom(s->geoms[saved.q_geom[q]], s->set.nq).n[2]);
    // z-column lengths: whole columns, halves, thirds, quarters, and short
    // columns for small lattices that need more workgroups
    std::vector<int> zcs = {0};
    for (int div : {2, 3, 4}) zcs.push_back((nz_max + div - 1) / div);
    for (int z : {1, 2, 4, 8, 16}) zcs.push_back(z);
    std::sort(zcs.begin(), zcs.end());
    zcs.erase(std::unique(zcs.begin(), zcs.end()), zcs.end());
    zcs.erase(std::remove_if(zcs.begin(), zcs.end(), [&](int z) { return z >= nz_max; }), zcs.end());
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
            const btl_status rr = forward_entry(s, saved.dt, K_probe, saved.D.data(),
                                                saved.T2.data(), saved.kappa.data(), Qr,
                                                saved.q_geom.data(), saved.gG0.data(), f.data(),
                                                s->tune_E.p, nullptr, 0, stream);
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
    const bool verbose = getenv("BTLBM_VERBOSE") != nullptr;
    rc = BTL_OK;
    std::vector<int> shapes;
    if (s->set.nq == 5)
        shapes.push_back(kTile256x1);
    else
        shapes.assign(kShapes3D, kShapes3D + kShapeCount3D);
    // shape, z-column length and workgroup order are searched jointly: the
    // best column length differs between the orders.  Orders: bit 0 the
    // XCD-contiguous numbering, bit 1 the fields of a geometry interleaved
    // block by block (searched with the others when the geometry carries
    // membrane positions or term lists, which every field reads; otherwise
    // tried on the best shape and column length found)
    const int n_orders = shared_geom && geom_tables ? 4 : 2;
    struct Cand {
        float ms;
        int sh, zc, xo;
    };
    std::vector<Cand> timed;
    auto consider = [&](int sh, int zc, int xo) -> btl_status {
        s->set.tile_shape = sh;
        s->set.zc = zc;
        s->set.xcd = xo;
        float ms = 0.0f;
        const btl_status r = time_probe(&ms);
        if (r == BTL_OK) timed.push_back({ms, sh, zc, xo});
        if (r == BTL_OK && verbose)
            fprintf(stderr, "btlbm autotune: shape %d, z-column %d, order %d: %.3f ms\n", sh, zc, xo, ms);
        if (r == BTL_OK && (best < 0.0f || ms < best)) {
            best = ms;
            best_shape = sh;
            best_zc = zc;
            best_xcd = xo;
        }
        return r;
    };
    for (int sh : shapes) {
        for (int zc : zcs) {
            for (int xo = 0; xo < n_orders && rc == BTL_OK; ++xo) rc = consider(sh, zc, xo);
            if (rc != BTL_OK) break;
        }
        if (rc != BTL_OK) break;
    }
    if (rc == BTL_OK && shared_geom && n_orders == 2) {
        const int sh = best_shape, zc = best_zc;
        for (int xo = 2; xo < 4 && rc == BTL_OK; ++xo) rc = consider(sh, zc, xo);
    }
    // the few candidates within 4 % of the best are timed again, in turns,
    // and the fastest of all their timings wins: single probes of a busy
    // device differ by a few per cent, as much as these candidates do
    if (rc == BTL_OK && timed.size() > 1) {
        std::sort(timed.begin(), timed.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
        std::vector<Cand> top;
        for (const Cand& c : timed)
            if (top.size() < 4 && c.ms <= 1.04f * timed[0].ms) top.push_back(c);
        if (top.size() > 1) {
            std::vector<float> bestv(top.size(), -1.0f);
            for (int r = 0; r < kTuneReps && rc == BTL_OK; ++r)
                for (size_t i = 0; i < top.size() && rc == BTL_OK; ++i) {
                    s->set.tile_shape = top[i].sh;
                    s->set.zc = top[i].zc;
                    s->set.xcd = top[i].xo;
                    (void)hipEventRecord(e0, st);
                    rc = forward_entry(s, saved.dt, K_probe, saved.D.data(), saved.T2.data(),
                                       saved.kappa.data(), Qr, saved.q_geom.data(),
                                       saved.gG0.data(), f.data(), s->tune_E.p, nullptr, 0,
                                       stream);
                    if (rc != BTL_OK) break;
                    (void)hipEventRecord(e1, st);
                    if ((e = hipEventSynchronize(e1)) != hipSuccess) {
                        rc = hip_fail(s, e, "autotune timing");
                        break;
                    }
                    float ms = 0.0f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (bestv[i] < 0.0f || ms < bestv[i]) bestv[i] = ms;
                }
            if (rc == BTL_OK && verbose)
                for (size_t i = 0; i < top.size(); ++i)
                    fprintf(stderr, "btlbm autotune: again shape %d, z-column %d, order %d: %.3f ms\n",
                            top[i].sh, top[i].zc, top[i].xo, bestv[i]);
            if (rc == BTL_OK) {
                size_t w = 0;
                for (size_t i = 0; i < top.size(); ++i)
                    if (std::min(bestv[i], top[i].ms) < std::min(bestv[w], top[w].ms)) w = i;
                best = std::min(bestv[w], top[w].ms);
                best_shape = top[w].sh;
                best_zc = top[w].zc;
                best_xcd = top[w].xo;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->last = saved;
    // the probes' states span a whole q-wave: freed, so that memory the
    // caller allocates next (outputs, M_final) does not compete with them
    drop_states(s);
    if (rc != BTL_OK) {
        s->set.tile_shape = -1;
        s->set.zc = 0;
        s->set.xcd = -1;
        return rc;
    }
    s->set.tile_shape = best_shape;
    s->set.zc = best_zc;
    s->set.xcd = best_xcd;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache.push_back({key, best_shape, best_zc, best_xcd});
    }
    if (verbose)
        fprintf(stderr, "btlbm autotune: tile shape %d, z-column %d, xcd order %d (%.3f ms per probe)\n",
                best_shape, best_zc, best_xcd, best);
    return BTL_OK;
}

extern "C" btl_status btl_get_launch(const btl_sim* s, int32_t* tile_shape, int32_t* zc,
                                     int32_t* xcd) {
    if (!s || !tile_shape || !zc || !xcd) return BTL_E_INVAL;
    *tile_shape = s->set.tile_shape;
    *zc = s->set.zc;
    *xcd = s->set.xcd;
    return BTL_OK;
}

extern "C" btl_status btl_set_launch(btl_sim* s, int32_t tile_shape, int32_t zc, int32_t xcd) {
    if (!s) return BTL_E_INVAL;
    if (tile_shape < -1 || tile_shape >= kTileCount)
        return fail(s, BTL_E_INVAL, "tile_shape must be -1 or 0..5");
    if (zc < 0 || zc > kMaxZc) return fail(s, BTL_E_INVAL, "zc must be in 0..1024");
    if (xcd < -1 || xcd > 3) return fail(s, BTL_E_INVAL, "xcd must be -1 or 0..3");
    s->set.tile_shape = tile_shape;
    s->set.zc = zc;
    s->set.xcd = xcd;
    return BTL_OK;
}

extern "C" btl_status btl_set_adjoint_launch(btl_sim* s, int32_t zc, int32_t xcd) {
    if (!s) return BTL_E_INVAL;
    if (zc < -1 || zc > kMaxZc) return fail(s, BTL_E_INVAL, "zc must be in -1..1024");
    if (xcd < -1 || xcd > 1) return fail(s, BTL_E_INVAL, "xcd must be -1, 0 or 1");
    s->set.adj_zc = zc;
    s->set.adj_xcd = xcd;
    return BTL_OK;
}

extern "C" btl_status btl_set_memory_budget(btl_sim* s, int64_t bytes) {
    if (!s) return BTL_E_INVAL;
    if (bytes < 0) return fail(s, BTL_E_INVAL, "the memory budget must be >= 0 (0: none)");
    s->mem_limit = bytes;
    return BTL_OK;
}

extern "C" btl_status btl_set_graphs(btl_sim* s, int32_t on) {
    if (!s) return BTL_E_INVAL;
    if (on != 0 && on != 1) return fail(s, BTL_E_INVAL, "btl_set_graphs takes 0 or 1");
    s->use_graphs = on;
    return BTL_OK;
}

extern "C" btl_status btl_set_lattice(btl_sim* s, int32_t lattice) {
    if (!s) return BTL_E_INVAL;
    if (lattice != BTL_D3Q7 && lattice != BTL_D2Q5)
        return fail(s, BTL_E_INVAL, "lattice must be BTL_D3Q7 or BTL_D2Q5");
    s->set.nq = lattice == BTL_D2Q5 ? 5 : 7;
    s->tape.valid = false;
    s->last.valid = false;
    return BTL_OK;
}

extern "C" btl_status btl_set_grad_gG0(btl_sim* s, int32_t on) {
    if (!s) return BTL_E_INVAL;
    if (on != 0 && on != 1) return fail(s, BTL_E_INVAL, "btl_set_grad_gG0 takes 0 or 1");
    s->set.grad_g = on;
    return BTL_OK;
}

extern "C" btl_status btl_set_substeps(btl_sim* s, int32_t m) {
    if (!s) return BTL_E_INVAL;
    if (m < 1 || m > 65536) return fail(s, BTL_E_INVAL, "substeps must be in 1..65536");
    s->set.msub = m;
    s->last.valid = false;
    return BTL_OK;
}

extern "C" btl_status btl_set_scheme(btl_sim* s, int32_t scheme) {
    if (!s) return BTL_E_INVAL;
    if (scheme != BTL_HYBRID && scheme != BTL_CLASSICAL)
        return fail(s, BTL_E_INVAL, "scheme must be BTL_HYBRID or BTL_CLASSICAL");
    s->set.scheme = scheme;
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
    for (GraphSlot& g : s->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
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
    s->cvm.release();
    s->cvh.release();
    s->cvt.release();
    for (int i = 0; i < 2; ++i) {
        if (s->stage[i]) (void)hipHostFree(s->stage[i]);
        if (s->stage_ev[i]) (void)hipEventDestroy(s->stage_ev[i]);
    }
    if (s->nf_host) (void)hipHostFree(s->nf_host);
    for (hipEvent_t ev : s->tev) (void)hipEventDestroy(ev);
    delete s;
}

extern "C" const char* btl_last_error(const btl_sim* s) {
    return s ? s->err.c_str() : g_create_error.c_str();
}
