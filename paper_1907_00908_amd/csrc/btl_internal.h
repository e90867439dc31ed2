// Internal declarations shared by the kernels and the host runtime of
// libbtlbm.  Not part of the public interface (include/btlbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace btl {

constexpr int kQ = 7;          // D3Q7: 0 rest, 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z
constexpr int kBlock = 256;    // threads per workgroup (4 wavefronts of 64)
constexpr int kMaxZc = 1024;   // longest z column one thread walks (LDS z-phase row)
constexpr int kTabSteps = 32;  // steps whose phase tables one table launch computes
constexpr int kMaxPhase = 8;   // material phases (3-bit neighbour phase in the site word)

// Lattices: D3Q7 (nq = 7: eps_D = 1/4, w_0 = 1/4, w_i = 1/8) and, on a single
// layer, D2Q5 (nq = 5: the first five directions; Sec. 2.2, Eq. omega_i:
// eps_D = 1/3, w_0 = 1/3, w_i = 1/6).
__host__ __device__ constexpr double lattice_w0(int nq) { return nq == 5 ? 1.0 / 3.0 : 0.25; }
__host__ __device__ constexpr double lattice_w1(int nq) { return nq == 5 ? 1.0 / 6.0 : 0.125; }
__host__ __device__ constexpr double lattice_eps(int nq) { return nq == 5 ? 1.0 / 3.0 : 0.25; }

// Face f = 2*a + h of axis a: h = 0 the low face (node 0, pulls direction
// +a), h = 1 the high face (node n_a - 1, pulls direction -a).
enum FaceKind : int32_t {
    kFacePeriodic = 0,   // same field, wrapped site, same direction
    kFaceMirror = 1,     // source field at the same site, reflected direction
    kFaceConj = 2        // OR-ed: take the complex conjugate of the source
};

// One field = one q-sample's magnetization (or one of its reflected image
// copies when a mirrored axis sees an oblique gradient) on one geometry.
struct FieldDesc {
    int64_t pop;            // element offset of the direction-0 plane
    int64_t words;          // offset of the geometry's site words
    int32_t n[3];           // sites per axis
    int32_t nsites;
    int32_t blk0;           // first workgroup of this field in a step launch
    int32_t nblk;           // workgroups of this field = tiles[0]*tiles[1]*tiles[2]
    int32_t q;              // signal row when this is a primary field, else -1
    int32_t zc;             // sites per thread along z (tile depth)
    int32_t tiles[3];       // tiles along x, y (of TX x TY sites) and z (of zc)
    int32_t tab;            // offset of this field's phase table (double2 entries):
                            //   [n0] exp(-i fdt c0 j0), [n1] exp(-i fdt c1 j1),
                            //   [n2] exp(-i fdt (c2 j2 + cu)), [6] face factors
    double c[3];            // reaction angle per unit step: -fdt*(c.j + cu)
    double cu;
    int64_t face_pop[6];    // direction-0 plane offset of each face's source field
    double beta[6];         // face factor exp(i * beta * F_k)
    int32_t face_kind[6];
    // Adjoint pull through face f (f = 2a+1 for direction +a at node n_a-1,
    // f = 2a for direction -a at node 0): the field whose adjoint is read,
    // how (kind), and where its forward coefficient sits in a step table.
    int32_t adj_kind[6];
    int64_t adj_pop[6];
    int32_t adj_fac[6];
    int64_t gm;             // offset of the geometry's membrane-position table
                            // ([6][nsites] floats, see StepArgs::gm), or -1
    int64_t cv;             // offset of the geometry's curved-link masks
                            // ([nsites] bytes, see StepArgs::cvm), or -1
    int32_t cv_h0, cv_nh;   // the geometry's curved links in cvh: first entry, count
};

// One term of a curved membrane link: the arriving population is
// sum_k w_k ghat(site + off_k) (off: element offset from the receiving
// site's direction-0 element, plane included), each times the factors of
// the periodic faces its node lies beyond: bits 2f, 2f + 1 of wrap count
// how often the factor of face f applies (a node one period below the
// lattice along kernel axis a takes face 2a once, one above takes 2a + 1).
struct CvTerm {
    double w;
    int32_t off;
    int32_t wrap;
};

constexpr int kAdjMaxPhase = 4;
// gradient accumulators per step: w[P], decay[P], trans[P*P], f, F
// with the gradient-strength sensitivities: + R_x, R_y, R_z, R_0, X_f[6]
constexpr int kNGGrad = 10;
constexpr int kNGMax = 2 * kAdjMaxPhase + kAdjMaxPhase * kAdjMaxPhase + 2 + kNGGrad;
// per-field constants of the gamma G0 gradient: q-sample, s_b [3],
// sigma_b [3], d beta_f / d G_b [6][3]
constexpr int kGMeta = 25;

struct AdjArgs {
    const void* lam_in;     // adjoint of the post-stream populations of step k (NULL: k = K)
    void* lam_out;          // same for step k-1
    const void* fwd;        // post-collision populations entering step k-1
    const uint32_t* words;
    const FieldDesc* fields;
    const int2* blk_field;    // per workgroup: field, block of the field (tile and z chunk)
    const double2* tab_prev;  // phase tables of step k-1
    const double2* tab_cur;   // phase tables of step k (face factors of its stream)
    const double* w;
    const double* decay;
    const double* trans;
    const double2* dLdE;    // [Q][K+1]
    double* gpart;          // [segment slot][blocks][NG] per-workgroup gradient sums
                            // (launch_adj_gsum adds them up per field)
    double dt;
    int32_t n_phase;
    int32_t k;
    int32_t K;
    int32_t top;            // 1 when k = K (no adjoint from later steps)
    int32_t ng;
    int32_t xcd;            // 1: XCD-contiguous workgroup order (xcd_tile)
    int32_t slot;           // slot of this step in gpart (k - 1 - first step of the segment)
    int32_t gradg;          // 1: also the gamma G0 sensitivities (ng includes kNGGrad)
    int32_t nq;             // 7 (D3Q7) or 5 (D2Q5 on a single layer)
};

struct StepArgs {
    const void* src;        // post-collision populations of step k (T*)
    void* dst;              // post-collision populations of step k+1
    const uint32_t* words;  // site words: bits 0-3 phase, bit 4+d-1 membrane on pull link d,
                            // bits 10+3(d-1).. the phase across that link
    const FieldDesc* fields;
    const int2* blk_field;  // per workgroup: field, block of the field (tile and z chunk)
    const double* fdt;      // [K] f_k * dt
    const double* Fk;       // [K+1] sum_{m<k} f_m dt
    const double* w;        // [P] 1/tau
    const double* decay;    // [P] exp(-dt/T2)
    const double* trans;    // [P*P] transmitted share 1/(1+P) of a membrane link
    double2* partial;       // [kTabSteps][blocks][kBlock/64] per-wave signal partial sums
                            // of step k in slot k mod kTabSteps (launch_esum adds them up)
    const double* rdt;      // [P] dt/T2 (classical scheme)
    // General membrane condition (theta = 0, membrane anywhere on the link):
    // gm[(d-1)*nsites + s] is, for the pull link of direction d into site s,
    // 0 when the half-link rule applies, else the link's membrane position
    // as given (v > 0: distance from s is v; v < 0: distance is 1 + v).
    const float* gm;
    const double* kdt;      // [P*P] kappa * dt
    // Membrane condition at any angle (curved membranes): bit d-1 of
    // cvm[f.cv + s] marks the pull link d of site s as one; cvh[k] = (first
    // term, count in cvt, receiving site's direction-0 element, pull
    // direction d) of link k.  k_links evaluates every such link of a field
    // into the destination state at (site, d) before the step, which then
    // reads it there.
    const uint8_t* cvm;
    const int4* cvh;
    const CvTerm* cvt;
    double edx;             // eps_D * dx
    double2* tab;           // phase table of step k (T entries); the table kernel
                            // fills kTabSteps consecutive steps from here
    const int32_t* tab_field;  // [T] field of each table entry
    int32_t T;              // entries per step
    int32_t n_phase;
    int32_t k;
    int32_t K;
    int32_t classical;      // 1: reaction term in the collision, no split
    int32_t nq;             // 7 (D3Q7) or 5 (D2Q5 on a single layer)
    int32_t xcd;            // 1: XCD-contiguous workgroup order (xcd_tile)
    int32_t first;          // 1: the step starts from the equilibrium state at M = 1,
                            // which src does not hold (hybrid scheme without curved
                            // links only; the step kernel uses the constants)
};

// Workgroup tile shapes (TX x TY threads, one site column along z each).
// kTile256x1 serves single-layer (D2Q5) lattices only, whose rows are walked
// as columns (see kernel_geom in the runtime).  kTileRows (3D lattices) cuts
// the x-y plane, read row after row, into runs of kBlock consecutive sites:
// no idle lanes where n0 is not a multiple of a tile width (kernel template
// TX = 0).
enum TileShape : int32_t {
    kTile64x4 = 0, kTile32x8 = 1, kTile16x16 = 2, kTile128x2 = 3, kTile256x1 = 4,
    kTileRows = 5, kTileCount = 6
};
// the shapes a 3D lattice may use, in the order ties are broken
constexpr int kShapes3D[] = {kTile128x2, kTile64x4, kTile32x8, kTile16x16, kTileRows};
constexpr int kShapeCount3D = 5;
inline void tile_dims(int shape, int* tx, int* ty) {
    *tx = shape == kTile64x4 ? 64 : shape == kTile32x8 ? 32 : shape == kTile128x2 ? 128
        : shape == kTile256x1 ? 256 : shape == kTileRows ? 0 : 16;
    *ty = *tx ? kBlock / *tx : 0;
}
// workgroups per z chunk of an n0 x n1 plane, as [x][y] tile counts
inline void tile_grid(int shape, int32_t n0, int32_t n1, int32_t* t0, int32_t* t1) {
    int tx, ty;
    tile_dims(shape, &tx, &ty);
    if (tx == 0) {
        *t0 = (int32_t)(((int64_t)n0 * n1 + kBlock - 1) / kBlock);
        *t1 = 1;
    } else {
        *t0 = (n0 + tx - 1) / tx;
        *t1 = (n1 + ty - 1) / ty;
    }
}

// Launchers (btl_kernels.hip, btl_adjoint.hip)
hipError_t launch_adj(int prec, int shape, const AdjArgs& a, int32_t n_blocks, hipStream_t st);
// gfield[(k_first + j) * nf_total + f_off + f][g] = sum over the workgroups of
// field f of gpart[j][.][g], j = 0 .. nsteps - 1, in a fixed order (f_off:
// position of the call's first field in a record that spans several calls)
hipError_t launch_adj_gsum(const double* gpart, const FieldDesc* d_fields, int32_t n_fields,
                           int32_t nblk_total, int32_t ng, int32_t k_first, int32_t nsteps,
                           double* gfield, int32_t f_off, int32_t nf_total, hipStream_t st);
// dgG0 (device [Q][3] or NULL) needs gmeta (device [n_fields][kGMeta]) and
// the per-step angles fdt [K] and F [K].  A non-finite gradient sets
// *nonfinite (device-visible, may be NULL).
// An empty one-wave kernel.  A timing event recorded right after it takes
// its timestamp from a launch that lasts a few microseconds, whatever time
// the runtime gives a marker (the end of the previous launch or its start).
hipError_t launch_mark(hipStream_t st);
hipError_t launch_adj_final(const double* gfield, int32_t K, int32_t n_fields, int32_t P,
                            double dt, double dx, const double* w, const double* T2,
                            const double* kappa, double* dD, double* dT2, double* dkappa,
                            double* df, int32_t sub, int32_t ng, const double* gmeta,
                            const double* fdt, const double* Fk, int32_t Q, double* dgG0,
                            double eps, int32_t yz_swap, int32_t* nonfinite, hipStream_t st);
// The equilibrium state at M = 1 in pop and E_0 = 1 of every q-sample;
// with pops false only E_0 (the first step then starts from the constants).
hipError_t launch_init(int prec, void* pop, int64_t n_elem_per_dir_total,
                       const FieldDesc* d_fields, int32_t n_fields,
                       const FieldDesc* h_fields, double* E, int32_t Q, int32_t K, int32_t nq,
                       hipStream_t st, bool pops = true);
hipError_t launch_step(int prec, int shape, const StepArgs& a, int32_t n_blocks, hipStream_t st);
// The arriving populations of the curved membrane links of every field into
// the destination state (a.dst), from a.src, for step a.k (face factors from
// a.tab); max_links bounds the links of one geometry.
hipError_t launch_links(int prec, const StepArgs& a, int32_t max_links, int32_t n_fields,
                        hipStream_t st);
// initial post-collision state of the classical scheme (depends on R at t^0)
// (fdt: the waveform table f_k dt, of which the kernel reads entry 0)
hipError_t launch_init_classical(int prec, void* pop, const FieldDesc* h_fields, int32_t n_fields,
                                 const uint32_t* words, const double* fdt, const double* rdt,
                                 int32_t nq, hipStream_t st);
// phase tables of steps a.k .. a.k + nsteps - 1 into a.tab[0 .. nsteps*T)
hipError_t launch_tables(const StepArgs& a, int32_t nsteps, hipStream_t st);
// signal E_{k+1} of steps k = k0 .. k0 + nsteps - 1 (nsteps <= kTabSteps) from
// the per-wave partial sums the step kernels left in partial; a non-finite
// signal value sets *nonfinite (device-visible, may be NULL)
hipError_t launch_esum(const double2* partial, const FieldDesc* d_fields, int32_t n_fields,
                       int32_t nblk_total, int32_t k0, int32_t nsteps, double* E, int32_t K,
                       int32_t* nonfinite, hipStream_t st);
hipError_t launch_mfinal(int prec, const void* pop, const FieldDesc* h_fields,
                         int32_t n_fields, void* M_out, int32_t nq, hipStream_t st);

}  // namespace btl
