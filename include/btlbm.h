/*
 * btlbm -- hybrid lattice Boltzmann solver of the Bloch-Torrey equation for
 * diffusion MRI in multiphase tissue (Naughton, Tennyson, Georgiadis,
 * arXiv:1907.00908), on AMD Instinct MI355X (gfx950).
 *
 * One call to btl_forward advances the complex transverse magnetization of
 * Q gradient samples ("q-samples") for K time steps on a D3Q7 lattice and
 * returns the signal after every step.  Each step is the paper's hybrid
 * scheme (Sec. 2.3, Eq. LBM_process_list_2):
 *   - BGK collision, g_eq = w_i M, tau = 1/2 + dt D / (eps_D dx^2),
 *     eps_D = 1/4, w_0 = 1/4, w_1..6 = 1/8      (Eqs. collision_LBM, g_eq, tau_def)
 *   - streaming                                  (Eq. streaming_LBM)
 *     with modified periodic outer faces        (Sec. 2.4.3, Eq. collision_BC)
 *     or mirroring outer faces                   (Sec. 2.4.4)
 *     and the half-link membrane condition on every link that joins two
 *     different compartments                    (Sec. 2.4.2, Eqs. B5, P_def,
 *                                                 permeability_BC)
 *   - reaction: gradient phase exp(-i gamma (x.G0) f_k dt) and T2 decay
 *     exp(-dt/T2)                                (Eqs. reaction_LBM, delta_phi)
 *   - signal E_k = mean over the REV of M = sum_i g_i  (Sec. 2.1, Eq. M'summation)
 * with M = 1 + 0i at t = 0 (Sec. 2.1).
 *
 * Units: um, ms.  D in um^2/ms, T2 in ms, permeability kappa in um/ms, the
 * gradient as gamma*G0 in rad/(um*ms).  Lattice node j on an axis sits at
 * x = j*dx (the origin, where G0.x = 0, is node 0).
 *
 * Mirroring faces with a gradient that is oblique to them (a case the paper
 * leaves open, Sec. 2.4.4) are computed as the reflected medium: the REV
 * mirrored across the face and tiled periodically.  The solver carries the
 * needed reflected copies of the field ("image fields", up to 4 per q-sample)
 * internally; for a gradient normal or parallel to the face this reduces
 * exactly to the paper's rule.
 *
 * Memory and streams: every pointer documented as "device" must be device
 * memory of the current HIP device; all work is enqueued on the given
 * hipStream_t (pass NULL for the null stream) and is asynchronous unless
 * stated otherwise.  Host pointers are read before the call returns.
 *
 * Errors: functions return a btl_status; nothing unwinds across this
 * interface.  btl_last_error returns a text describing the last failure of
 * that simulator.  A simulator is not thread-safe: use one per host thread.
 *
 * Non-finite results: the kernels that form the signal (Sec. 2.1) and the
 * gradients set a flag of the simulator when a value they write is not
 * finite (for instance when gamma G0, f and dt overflow a phase angle).
 * Because calls are asynchronous the flag is reported later: by
 * btl_synchronize, or by the first btl_forward, btl_forward_noalloc,
 * btl_backward or btl_autotune that finds it set when it starts, which then
 * returns BTL_E_NONFINITE without enqueuing work.  Reporting clears it.
 */
#ifndef BTLBM_H
#define BTLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct btl_sim btl_sim;

typedef enum {
    BTL_OK = 0,
    BTL_E_INVAL = 1,        /* invalid argument (message says which) */
    BTL_E_UNSUPPORTED = 2,  /* valid request the library does not implement */
    BTL_E_NOMEM = 3,        /* device memory exhausted */
    BTL_E_HIP = 4,          /* a HIP runtime call failed */
    BTL_E_NONFINITE = 5     /* an earlier call produced a non-finite signal value or
                               gradient (see btl_synchronize) */
} btl_status;

enum { BTL_PERIODIC = 0, BTL_MIRROR = 1 };   /* outer boundary per axis */
enum { BTL_F64 = 0, BTL_F32 = 1 };           /* population storage precision */
enum { BTL_HYBRID = 0, BTL_CLASSICAL = 1 };  /* time integration scheme */
enum { BTL_D3Q7 = 0, BTL_D2Q5 = 1 };         /* lattice */

/* One geometry: a compartment-label volume.  Every lattice link joining two
 * different compartments carries a membrane whose permeability is chosen by
 * the phases of the two compartments (Sec. 2.4.2; cell-to-cell membranes of
 * Sec. 3.6 are links between different compartments of one phase).  The
 * pointers are host memory and are copied by btl_create. */
typedef struct {
    int32_t n[3];               /* sites per axis, x fastest; n[0], n[1] >= 2,
                                 * n[2] >= 1 (1: a single layer) */
    double dx;                  /* lattice spacing, um, > 0 */
    int32_t bc[3];              /* BTL_PERIODIC or BTL_MIRROR per axis */
    int32_t n_comp;             /* number of compartments C >= 1 */
    const uint32_t *comp_id;    /* host [n2][n1][n0], values < C */
    const uint8_t *comp_phase;  /* host [C], values < n_phase */
    int32_t n_phase;            /* number of material phases P, 1..8 */
    const float *link_delta;    /* host [3][n2][n1][n0] or NULL: where each
                                 * membrane cuts its link (see below) */
    const float *link_normal;   /* host [3][3][n2][n1][n0] or NULL (needs
                                 * link_delta): the membrane's unit normal
                                 * where it cuts each link (see below) */
} btl_geom;

/* link_delta: entry [a][j] is the distance, in units of dx, from node j to
 * the membrane on the link j -> j + e_a (the last node of a periodic axis
 * links to node 0); it must lie in (0, 1) on every link that joins two
 * compartments and is not read elsewhere.  With it, a membrane link whose
 * stencil x - 2e_i .. x + e_i (i the direction entering x) lies inside the
 * lattice, with x + e_i in x's compartment and x - 2e_i in the other one,
 * takes the general membrane condition for a straight membrane normal to
 * the link at that position (Sec. 2.4.2, Eqs. B2a_text/B2b_text with the
 * theta = 0 coefficients of Eqs. B4a-B4c and the Dirichlet/Neumann
 * coefficients of Eqs. c_d, c_n):
 *   g'_i(x) = A_1 ghat_ibar(x) + A_2 ghat_ibar(x + e_i) + A_3 ghat_i(x)
 *           + B_1 ghat_i(x - e_i) + B_2 ghat_i(x - 2e_i) + B_3 ghat_ibar(x - e_i);
 * every other membrane link, and every link when link_delta is NULL, uses
 * the half-link form (Eqs. B5, permeability_BC: the membrane at mid-link).
 *
 * link_normal: entry [a][c][j] is component c of a unit normal (either
 * orientation) of the membrane on the link j -> j + e_a.  With it, a
 * membrane link takes the general condition for a membrane at any angle to
 * the link (Sec. 2.4.2, Appendix B): on each side the Dirichlet and Neumann
 * link relations (Eqs. dirichlet_1/2, neumann_1/2; coefficients Eqs. c_d,
 * c_n) give the value at the membrane and the inflow flux along the link;
 * the flux along each orthogonal lattice direction (one in 2D, two in 3D)
 * comes from the same relations with the coefficients for Delta_m = 0 on the
 * lattice line through the membrane point (Eqs. phi_1, phi_2), whose
 * populations at x' (the membrane point and one spacing from it along
 * e_betabar) are interpolated quadratically along the link direction from
 * the three nearest nodes of the same compartment; the normal inflow, their
 * combination with the normal's direction cosines, satisfies the
 * permeability condition with flux continuity on both sides (Eqs. B1, B1.5).
 * Stencils may reach through periodic faces (with the modified periodic
 * phase) but not through mirroring faces; a link without a complete stencil
 * keeps the rule above.  The weights depend on kappa, dt and the lattice;
 * they are built on the host (about 45 weights per link) when a forward's
 * constants differ from the last ones, after the work queued on its stream
 * has finished.
 * btl_backward does not support simulators whose forward used link_delta. */

/* Create a simulator for n_geom geometries (all with the same dx and
 * n_phase; sizes may differ: q-samples of all geometries run in one batch).
 * prec selects FP64 or FP32 population storage; the arithmetic of a forward
 * step is FP64 in both (the FP32 adjoint step computes per site in FP32),
 * and every sum (signal, gradients) is FP64.  On success *out owns all
 * device memory of the simulator; free it with btl_destroy.
 * Errors: BTL_E_INVAL (bad geometry), BTL_E_NOMEM, BTL_E_HIP. */
btl_status btl_create(const btl_geom *geoms, int32_t n_geom, int32_t prec,
                      btl_sim **out);

/* Run K steps for Q q-samples.
 *   dt      time step, ms, > 0
 *   D, T2   host [P] per-phase diffusivity (> 0) and T2 (> 0, +inf allowed)
 *   kappa   host [P*P] symmetric membrane permeability per phase pair,
 *           >= 0; +inf means no membrane between those phases
 *   q_geom  host [Q] geometry index of each q-sample
 *   gG0     host [Q][3] gamma*G0 of each q-sample
 *   f       host [K] waveform sample f_k applied on [k dt, (k+1) dt)
 *           (the same waveform for all q-samples); with m reaction
 *           sub-steps (btl_set_substeps) host [K*m], sample f[k m + j]
 *           applied on sub-step j of step k
 *   E       device [Q][K+1][2] doubles, caller-allocated: E[q][k] is the
 *           complex signal at t = k dt, E[q][0] = 1
 *   M_final device or NULL: the magnetization at t = K dt of every q-sample,
 *           complex in the storage precision (float2 or double2), q-samples
 *           concatenated, each [n2][n1][n0]
 *   ckpt_every  0: no adjoint tape; > 0: record a tape so that btl_backward
 *           can run afterwards.  When ceil(K/C) + C + 4 states (C =
 *           ckpt_every, one state = every field of every q-sample) fit the
 *           memory budget (btl_set_memory_budget), the state is kept every
 *           C steps; otherwise the tape is "deferred": only the inputs are
 *           kept and btl_backward replays the forward from t = 0 (the
 *           equilibrium at M = 1) in groups of q-samples with a binomial
 *           checkpointing schedule sized to the budget.  The gradients are
 *           the same either way.
 *   stream  hipStream_t or NULL
 * Batches whose two population copies exceed the budget run as consecutive
 * groups of q-samples ("q-waves") on the stream.
 * Errors: BTL_E_INVAL, BTL_E_UNSUPPORTED (a tape for a case the adjoint does
 * not cover: see btl_backward), BTL_E_NOMEM, BTL_E_HIP, BTL_E_NONFINITE. */
btl_status btl_forward(btl_sim *s, double dt, int32_t K, const double *D,
                       const double *T2, const double *kappa, int32_t Q,
                       const int32_t *q_geom, const double *gG0, const double *f,
                       double *E, void *M_final, int32_t ckpt_every, void *stream);

/* Gradients of a real loss L with respect to the inputs of the last
 * btl_forward that kept a tape (ckpt_every > 0); the adjoint of the hybrid
 * scheme (Sec. 2.3) with half-link membranes and at most 4 phases, on
 * either lattice.  dL_dE is device
 * [Q][K+1][2] with dL/dE = dL/dRe E + i dL/dIm E.  Outputs are device
 * doubles, overwritten (NULL = not wanted): dD [P], dT2 [P], dkappa [P*P],
 * df [K] (or [K*m] with m reaction sub-steps: dL per waveform sample),
 * dgG0 [Q][3] (dL/d(gamma G0) of each q-sample: through the reaction phase
 * gamma G.x and the face phase factors of Eqs. periodic_phi, collision_BC
 * and the mirror rule; asking for it runs a variant of the adjoint step with
 * ten more accumulators per workgroup).
 * dkappa is the gradient per matrix entry: for a != b the entries
 * [a][b] and [b][a] each hold half of dL/dkappa_ab, so that a symmetric
 * parametrization (both entries set from one value) gets the full value.
 * A deferred tape (see btl_forward) is reversed group by group; each group
 * replays its forward with binomial checkpointing (repetition number t and
 * s kept states reverse up to C(s + t, t) steps), so a backward can take a
 * few times the forward's steps.
 * Errors: BTL_E_INVAL (no tape), BTL_E_UNSUPPORTED (dgG0 asked of a tape
 * whose field set is not the full one: see btl_set_grad_gG0), BTL_E_NOMEM
 * (one q-sample's reverse sweep exceeds the budget), BTL_E_HIP,
 * BTL_E_NONFINITE. */
btl_status btl_backward(btl_sim *s, const double *dL_dE, double *dD, double *dT2,
                        double *dkappa, double *df, double *dgG0, void *stream);

/* What the last btl_backward of s did: the forward steps it recomputed, the
 * groups of q-samples it reversed one after another, and the states kept
 * per group by the binomial schedule (the smallest over the groups; 0 after
 * a uniform tape).  Host pointers, written on success; no device call.
 * Errors: BTL_E_INVAL (a NULL argument). */
btl_status btl_get_backward_stats(const btl_sim *s, int64_t *fwd_steps, int32_t *groups,
                                  int32_t *snapshots);

/* Device time of the adjoint steps of the last btl_backward of s (a uniform
 * tape): the elapsed time between HIP events recorded on its stream before
 * and after each segment's run of adjoint-step launches (the segment's
 * forward recompute and the gradient sums are outside them), summed over the
 * segments, and the number of adjoint steps they bracket.  Waits for those
 * events.  Host pointers, written on success.
 * Errors: BTL_E_INVAL (a NULL argument; no backward ran, or it replayed a
 * deferred tape, whose adjoint steps interleave with recomputes and are not
 * timed), BTL_E_HIP. */
btl_status btl_get_backward_timing(btl_sim *s, double *ms_adjoint, int64_t *adjoint_steps);

/* Select the lattice of later btl_forward calls.  BTL_D3Q7 (default):
 * eps_D = 1/4, w_0 = 1/4, w_i = 1/8.  BTL_D2Q5: the two-dimensional lattice
 * of Sec. 2.2 (Eq. omega_i: eps_D = 1/3, w_0 = 1/3, w_{1..4} = 1/6) on
 * single-layer geometries (n[2] = 1) with no gradient along z; eps_D enters
 * tau (Eq. tau_def) and the membrane number P (Eq. P_def), every other rule
 * is unchanged.  A D2Q5 forward returns BTL_E_INVAL for a geometry with
 * n[2] != 1 or a q-sample with gG0 z != 0.  btl_backward works on either
 * lattice; on D2Q5 the z component of dgG0 is 0 (not a parameter of the
 * layer).  Errors: BTL_E_INVAL (unknown lattice). */
btl_status btl_set_lattice(btl_sim *s, int32_t lattice);

/* Reaction sub-stepping (Sec. 2.3: the reaction may run with its own time
 * step dt' = dt/m while diffusion keeps dt).  Later btl_forward calls take
 * m waveform samples per step; step k applies the m reaction sub-steps
 * exp(-i gamma (x.G0) f[k m + j] dt') exp(-dt'/T2), j = 0..m-1, whose
 * product is one phase factor with the summed angle, and the modified
 * periodic and mirror phases use F advanced by the same sums.  m = 1 is the
 * default (dt' = dt).  Hybrid scheme only: a classical forward with m > 1
 * returns BTL_E_UNSUPPORTED.  Errors: BTL_E_INVAL (m outside 1..65536). */
btl_status btl_set_substeps(btl_sim *s, int32_t m);

/* Plan the fields of later taped btl_forward calls (ckpt_every > 0) so that
 * btl_backward can return dgG0 for every q-sample: every mirrored axis gets
 * its reflected image fields even where the q-sample has no gradient
 * component along it, and the conjugate pairing is kept only when all three
 * axes are mirrored (Sec. 2.4.4's mirror rule is exact for any G only with
 * the image fields a non-zero component would need).  Costs up to 2^3 fields
 * per q-sample instead of 1-4; on = 0 (default) plans the minimal set, with
 * which btl_backward returns dgG0 only where that set is already the full
 * one.  The signal is the same either way (the extra fields are exact
 * copies).  Errors: BTL_E_INVAL (on not 0 or 1). */
btl_status btl_set_grad_gG0(btl_sim *s, int32_t on);

/* Select the scheme of later btl_forward calls.  BTL_HYBRID (default) is
 * the paper's split scheme (Sec. 2.3).  BTL_CLASSICAL is the classical LBM
 * the paper compares it with (Appendix A, Eq. A12): no reaction split; the
 * collision carries dt w_i R M with R = -i gamma (x.G0) f(t^k) - 1/T2, and the
 * boundary and membrane rules are unchanged (mirrored faces with a gradient
 * component use the reflected medium, without the conjugate pairing that
 * only the split reaction makes exact).  btl_backward supports BTL_HYBRID
 * only.  Errors: BTL_E_INVAL (unknown scheme). */
btl_status btl_set_scheme(btl_sim *s, int32_t scheme);

/* Choose the launch shape (workgroup tile, z-column length and workgroup
 * order) of this simulator by timing every combination on the inputs of
 * the last btl_forward (its first Q q-samples, at most those whose states
 * fit device memory together -- one q-wave --, K_probe steps, waveform
 * repeated if shorter) and keeping the fastest.  Synchronizes the stream.
 * The probes are forwards of their own: the adjoint tape of an earlier
 * taped btl_forward is discarded, and the device memory of the probes'
 * states is freed before the call returns (the next forward allocates its
 * own).  The choice is remembered for the life of
 * the process, keyed by device, storage precision, lattice, scheme and the
 * sizes of the fields: a later call for the same shape of workload (on any
 * simulator) takes it without timing.  Without autotuning (or
 * btl_set_launch) a shape with the fewest idle lanes and whole z columns is
 * used.
 * Errors: BTL_E_INVAL (no previous forward, K_probe < 1), BTL_E_NOMEM,
 * BTL_E_HIP, BTL_E_NONFINITE. */
btl_status btl_autotune(btl_sim *s, int32_t Q, int32_t K_probe, void *stream);

/* Fix the launch shape of later forwards (as btl_autotune would set it):
 * tile_shape 0..5 as in btl_get_launch (-1: chosen per call; 4 is the
 * single-layer shape and 5 is for 3D lattices, other choices are replaced
 * by one that fits the lattice), zc the sites per thread along z (0: whole
 * columns, at most 1024), xcd the workgroup order: bit 0 the XCD-contiguous
 * numbering (neighbouring tiles of a field on one XCD), bit 1 the fields
 * that share a geometry interleaved block by block (so that the workgroups
 * running together read one block's site words, membrane positions and
 * term lists once for all those fields); 0..3, -1 by grid size.  Results do
 * not depend on the launch shape beyond the order of floating-point sums.
 * Errors: BTL_E_INVAL (a value out of range). */
btl_status btl_set_launch(btl_sim *s, int32_t tile_shape, int32_t zc, int32_t xcd);

/* Launch shape of the adjoint steps of later taped forwards: zc the sites
 * per thread along z (-1: chosen from the grid size, 0: whole columns, at
 * most 1024) and xcd the workgroup order (-1 by grid size, 0 plain, 1
 * XCD-contiguous).  Errors: BTL_E_INVAL (a value out of range). */
btl_status btl_set_adjoint_launch(btl_sim *s, int32_t zc, int32_t xcd);

/* Limit the device memory, in bytes, that later calls plan population
 * states into: the two copies of a forward (above it the q-samples run in
 * q-waves), the uniform tape and the snapshots of a reverse sweep.  0 (the
 * default) uses 85 % of the device memory that is free or already held by
 * the simulator's states.  Errors: BTL_E_INVAL (bytes < 0). */
btl_status btl_set_memory_budget(btl_sim *s, int64_t bytes);

/* 1 (default): forwards of at least 16 steps are captured once into a
 * hipGraph and replayed while their shape and buffers are unchanged (up to
 * four graphs per simulator, e.g. one per q-wave size); 0: every launch is
 * enqueued directly.  Results are identical either way.
 * Errors: BTL_E_INVAL (on not 0 or 1). */
btl_status btl_set_graphs(btl_sim *s, int32_t on);

/* Wait for the work enqueued on stream, then report a non-finite signal or
 * gradient produced since the last report (BTL_E_NONFINITE, which clears
 * it).  Errors: BTL_E_HIP, BTL_E_NONFINITE. */
btl_status btl_synchronize(btl_sim *s, void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): btl_forward
 * without tape (ckpt_every = 0), computed by the same kernels, with every
 * device buffer beyond E and M_final -- the two population copies, the
 * signal partials, the phase tables and the call's small tables -- in a
 * fixed device scratch array of 128 MiB that the library holds per device
 * for the life of the process.  Neither this call nor its kernels allocate
 * device or pinned memory: the tables travel through the pinned staging
 * that btl_create set up (1 MiB per slot, or larger after bigger btl_forward
 * calls); no q-waves and no hipGraph.  The scratch is shared by every call
 * on one device and keeps the last call's contents: calls that overlap on
 * one device (several streams or host threads) race and must be ordered by
 * the caller.  Arguments and results as btl_forward.  Geometries with
 * link_normal take the term tables of their membrane links from the device
 * buffers btl_forward made: new dt, kappa or lattice rebuild them in place
 * (the call then waits for the stream) when they fit, else the call fails.
 * Errors: BTL_E_INVAL (also when the call needs more than the scratch --
 * about 1.1e6 field-site states in FP32 storage -- or than the staging
 * holds; the message gives the sizes), BTL_E_UNSUPPORTED (membrane term
 * tables larger than those a btl_forward of this simulator built),
 * BTL_E_HIP, BTL_E_NONFINITE. */
btl_status btl_forward_noalloc(btl_sim *s, double dt, int32_t K, const double *D,
                               const double *T2, const double *kappa, int32_t Q,
                               const int32_t *q_geom, const double *gG0, const double *f,
                               double *E, void *M_final, void *stream);

/* The launch shape the forwards of s use, as set by btl_autotune or
 * btl_set_launch: the tile
 * shape (0 64x4, 1 32x8, 2 16x16, 3 128x2, 4 256x1, 5 runs of 256
 * consecutive sites; -1: chosen per call), the z-column length (0: whole
 * columns) and the workgroup order (0..3 as in btl_set_launch; -1: by grid
 * size).  Host pointers, written on success.  Makes no device call.
 * Errors: BTL_E_INVAL (a NULL argument). */
btl_status btl_get_launch(const btl_sim *s, int32_t *tile_shape, int32_t *zc, int32_t *xcd);

/* Release all memory of the simulator (synchronizes the device). */
void btl_destroy(btl_sim *s);

/* Text of the last error of s (or of the last failed btl_create when s is
 * NULL).  Owned by the library; valid until the next call on s. */
const char *btl_last_error(const btl_sim *s);

#ifdef __cplusplus
}
#endif

#endif /* BTLBM_H */
