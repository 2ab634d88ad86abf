/*
 * hyb.h -- C ABI of the MI355X library for the hybrid multi-time-step
 * FEM/LBM coupling of Karimi and Nakshatrala (arXiv:1601.02708).
 *
 * Problem (Sec. 6, eq. CouplingPDE): an advection-diffusion-reaction
 * equation on the square [0, L]^2 solved by bilinear (Q1) finite elements
 * (the coarse subdomain, Sec. 3), overlapped by a square patch of N x N
 * D2Q9 lattice nodes (the fine subdomain, Sec. 4) on which a lattice
 * Boltzmann method runs eta fine steps per coarse step.  The two exchange
 * Dirichlet data (Secs. 5 and 6.2) inside the Schwarz iteration of
 * Algorithm 1.  Everything is in lattice units: fine spacing 1, fine step
 * 1, coarse step eta.
 *
 * Geometry: fine node (i, j), 0 <= i, j < N, sits at (x0 + i, y0 + j); the
 * mesh has M x M squares of side L/M, node (k, l) at (k L/M, l L/M).  The
 * fine interface Gamma_{c->f} is the whole lattice perimeter: 4(N-1)
 * "perimeter slots" numbered along the bottom row (j = 0, i = 0..N-1), the
 * top row (j = N-1, i = 0..N-1), the left column (i = 0, j = 1..N-2) and the
 * right column (i = N-1, j = 1..N-2).  The coarse interface Gamma_{f->c} is
 * the set of mesh nodes inside the patch at least `overlap_elems` elements
 * from its boundary; together with the outer edge of the mesh these nodes
 * carry strong Dirichlet data.
 *
 * Memory: host arrays passed to hyb_create are copied and may be freed
 * after it returns.  Device memory is owned by the caller: three population
 * buffers of hyb_query()'s f_bytes and one workspace of ws_bytes, all
 * 256-byte aligned, which must outlive the handle.  The library allocates
 * no device memory (a handle holds a small pinned host buffer for the
 * commit's read-back, a second stream and events).  Every call enqueues
 * work on the lattice's stream and
 * returns without waiting, except hyb_commit, hyb_stats, hyb_concentration,
 * hyb_get_populations, hyb_set_populations and hyb_create, which synchronise
 * that stream.  A handle is not thread-safe.
 *
 * Errors: every int-returning call returns HYB_OK (0) or a negative code;
 * hyb_last_error() describes the last failure on the handle.  After
 * HYB_EHIP the handle's device state is undefined.
 */
#ifndef HYB_H
#define HYB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HYB_OK = 0,
    HYB_EINVAL = -1,       /* invalid argument or call order */
    HYB_EHIP = -2,         /* a HIP runtime call failed */
    HYB_ENOCONV = -3,      /* coarse solve did not reach its tolerance */
    HYB_ENONFINITE = -4    /* a NaN/Inf concentration appeared in the lattice */
};

/* Population storage and arithmetic.  HYB_FP64, HYB_FP32: stored and
 * computed in that precision.  HYB_FP16S: FP16 shifted storage -- each
 * population is stored as the binary16 value g = (f - w_q c_ref) * 2^s
 * (round to nearest even), where c_ref is the mean of u0 over the fluid
 * nodes and 2^s the largest power of two with (4/9) U 2^s <= 16384,
 * U = max(1, max |u0 - c_ref|), both fixed at hyb_create; arithmetic in
 * FP32, closures in FP64; a sweep launch that takes several fine steps
 * keeps its intermediate states in FP32 on chip and rounds to binary16 only
 * when it stores, so results depend on the steps per launch to within a
 * few binary16 roundings.  Concentrations beyond about 4.5 U from c_ref
 * overflow binary16 and are reported as non-finite (by the commit of the
 * coarse step whose fine steps read the overflowed value). */
enum { HYB_FP64 = 0, HYB_FP32 = 1, HYB_FP16S = 2 };
enum { HYB_F2C = 0, HYB_C2F = 1 };              /* hyb_interface_exchange direction */
enum { HYB_FINE = 0, HYB_COARSE = 1 };          /* hyb_concentration field */
enum { HYB_BC_DIRICHLET = 0, HYB_BC_NEUMANN = 1 };
enum { HYB_OVERLAP_AUTO = -1 };                  /* hyb_set_overlap: tune the depth */

typedef struct hyb_handle hyb_handle;

/* Coarse mesh (Sec. 3, Sec. 6.1).  May be NULL in hyb_create: the handle is
 * then lattice-only and its interface data come from hyb_set_boundary. */
typedef struct {
    int M;                  /* elements per side, >= 2 */
    double L;               /* side of the coarse domain [0, L]^2 */
    double outer_value;     /* Dirichlet value on the outer edges (those not natural) */
    int overlap_elems;      /* width of the overlap strip in elements, >= 1 */
    int supg;               /* 0: Galerkin, eq. (Galerkin); 1: SUPG, eqs. (SUPG), (SUPG_tau) */
    const double *d0;       /* host [(M+1)^2] initial nodal concentration, index l*(M+1)+k */
    int outer_natural;      /* bit e set: outer edge e (0: x = 0, 1: x = L, 2: y = 0, 3: y = L)
                               takes the natural condition of the weak form (zero diffusive
                               flux) instead of the Dirichlet value; 0: all four Dirichlet */
} hyb_mesh;

/* Fine lattice (Sec. 4.1). */
typedef struct {
    int N;                  /* nodes per side, >= 3 */
    double x0, y0;          /* domain coordinates of node (0, 0) */
    int precision;          /* HYB_FP64, HYB_FP32 or HYB_FP16S */
    double tau;             /* BGK relaxation time; <= 0 selects 1/2 + 3 D (Sec. 4.1) */
    int eta;                /* fine steps per coarse step, >= 1 */
    int bc_clamp;           /* maxent Dirichlet closure, eq. (LBM_Dir): 0 applied as
                               printed, 1 unknowns clamped at 0 when the closure would
                               make them negative */
    const uint8_t *solid;   /* host [N*N], 1 = solid node, index j*N+i; NULL = none.
                               Solid nodes on the perimeter are rejected. */
    const double *u0;       /* host [N*N] initial concentration (ignored at solid nodes) */
    void *f_buf[3];         /* device population buffers, each >= f_bytes */
    void *workspace;        /* device workspace, >= ws_bytes */
    void *stream;           /* hipStream_t for all work; NULL = default stream */
    int dissolution;        /* 1: reserve the workspace of dissolving solids
                               (hyb_set_dissolution); 0: solids are fixed */
    int wall_closure;       /* 1: reserve the workspace of the maximum-entropy
                               closure at solid walls (hyb_set_wall_normals) */
} hyb_lattice;

/* Advection velocity (divergence-free in the continuum, eq. AD). */
typedef struct {
    const float *fine;      /* host [2][N*N]: x plane then y plane, lattice units per fine step */
    const double *coarse;   /* host [(M+1)^2][2] nodal velocity of the mesh (ignored without mesh);
                               inside an element the velocity is its bilinear interpolant */
} hyb_velocity;

/* First-order reaction s = -k u (per unit time; the fine step is 1). */
typedef struct {
    double k;               /* uniform rate, 0 <= k < 1 */
    const double *k_field;  /* host [N*N] per-node fine rate in [0, 1), or NULL for the uniform k;
                               the coarse model always uses the uniform k */
} hyb_reaction;

typedef struct {
    int64_t infeasible;     /* cumulative count of closures whose unknowns would be negative
                               (Dirichlet) or that have no solution (Neumann) */
    int64_t nonfinite;      /* non-finite concentrations seen by the fine kernels */
    int32_t krylov_iters;   /* iterations of the last coarse solve */
    int32_t krylov_converged;
    double krylov_relres;   /* ||b - A x|| / ||b|| of the last coarse solve */
    int64_t coarse_steps;   /* committed coarse steps */
    int64_t fine_steps;     /* fine steps run since creation (all Schwarz passes) */
    int32_t overlap_depth;  /* overlap depth hyb_step uses (-1 while it is still being tuned) */
    int32_t pad;
    /* diagnostics of the current fine state, as hyb_diagnostics out[0..2] */
    double mass;            /* sum over fluid nodes of the concentration */
    double min_f;           /* smallest post-collision population at a fluid node */
    double h_function;      /* Boltzmann H of eq. (BH) over the fluid nodes */
} hyb_run_stats;

/* Device memory the caller must provide for this problem. */
int hyb_query(const hyb_mesh *mesh, const hyb_lattice *lattice, size_t *f_bytes, size_t *ws_bytes);

/* Build a handle: validates the inputs, uploads geometry, velocity and the
 * static interface lists, assembles and preconditions the coarse system
 * A = (M + Ms) + eta/2 (K + Ks), B = (M + Ms) - eta/2 (K + Ks) (trapezoidal
 * rule, eq. FEM_discrete, theta = 1/2) and initialises f*(0) = collide(f^eq(u0))
 * (Sec. 6.2, item i) and d(0) = d0.  D is the diffusion coefficient (> 0). */
int hyb_create(const hyb_mesh *mesh, const hyb_lattice *lattice, double D,
               const hyb_velocity *u, const hyb_reaction *k, hyb_handle **out);

/* HYB_F2C: bilinear interpolation of the current lattice concentration at
 * the Gamma_{f->c} mesh nodes (Sec. 6.2, item ii).  Solid corners are left
 * out with the remaining weights rescaled; a node with four solid corners
 * takes the nearest fluid node.
 * HYB_C2F: FEM interpolant of d(t_n) and of the latest coarse solution at
 * every perimeter slot (the two time levels of eq. MTS). */
int hyb_interface_exchange(hyb_handle *h, int direction);

/* One trapezoidal coarse step from the committed d(t_n) with the Dirichlet
 * data of the last HYB_F2C exchange (Algorithm 1, "advance the solution in
 * Omega_c").  Solved on the GPU by right-preconditioned BiCGSTAB (sparse
 * approximate inverse) in FP64 to ||r|| <= 1e-14 ||b||, at most max_iter
 * iterations (<= 0: 200).  Does not commit. */
int hyb_coarse_step(hyb_handle *h, int max_iter);

/* n_sub fine steps (Sec. 4.1, eqs. LBE, Collision): pull streaming with
 * halfway bounce-back at solids, the maxent closure at the perimeter with
 * the interface value of eq. (MTS), (1 - j/eta) a + (j/eta) b at fine step
 * j, and BGK collision with the reaction source -k w_i u.  restart = 1
 * starts from the committed state f*(t_n) at j = 0 (a new Schwarz
 * iteration); restart = 0 continues.  j may not pass eta. */
int hyb_lbm_substeps(hyb_handle *h, int n_sub, int restart);

/* End the coarse step: checks the device error counters (synchronises),
 * then makes the last fine state and coarse solution the committed state.
 * Returns HYB_ENONFINITE / HYB_ENOCONV (state left uncommitted) on failure. */
int hyb_commit(hyb_handle *h);

/* Algorithm 1 for one coarse step: max_schwarz times {F2C exchange, coarse
 * step, C2F exchange, eta fine steps from f*(t_n)}, then commit. */
int hyb_step(hyb_handle *h, int max_schwarz);

/* Lattice-only use and tests: per-slot closure kind (HYB_BC_*, NULL = all
 * Dirichlet) and its values at the start (a) and end (b) of the coarse step
 * (concentration for Dirichlet, outward normal flux sum_i f_i e_i.n for
 * Neumann).  Host arrays of 4(N-1) entries; b == NULL means b = a.  A later
 * HYB_C2F exchange overwrites a and b. */
int hyb_set_boundary(hyb_handle *h, const int8_t *kind, const double *a, const double *b);

/* Concentration readout (synchronises): HYB_FINE -> out[N*N] = sum_i f*_i / (1 - k)
 * of the current fine state (0 at solid nodes); HYB_COARSE -> out[(M+1)^2] =
 * latest coarse solution.  out_is_device: out is a device pointer. */
int hyb_concentration(hyb_handle *h, int which, double *out, int out_is_device);

/* Populations of the current fine state as host FP64 [9][N*N] (get), or
 * replace the committed state f*(t_n) with them (set; cast to the storage
 * precision).  Velocity order: rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-). */
int hyb_get_populations(hyb_handle *h, double *out);
int hyb_set_populations(hyb_handle *h, const double *f);
/* The current fine state into device FP64 [9][N][N] (index (q*N + j)*N + i)
 * on the handle's stream, no synchronisation; HYB_FP64 and HYB_FP32 storage
 * only; values at solid nodes are unspecified. */
int hyb_populations_device(hyb_handle *h, double *out);

/* Replace the committed coarse solution d(t_n) with host FP64 d[(M+1)^2]
 * (node l*(M+1) + k); also taken as d(t_{n-1}) by the next step's
 * extrapolated first guess.  Like hyb_set_populations it abandons a coarse
 * step in progress.  Synchronises. */
int hyb_set_coarse(hyb_handle *h, const double *d);

/* Controls of the reverse mode, replaced between steps without re-creating
 * the handle (the committed state is left as it is):
 *   hyb_set_reaction_field: the fine per-node rate k of the reaction source
 *     s = -k u (eq. CouplingPDE, Sec. 4.1), host FP64 [N*N] (node j*N + i),
 *     every value in [0, 1), else HYB_EINVAL and nothing changes; stored in
 *     the storage precision's arithmetic type (FP64 for HYB_FP64, FP32
 *     otherwise); also allowed on a handle created with a uniform k, which
 *     then uses the field.  The coarse model keeps the uniform k.
 *     Synchronises.
 *   hyb_set_outer_value: the Dirichlet value of the outer edges that are not
 *     natural (hyb_mesh.outer_value; a strong Dirichlet row of eq.
 *     FEM_discrete), finite, taken by the next coarse solve; HYB_EINVAL
 *     without a coarse mesh. */
int hyb_set_reaction_field(hyb_handle *h, const double *k_field);
int hyb_set_outer_value(hyb_handle *h, double value);

/* Counters, the last coarse solve's result and the diagnostics of the
 * current fine state (runs hyb_diagnostics).  Synchronises. */
int hyb_stats(hyb_handle *h, hyb_run_stats *out);

/* Diagnostics of the current fine state f* (the committed state after
 * hyb_commit, else the latest fine step), over the fluid nodes (Sec. 4.1):
 *   out[0] = sum of the concentration u = sum_q f*_q / (1 - k)   (eq. LBM_Macro
 *            with the reaction readout; the lattice's mass),
 *   out[1] = smallest post-collision population f*_q (non-negativity, eq. NN_Cond),
 *   out[2] = H = sum_q f*_q ln(f*_q / w_q) over f*_q > 0         (eq. BH),
 *   out[3] = number of nodes holding a non-finite population.
 * FP64 from the decoded stored values; the sums run in a fixed order, so the
 * values are reproducible.  out: 4 doubles, host (out_is_device = 0: the
 * call synchronises) or device (the call only enqueues work on the handle's
 * stream).  Row partials use the handle's workspace, so calls on one
 * handle are serialised by its stream. */
int hyb_diagnostics(hyb_handle *h, double *out, int out_is_device);

/* hyb_diagnostics for callers that cannot allocate or synchronise (code
 * under HIP graph capture, tight serving loops): the same kernels and
 * results as hyb_diagnostics(h, out, 1), with the row partials in a static
 * device array of the library instead of the handle's workspace.  out:
 * device, 4 doubles as above; the call only enqueues work on the handle's
 * stream and allocates nothing.  Limit: N <= 16384 (HYB_EINVAL beyond).
 * The array is one per device and shared by every call on that device, so
 * calls on one device whose work may overlap (several handles on different
 * streams) race; serialise them.  Each call overwrites every partial it
 * reads. */
int hyb_diagnostics_noalloc(hyb_handle *h, double *out);

/* ---- differentiation form (reverse mode) of the fine sub-steps ----------
 *
 * The fine step (Sec. 4.1: pull streaming with halfway bounce-back, the
 * Dirichlet closure of eq. (LBM_Dir) with u^p from eq. (MTS), BGK collision
 * with the reaction source) is linear in (f*, u^p) for fixed velocity and
 * reaction rate when the closure is applied as printed; where the clamp
 * option zeroes a closure its unknowns are constant.  The adjoint maps
 * dJ/df* at the end of n_sub fine steps to dJ/df* at the committed state
 * f*(t_n) and accumulates dJ/da, dJ/db (the two interface arrays of
 * hyb_set_boundary / hyb_interface_exchange, u^p = (1 - j/eta) a + (j/eta) b
 * at fine step j) and dJ/dk (per-node reaction rate).  Supported for
 * HYB_FP64 and HYB_FP32 storage (arithmetic in that precision) with every
 * perimeter slot Dirichlet; HYB_EINVAL otherwise.
 *
 * hyb_adjoint_query: device bytes of the tape for n_sub >= 1 fine steps,
 *   (n_sub + 4) population buffers (f_bytes each) and n_sub planes of the
 *   arithmetic type.
 * hyb_lbm_substeps_record: like hyb_lbm_substeps(h, n_sub, 1), recording
 *   the intermediate states f*(1) .. f*(n_sub - 1) and, without dissolving
 *   solids, u of each fine step's collision (the reversed steps read it for
 *   dJ/dk) in the caller's device tape (256-byte aligned, >= tape bytes);
 *   f*(0) and f*(n_sub) stay in the handle's committed and current buffers.
 *   1 <= n_sub <= eta.
 * hyb_lbm_adjoint: tape and n_sub of the last record; the handle must be
 *   unchanged since (HYB_EINVAL after any call that steps, commits, or sets
 *   populations, interface values or rates); lam_in, lam_out: device FP64
 *   [9][N][N] (index (q*N + j)*N + i), lam_in = dJ/df*(n_sub) (kept),
 *   lam_out = dJ/df*(0) (may alias lam_in); grad_a, grad_b: device FP64
 *   [4(N-1)] and grad_k: device FP64 [N*N] or NULL, each ADDED to.  The
 *   tape's last three buffers are scratch.  Enqueued on the handle's stream;
 *   no synchronisation. */
int hyb_adjoint_query(const hyb_handle *h, int n_sub, size_t *tape_bytes);
int hyb_lbm_substeps_record(hyb_handle *h, int n_sub, void *tape);
int hyb_lbm_adjoint(hyb_handle *h, int n_sub, const void *tape, const double *lam_in, double *lam_out,
                    double *grad_a, double *grad_b, double *grad_k);

/* ---- differentiation form of one whole coarse step (Algorithm 1) -------
 *
 * One coarse step with a fixed number of Schwarz passes maps the committed
 * state (f*(t_n), d^n) to (f*(t_{n+1}), d^{n+1}) through the fine steps
 * above, the coarse-to-fine interpolation (Sec. 6.2 item i), the
 * trapezoidal coarse step with strong Dirichlet rows (eq. FEM_discrete) and
 * the fine-to-coarse transfer (Sec. 6.2 item ii); with the closure applied
 * as printed the map is affine, and its adjoint runs the passes backwards
 * through the transposes of those pieces (the coarse solve transposed as
 * (A P)^T mu = P^T lam by the same BiCGSTAB kernels, FP64).
 * Same storage and boundary restrictions as the fine-step adjoint; a coarse
 * mesh is required.
 *
 * hyb_step_adjoint_query: device bytes of the tape for `passes` >= 1.
 * hyb_step_record: hyb_step(h, passes) run with one- and two-step
 *   launches, recording the fine states (and, without dissolving solids, u
 *   of each fine step's collision), interface arrays and the state the
 *   transfers read in the caller's device tape (256-byte aligned); f*(t_n)
 *   and the step's end state stay in the handle's buffers.  Commits the step
 *   as hyb_step does (same errors; nothing is recorded on an error).
 * hyb_step_adjoint: for the last record (tape pointer of that call; the
 *   handle must be unchanged since, HYB_EINVAL after any call that steps,
 *   commits, or sets populations, interface values or rates):
 *   lam_f = dJ/df*(t_{n+1}) (device FP64 [9][N][N], index (q*N + j)*N + i),
 *   lam_sub = the cotangent of every intermediate fine state of the
 *   committed (last) pass, f*(t_n + j) for j = 1 .. eta-1 (same layout, or
 *   NULL for none: an objective that integrates over every fine step
 *   passes its per-state weight here and in lam_f),
 *   lam_d = dJ/dd^{n+1} (device FP64 [(M+1)^2], mesh node l*(M+1) + k, or
 *   NULL for zero); writes lam_f_out = dJ/df*(t_n) (may alias lam_f) and
 *   lam_d_out = dJ/dd^n; grad_k (device FP64 [N*N] or NULL) += dJ/dk of the
 *   fine per-node reaction rate; grad_outer (device FP64 [(M+1)^2] or NULL)
 *   += dJ/dg for the value g each outer-edge node of the coarse mesh is held
 *   at during the step (zero elsewhere; the control of a prescribed inlet).
 *   Synchronises; HYB_ENOCONV if a transposed coarse solve does not reach
 *   1e-14 relative residual. */
int hyb_step_adjoint_query(const hyb_handle *h, int passes, size_t *tape_bytes);
int hyb_step_record(hyb_handle *h, int passes, void *tape);
int hyb_step_adjoint(hyb_handle *h, const void *tape, const double *lam_f, const double *lam_sub, const double *lam_d,
                     double *lam_f_out, double *lam_d_out, double *grad_k, double *grad_outer);

/* Overlap in hyb_step (default HYB_OVERLAP_AUTO): with multi-step
 * launches (hyb_set_steps_per_launch), the deep interior tiles of each
 * Schwarz pass's first `depth` launches run on a second stream owned by the
 * handle while the pass's fine-to-coarse transfer, coarse solve and
 * coarse-to-fine transfer run on the caller's stream; the remaining tiles
 * follow on the caller's stream.  Launch j (j = 0 .. depth-1, its fine
 * steps) splits at the rectangle of tiles whose ring (one node, or K-1 in
 * passes with K-step launches) stays clear of the patch perimeter, shrunk by j tiles on every side: such tiles read no interface
 * value and, with their halo, only the deep tiles of launch j-1.  Depth is
 * capped at D, the pass's number of leading multi-step launches (eta / 2
 * with pairs; at eta = 10, 4 with 3 + 3 + 2 + 2, 3 with 4 + 3 + 3 and 2 with
 * 5 + 5).  Results are bit-identical to the serial order for every depth.
 * depth = 0 runs everything on the caller's stream.  HYB_OVERLAP_AUTO: of
 * the handle's next 1 + 3 (D + 1) successful hyb_step calls, the first runs
 * serially and the others at depths 0 .. D three times over, each timed on
 * the caller's stream; later calls use the depth with the fastest step;
 * hyb_stats reports the depth (-1 while tuning).  Other negative depths:
 * HYB_EINVAL. */
int hyb_set_overlap(hyb_handle *h, int depth);

/* Most fine steps per lattice-sweep launch (1 to 5; default 5 for HYB_FP32,
 * 4 for HYB_FP64 and HYB_FP16S storage, the fastest measured for each).  With 2 or
 * more, while every perimeter slot is Dirichlet, hyb_lbm_substeps takes fine
 * steps in temporally blocked launches (the state between the steps of one
 * launch stays on chip), never leaving a lone single step where it can be
 * avoided: with 2, in pairs; with 3, in threes, a remainder of 4 taken as
 * two pairs (eta = 10: 3 + 3 + 2 + 2); with 4, in fours, remainders of 5 and
 * 6 starting with a three (eta = 10: 4 + 3 + 3); with 5, in fives,
 * remainders of 6, 7, 8 and 9 as 3 + 3, 4 + 3, 4 + 4 and 5 + 4 (eta = 10:
 * 5 + 5).  A remaining single step, and
 * every step when some slot is Neumann, the wall closure is on, or a
 * population buffer reaches 4 GiB (the multi-step kernels use 32-bit byte
 * offsets), uses the single-step sweep.  Results agree with the single-step
 * path to rounding (same operations per node; pairs give its bits, and
 * three- to five-step launches FP64 states identical to pairs' and FP32
 * ones within a few ulp, from the compiler's fusing of multiply-adds; FP16
 * shifted storage rounds to binary16 once per launch instead of once per
 * step).  With 2 or more, hyb_lbm_adjoint and hyb_step_adjoint also reverse
 * fine steps in pairs, one launch each (same bits as single reversed
 * steps).  Returns HYB_EINVAL for other values.  Takes effect at the next
 * hyb_lbm_substeps or adjoint call and restarts the overlap tuning of
 * HYB_OVERLAP_AUTO. */
int hyb_set_steps_per_launch(hyb_handle *h, int steps);

/* Measurement: while enabled, every hyb_lbm_substeps call records HIP
 * events on the handle's stream around its lattice-sweep kernels: one pair
 * around the whole batch when all perimeter slots are Dirichlet (only sweep
 * kernels are launched, back to back), else one pair around each
 * interior-node kernel.  hyb_kernel_time returns the summed elapsed
 * milliseconds and the number of sweep launches they cover since the last
 * call, and synchronises. */
int hyb_kernel_timing(hyb_handle *h, int enable);
int hyb_kernel_time(hyb_handle *h, double *total_ms, int64_t *launches);

/* ---- dissolving solids ---------------------------------------------------
 *
 * An extension of the pore-scale setting of Sec. 7.4, whose solids stay
 * fixed: each solid node holds a mass, and the halfway bounce-back of
 * Sec. 4.1 carries a first-order surface reaction.  A population returned
 * across a fluid-solid link relaxes towards w_q c_sat,
 *   f_q(x) = (1 - kappa_s) f*_opp(q)(x) + kappa_s w_q c_sat,
 * and the link moves kappa_s (w_q c_sat - f*_opp(q)(x)) into the fluid,
 * taken from the solid node.  The geometry is frozen within a coarse step:
 * every Schwarz pass sums the link fluxes of its fine steps per solid node,
 * and the commit debits the last pass's sums from the masses.  A solid
 * whose mass is then <= 0 becomes fluid with f*_q = w_q u_mean (1 - k),
 * u_mean the mean concentration of its fluid neighbours (8-neighbourhood,
 * before the commit), at zero velocity.  With the workspace reserved
 * (hyb_lattice.dissolution = 1) the fine-to-coarse transfer (Sec. 6.2 item
 * ii) weights the current fluid corners, sum w_m u_m / sum w_m over the
 * fluid ones; a coarse node none of whose fluid corners carries weight
 * keeps the nearest fluid node of the initial geometry.  While the
 * reaction is on, hyb_step runs without overlap (whole-patch launches).
 *
 * hyb_set_dissolution: reaction rate 0 <= kappa_s <= 1 (0 switches the
 *   reaction and the mass bookkeeping off), c_sat finite, mass host FP64
 *   [N*N] (index j*N + i, read at solid nodes; NULL keeps the current
 *   masses, 0 after hyb_create).  Only between coarse steps (no fine steps
 *   pending); HYB_EINVAL without the reserved workspace.  Synchronises.
 * hyb_dissolution_state: current solid flags (host u8 [N*N]), masses (host
 *   FP64 [N*N], 0 at fluid nodes) and the number of nodes solid at
 *   hyb_create that are fluid now (the conversions so far: fluid never turns
 *   solid); each output may be NULL.  Synchronises.
 * hyb_set_solids: replace the geometry and masses (host u8 / FP64 [N*N],
 *   e.g. a checkpoint taken with hyb_dissolution_state): only nodes solid at
 *   hyb_create may be solid (HYB_EINVAL otherwise); the flag words are
 *   rebuilt; only between coarse steps.  Synchronises.
 * Reverse mode: the fine-step adjoint carries the link factor 1 - kappa_s
 * (the recorded steps also sum the link fluxes).  hyb_step_record records
 * the step's flag words and the solids left by its commit; hyb_step_adjoint
 * then reverses the step on that geometry, with the commit's conversion
 * transposed for its set of converted nodes (a converted node's cotangent
 * reaches its fluid neighbours through their mean concentration, and the
 * (1 - k) factors enter dJ/dk); the conversion decision itself and the
 * masses are not differentiated (piecewise constant). */
int hyb_set_dissolution(hyb_handle *h, double kappa_s, double c_sat, const double *mass);

/* Maximum-entropy Neumann closure at the walls of the solid grains (Sec.
 * 4.1.1, eq. LBM_Neu, with zero prescribed flux: an impermeable wall) in
 * place of halfway bounce-back.  An interior fluid node (1 <= i, j <= N-2)
 * with solid upstream nodes is a boundary point with normal n: all its
 * populations with e_q.n < 0 (the set M- of the paper) become
 * w_q exp(-1 - gamma e_q.n), gamma from an FP64 Newton solve of the flux
 * condition sum_q (e_q.n) f_q = 0, and populations streamed from a solid
 * node with e_q.n >= 0 (links the wall grazes) are bounced back.  No
 * solution (the other populations carry no flux into the wall) sets M- to
 * 0 and counts the node as infeasible.  Perimeter nodes keep their own
 * closure.
 * normals: host [2][N*N] FP32 (x plane, then y plane): the unit outward
 * normal of the fluid domain (pointing into the solid) at every fluid node
 * that has a solid neighbour, unit length within 1e-3, else HYB_EINVAL;
 * other entries are ignored.  NULL switches back to bounce-back.  Needs
 * hyb_lattice.wall_closure = 1 at creation and no pending fine steps; not
 * with dissolving solids or the reverse mode (HYB_EINVAL).  Runs the
 * single-step sweeps.  Synchronises. */
int hyb_set_wall_normals(hyb_handle *h, const float *normals);
int hyb_dissolution_state(hyb_handle *h, uint8_t *solid, double *mass, int64_t *converted);
int hyb_set_solids(hyb_handle *h, const uint8_t *solid, const double *mass);

/* Checkpoint and restore on the device: the committed state between coarse
 * steps -- populations f*(t_n) in their storage format, the coarse
 * solutions d(t_n) and d(t_{n-1}) (the next step's first guess extrapolates
 * from both), and with dissolving solids the flag words, solid flags and
 * masses -- copied into or out of a caller's device buffer (256-byte
 * aligned, hyb_checkpoint_query bytes; the layout is internal to the
 * library).  A run continued from a loaded checkpoint repeats the original
 * run bit for bit.  Save needs no pending fine steps; load abandons a coarse
 * step in progress.  Both enqueue device copies on the handle's stream and
 * return without waiting. */
int hyb_checkpoint_query(const hyb_handle *h, size_t *bytes);
int hyb_checkpoint_save(hyb_handle *h, void *ckpt);
int hyb_checkpoint_load(hyb_handle *h, const void *ckpt);

/* ---- several fine patches around one coarse subdomain -----------------
 *
 * Algorithm 2 (Sec. 6.3) with one coarse subdomain: every Schwarz iteration
 * advances the coarse subdomain first, with each patch's transferred values
 * from the previous iteration (the first from the patches' states at t_n),
 * then advances every patch by eta fine steps from t_n with eq. (MTS) at its
 * own perimeter.  The coarse Dirichlet rows are the outer edges and, per
 * patch, the coarse nodes inside it at least overlap_elems elements from its
 * boundary (patches must not share such a node).
 *
 * The patches are handles created with mesh = NULL (their lattice's x0, y0
 * place them in the coarse domain), every perimeter slot Dirichlet, fixed
 * solids, one eta and the group's stream; the group writes their interface
 * arrays a, b (as hyb_set_boundary would) and commits them.  The group owns
 * the coarse operator (assembled like hyb_create's from D, the nodal
 * velocity vcoarse [(M+1)^2][2] and the uniform rate k) and per patch the
 * transfer lists, in the caller's device workspace (hyb_group_query bytes,
 * 256-byte aligned; lattices: the patches' lattice descriptors, N used).
 *
 * hyb_group_step: one coarse step with max_schwarz iterations; synchronises;
 *   HYB_ENOCONV as hyb_step (the patches are then not committed), or a
 *   patch's HYB_ENONFINITE.
 * hyb_group_coarse: the committed coarse solution, host or device
 *   [(M+1)^2]; synchronises.
 * The patches' own calls (readouts, checkpoints) keep working; hyb_step and
 * the reverse mode are not available on them. */
typedef struct hyb_group hyb_group;
int hyb_group_query(const hyb_mesh *mesh, int n_patches, const hyb_lattice *lattices, size_t *ws_bytes);
int hyb_group_create(const hyb_mesh *mesh, int n_patches, hyb_handle *const *patches, double D,
                     const double *vcoarse, double k, void *workspace, void *stream, hyb_group **out);
int hyb_group_step(hyb_group *g, int max_schwarz);
int hyb_group_coarse(hyb_group *g, double *out, int out_is_device);
void hyb_group_destroy(hyb_group *g);
const char *hyb_group_last_error(const hyb_group *g);

/* Storage layout actually used: row pitch and plane stride in elements. */
int hyb_layout(const hyb_handle *h, size_t *pitch, size_t *plane);

void hyb_destroy(hyb_handle *h);
const char *hyb_last_error(const hyb_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* HYB_H */
