// Internal declarations shared by the HIP kernels and the host runtime of
// libhyb (not part of the public C ABI in include/hyb.h).
#pragma once

#include <hip/hip_runtime.h>

#include "hyb.h"

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace hyb {

// ---------------------------------------------------------------------------
// D2Q9 velocity set (Sec. 4.1): rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-)
// ---------------------------------------------------------------------------
constexpr int kQ = 9;
constexpr int kCx[kQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[kQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[kQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr double kW[kQ] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                           1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
// weight class of each direction (rest, axis, diagonal); w_q depends on q
// only through it, and a direction and its opposite share it
constexpr int kWClass[kQ] = {0, 1, 1, 1, 1, 2, 2, 2, 2};
constexpr int kWClasses = 3;

// Per-node lattice flags (uint16).  Fluid node: bit q (1..8) = the upstream
// neighbour x - e_q is a solid node inside the patch (halfway bounce-back).
// Solid node: bit 15, and bit q = the neighbour x + e_q is a fluid node (the
// fluid end of a link whose population bounces back off this node).
constexpr uint16_t kMaskSolid = 1u << 15;

// Device error counters (uint64 slots in the workspace).
enum Counter { kCntInfeasible = 0, kCntNonfinite = 1, kCntSlots = 8 };

// Scalars of the coarse BiCGSTAB shared between its kernels.
struct KrylovState {
    double rho, rho_next, alpha, rnorm, bnorm, bb;
    // done is raised by the stop test (second kernel of an iteration) and
    // read by the first; skip, brk and bb (= b.b) are written by the first
    // and read by the second, so no kernel reads a field that its own
    // blocks write
    int iters, done, converged, brk, skip, pad1;
};
constexpr int kPartialValues = 8;    // reduction values per partials slot

// Result block written by the coarse solver.
struct KrylovResult {
    int iters;
    int converged;
    double relres;
    unsigned pad0;
    unsigned pad1;
};

// Coarse vectors live on a padded (M+1+2H)^2 grid whose halo stays zero, so
// stencils up to radius H need no bounds checks.
constexpr int kCoarseHalo = 3;
constexpr int kSpaiRadius = 2;                       // preconditioner stencil radius
constexpr int kSpaiW = 2 * kSpaiRadius + 1;          // 5
constexpr int kApW = 2 * (kSpaiRadius + 1) + 1;      // 7: A (radius 1) times P (radius 2)

struct LbmArgs {
    const void *src;
    void *dst;
    const uint16_t *mask;
    const float *vx;
    const float *vy;
    const void *kfield;      // T per node or nullptr
    double k;                // uniform reaction rate when kfield == nullptr
    double omega;            // 1 / tau
    int N;
    int pitch;               // elements between rows
    long long plane;         // elements between population planes
    // perimeter closure
    const int8_t *bc_kind;   // [4(N-1)] or nullptr (all Dirichlet)
    const double *bc_a;
    const double *bc_b;
    double lam;              // j / eta of the step being taken
    double lam2;             // (j + 1) / eta: second step of a two-step launch
    double lam3;             // (j + 2) / eta: third step of a three- or four-step launch
    double lam4;             // (j + 3) / eta: fourth step of a four- or five-step launch
    double lam5;             // (j + 4) / eta: fifth step of a five-step launch
    int clamp;
    unsigned long long *counters;
    // FP16 shifted storage: stored g = (f - w_q c_ref) * scale (binary16);
    // f = g / scale + w_q c_ref, scale a power of two.  hs_wc[c] = w c_ref
    // for weight class c (three values rather than nine: fewer scalar
    // registers, and a population decodes alike from plane q or its
    // opposite, so a bounce-back select needs one decode).
    float hs_scale;
    float hs_inv;
    float hs_wc[kWClasses];
    // surface reaction at fluid-solid links (dissolving solids): the
    // bounce-back value relaxes towards w_q c_sat at rate kappa_s (0: off)
    double kappa_s;
    double c_sat;
    // dissolving solids: flux[n] (pitched, FP64) at every solid node with a
    // fluid neighbour receives the mass its reactive links move into the
    // fluid during the step (overwritten when flux_first, else added to);
    // nullptr: not tracked
    double *flux;
    int flux_first;
    // two-step launches: when set, the first fine step's results of the
    // owned nodes are also stored here (a recording forward keeps every
    // fine state); nullptr: not stored
    void *mid;
    // maximum-entropy zero-flux closure at solid walls (single-step general
    // path): the fluid domain's unit outward normal per node (pitched FP32
    // planes); nullptr: halfway bounce-back
    const float *wall_nx;
    const float *wall_ny;
    // reverse mode: a recording forward also stores u of each fine step's
    // collision at the fluid nodes, a plane of the arithmetic type pitched
    // like a population plane (u_out: the launch's first step; u_out2: the
    // second step of a two-step launch); a reversed step reads the recorded u
    // of the collision it transposes from u_rec (for dJ/dk) instead of
    // summing the next state's nine populations.  nullptr: not stored / from
    // the state.
    void *u_out;
    void *u_out2;
    const void *u_rec;
};

// Population storage policy: FP64 and FP32 store what they compute; FP16
// shifted storage keeps g in binary16 and computes in FP32.  ld and st
// take the plane index q of the value.
template <typename S> struct Pop;
template <> struct Pop<double> {
    typedef double T;
    static __device__ __forceinline__ double ld(double x, int, const LbmArgs &) { return x; }
    static __device__ __forceinline__ double st(double f, int, const LbmArgs &) { return f; }
};
template <> struct Pop<float> {
    typedef float T;
    static __device__ __forceinline__ float ld(float x, int, const LbmArgs &) { return x; }
    static __device__ __forceinline__ float st(float f, int, const LbmArgs &) { return f; }
};
template <> struct Pop<_Float16> {
    typedef float T;
    // g * (1 / scale) is exact (power of two), so the FMA rounds once
    static __device__ __forceinline__ float ld(_Float16 x, int q, const LbmArgs &a) {
        return __builtin_fmaf(static_cast<float>(x), a.hs_inv, a.hs_wc[kWClass[q]]);
    }
    // round to nearest even
    static __device__ __forceinline__ _Float16 st(float f, int q, const LbmArgs &a) {
        return static_cast<_Float16>((f - a.hs_wc[kWClass[q]]) * a.hs_scale);
    }
};

// Launchers (lbm_kernels.hip); `prec` is HYB_FP64, HYB_FP32 or HYB_FP16S
// (storage double, float or binary16).
// One fine step.  general_perimeter: run the perimeter in the separate
// kernel that supports the Neumann closure (else one fused launch with the
// Dirichlet closure).  The optional events bracket the interior sweep.
hipError_t launch_lbm_step(const LbmArgs &a, int prec, bool general_perimeter, hipStream_t s,
                           hipEvent_t sweep_begin = nullptr, hipEvent_t sweep_end = nullptr);
// Two fine steps in one launch (Dirichlet closure on every perimeter slot):
// a.src holds f*(j), a.dst receives f*(j+2); u^p at a.lam, then a.lam2.
// part 0: every tile; part 1: the tiles of the interior rectangle of the
// given depth (depth 0: the tiles whose one-node ring stays clear of the
// patch perimeter, so they read no interface value; depth d: that rectangle
// shrunk by d tiles on every side); part 2: the others.  Parts 1 and 2 of
// one depth together update every node exactly as part 0.  ring 2 or 3: the
// rectangles of launch_lbm_stepk (ring K-1, for passes that mix them).
hipError_t launch_lbm_step2(const LbmArgs &a, int prec, hipStream_t s, int part = 0, int depth = 0,
                            int ring = 1);
// K = 3, 4 or 5 fine steps in one launch (Dirichlet closure on every slot;
// with the surface reaction of dissolving solids, and its link fluxes into
// a.flux, whole-patch launches only): a.src holds f*(j), a.dst receives
// f*(j+K); u^p at a.lam .. a.lam5.  Parts as launch_lbm_step2, the depth-0
// rectangle being the tiles whose ring of `ring` >= K-1 nodes stays clear
// of the patch perimeter.
hipError_t launch_lbm_stepk(const LbmArgs &a, int prec, int K, hipStream_t s, int part = 0, int depth = 0,
                            int ring = 0);
// Adjoint of one fine step (adjoint_kernels.hip), HYB_FP64 or HYB_FP32:
// a.src = the step's source state f*(t) (read only with clamped closures),
// snext = f*(t+1), lam = dJ/df*(t+1); nu is scratch; out = dJ/df*(t);
// grad_a, grad_b [4(N-1)] and grad_k (dense [N][N] or null) accumulate.
// inj (or null, storage type, pitched): a cotangent added to the output at
// fluid nodes.  lam_dense (or null): the cotangent read from a dense FP64
// [9][N][N] array instead of lam; out_dense (or null): the output written
// (accumulate: added) there instead of out -- the packing passes folded into
// the first and last launches of a reversed sweep.
hipError_t launch_adjoint_step(const LbmArgs &a, int prec, const void *snext, const void *lam, void *nu, void *out,
                               double *grad_a, double *grad_b, double *grad_k, hipStream_t s,
                               const void *inj = nullptr, const double *lam_dense = nullptr,
                               double *out_dense = nullptr, bool accumulate = false);
// Two reversed fine steps in one launch: step t (a1.src = f*(t), a1.lam,
// snext1 = f*(t+1)) then step t-1 (a2.src = f*(t-1), a2.lam, snext2 = f*(t)),
// lam = dJ/df*(t+1) -> out = dJ/df*(t-1); gradients as launch_adjoint_step
// for both steps.  Same results as two launch_adjoint_step calls.
// inj_mid, inj_out (or null): cotangents added at fluid nodes to dJ/df*(t)
// and to the output dJ/df*(t-1).
hipError_t launch_adjoint_step2(const LbmArgs &a1, const LbmArgs &a2, int prec, const void *snext1,
                                const void *snext2, const void *lam, void *out, double *grad_a, double *grad_b,
                                double *grad_k, hipStream_t s, const void *inj_mid = nullptr,
                                const void *inj_out = nullptr, const double *lam_dense = nullptr,
                                double *out_dense = nullptr, bool accumulate = false);
// dense FP64 [9][N][N] to pitched planes (to_pitched) or back; back with
// accumulate adds to the dense array instead of overwriting it
hipError_t launch_adjoint_pack(const LbmArgs &a, int prec, const double *dense, void *pitched, bool to_pitched,
                               hipStream_t s, bool accumulate = false);
hipError_t launch_lbm_init(const LbmArgs &a, const double *u0, int prec, hipStream_t s);
hipError_t launch_concentration(const LbmArgs &a, double *out, int prec, hipStream_t s);
// Diagnostics of the state a.src over the fluid nodes: out[0] = sum of the
// concentration, out[1] = smallest population, out[2] = H of eq. (BH),
// out[3] = nodes with a non-finite population (FP64, device).  part is
// device scratch of 4 a.N doubles (row partials).
hipError_t launch_diagnostics(const LbmArgs &a, int prec, double *part, double *out, hipStream_t s);
constexpr int kDiagValues = 4;

struct CoarseDev {
    int M;
    int n;                   // (M+1)^2 mesh nodes
    int S;                   // padded row length M + 1 + 2 kCoarseHalo
    int grid;                // workgroups of the one-lane-per-row kernels
    int grid8;               // workgroups of the eight-lanes-per-row kernels
    int pstride;             // partials per reduction value (>= grid, grid8)
    // A9, B9, P: offset-major, coef[o * n + node], o = (dl + R) * W + (dk + R),
    // so consecutive lanes (consecutive nodes) read consecutive addresses;
    // AP: node-major, coef[node * 49 + o], so the eight lanes of a row read
    // its seven stencil rows as contiguous runs
    const double *A9;        // [9][n] stencil of A
    const double *B9;        // [9][n]
    const double *AP;        // [n][kApW^2] stencil of A P
    const double *P;         // [kSpaiW^2][n] stencil of P
    const int *dkind;        // [n] -1 free (natural outer edges too), -2 outer Dirichlet, >= 0 index into ufc
    double outer_value;
    const double *ufc;       // fine-to-coarse values
    double *xn;              // padded d(t_n)
    double *x1;              // padded new solution
    double *xprev;           // padded d(t_{n-1}) (first-pass guess 2 d(t_n) - d(t_{n-1}))
    double *r, *rh, *p, *v, *s, *t, *y, *w, *z;   // padded Krylov vectors
    double *partials;        // [4 slots][kPartialValues][pstride] reduction partials
    KrylovState *state;
    KrylovResult *result;
};

hipError_t launch_coarse_rhs(const CoarseDev &c, const double *guess, hipStream_t s);
// x1 = 2 xn - xprev over the padded grid (the halo stays zero)
hipError_t launch_coarse_extrapolate(const CoarseDev &c, hipStream_t s);
// Enqueues `iterations` BiCGSTAB iterations (two kernels each; no-ops
// once converged or past max_iter), a closing convergence test and the
// update x1 = guess + P y.
hipError_t launch_coarse_solve(const CoarseDev &c, const double *guess, int iterations, int max_iter, double tol,
                               hipStream_t s);

// Solve (operator c.AP) y = rhs from y = 0 and write out = y (padded):
// the rhs kernel, `iterations` BiCGSTAB iterations, the closing pair and
// the copy; the iteration count and convergence go to *c.result.  With
// c.AP set to the (A P)^T stencil and rhs = P^T lam this is the transposed
// coarse solve mu = A^{-T} lam of the reverse mode.
hipError_t launch_coarse_solve_given(const CoarseDev &c, const double *rhs, double *out, int iterations, int max_iter,
                                     double tol, hipStream_t s);

// Interface transfers (coarse_kernels.hip)
hipError_t launch_c2f(const int *idx, const double *w, int nslots, const double *xa, const double *xb,
                      double *a, double *b, hipStream_t s);
hipError_t launch_f2c(const LbmArgs &lat, const int *idx, const double *w, int nfc, double *ufc, int prec,
                      hipStream_t s);

// Reverse mode of the coarse step and the transfers (coarse_adjoint.hip);
// coarse vectors are padded ((M+1+2 halo)^2, zero halo) unless named dense.
// lam_dn += C^T ga and lam_d1 = C^T gb (+ lam_d_dense when non-null) per
// mesh node, C the coarse-to-fine interpolation (CSR ptr/slot/w over nodes)
hipError_t launch_c2f_transpose(const CoarseDev &c, const int *ptr, const int *slot, const double *w, const double *ga,
                                const double *gb, const double *lam_d_dense, double *lam_dn, double *lam_d1,
                                hipStream_t s);
// out = S in for a node-major-to-offset-major stencil S of width W (5: P^T)
hipError_t launch_coarse_stencil(const CoarseDev &c, const double *coef, int W, const double *in, double *out,
                                 hipStream_t s);
// lam_dn += B^T (mu on the free rows); lam_ufc[c] = a_ii mu[row c] on the
// Gamma_{f->c} rows (fc_row: mesh node of each); grad_outer (dense, or
// null) += a_ii mu on the outer-edge rows
hipError_t launch_coarse_rhs_transpose(const CoarseDev &c, const int *fc_row, int nfc, const double *mu,
                                       double *lam_dn, double *lam_ufc, double *grad_outer, hipStream_t s);
// Fine-to-coarse transposed onto the lattice nodes it reads (CSR node/ptr/
// cidx/w over ntouched pitched nodes): lam_u = sum w lam_ufc[c]; every
// population of the node receives lam_u / (1 - k), added to lam_pitched
// (storage T planes) or, when that is null, to lam_dense (FP64 [9][N][N]);
// grad_k (dense [N][N], or null) += lam_u sum_q g_q / (1 - k)^2 for the
// state g the forward transfer read.  HYB_FP64 or HYB_FP32 storage.
hipError_t launch_f2c_transpose(const LbmArgs &lat, int prec, const int *node, const int *ptr, const int *cidx,
                                const double *w, int ntouched, const double *lam_ufc, const void *g_state,
                                void *lam_pitched, double *lam_dense, double *grad_k, hipStream_t s);
// Dissolving solids (dissolve_kernels.hip), HYB_FP64 / FP32 / FP16S storage;
// per-node arrays are pitched like the flag words.
// Commit of the geometry: at every solid node mass -= a.flux (solid nodes
// with a fluid neighbour; the others moved nothing); a node whose mass is
// then <= 0 becomes fluid (solid[] cleared) and takes f*_q = w_q u_mean (1 - k) in a.dst (the committed state),
// u_mean the mean concentration of its fluid neighbours there (flag words
// before the commit).  Then every flag word is rebuilt from solid[].
hipError_t launch_dissolve_commit(const LbmArgs &a, int prec, double *mass, uint8_t *solid, uint16_t *mask,
                                  hipStream_t s);
// Fine-to-coarse transfer with the bilinear weights of the current fluid
// corners: idx/w the four raw corners and weights of each Gamma_{f->c}
// node, fb[c] its fallback node (-1: none) used when no fluid corner
// carries weight.
hipError_t launch_f2c_dynamic(const LbmArgs &lat, const int *idx, const double *w, const int *fb, int nfc,
                              double *ufc, int prec, hipStream_t s);
// Flag words from solid[] alone (restoring a saved geometry).
hipError_t launch_mask_rebuild(int N, int pitch, const uint8_t *solid, uint16_t *mask, hipStream_t s);
// Reverse mode of a dissolving step (HYB_FP64 / FP32 storage; a.mask = the
// step's flag words before its commit, after[] = solid flags after it).
// Conversion transposed in place on lam (pitched cotangent of the committed
// state): each converted node's cotangent, through the mean concentration of
// its fluid neighbours in pre (the state before the commit), is added to
// those neighbours and the node's own is cleared; H (FP64, pitched) is
// scratch; grad_k (dense [N][N] or null) takes the (1 - k) terms.
hipError_t launch_conversion_transpose(const LbmArgs &a, int prec, const uint8_t *after, const void *pre, void *lam,
                                       double *H, double *grad_k, hipStream_t s);
// Transposed fine-to-coarse transfer with the weights of the step's fluid
// corners (lists of launch_f2c_dynamic's superset, a.mask the step's flag
// words); otherwise as launch_f2c_transpose.
hipError_t launch_f2c_dynamic_transpose(const LbmArgs &lat, int prec, const int *node, const int *ptr,
                                        const int *cidx, const int *slot, int ntouched, const int *fcr_idx,
                                        const double *fcr_w, const double *lam_ufc, const void *g_state,
                                        void *lam_pitched, double *lam_dense, double *grad_k, hipStream_t s);

// dense[(M+1)^2] = padded (unpad), or padded = dense (pad, halo untouched)
hipError_t launch_coarse_repad(const CoarseDev &c, const double *from, double *to, bool to_dense, hipStream_t s);

// ---------------------------------------------------------------------------
// host-side setup (coarse_setup.hip)
// ---------------------------------------------------------------------------
struct CoarseHost {
    int M = 0;
    double L = 0, h = 0;
    std::vector<double> A9, B9, AP, P;
    std::vector<int> dkind;
    std::vector<int> fc_nodes;             // mesh node ids on Gamma_{f->c}
    std::vector<int> fc_idx;               // [nfc][4] padded fine node offsets
    std::vector<double> fc_w;              // [nfc][4]
    std::vector<int> c2f_idx;              // [4(N-1)][4] padded coarse indices
    std::vector<double> c2f_w;             // [4(N-1)][4]
    // reverse mode: (A P)^T (node-major, like AP) and P^T (node-major, like
    // P) stencils; the coarse-to-fine transfer transposed per mesh node
    // (CSR over nodes: slots and weights, in slot order); the fine-to-coarse
    // transfer transposed per lattice node it reads (CSR over the touched
    // pitched nodes: Gamma_{f->c} indices and nonzero weights, in index order)
    // fine-to-coarse corners before the solid rule (dissolving solids):
    // pitched corner nodes, raw bilinear weights, and the fallback node of a
    // coarse node whose fluid corners carry no weight (-1 otherwise)
    std::vector<int> fcr_idx, fcr_fb;
    std::vector<double> fcr_w;
    // their transposed superset: per lattice node that is a raw corner or a
    // fallback node, the Gamma_{f->c} indices and slots (0..3 corner, 4
    // fallback), node then index order
    std::vector<int> f2cD_node, f2cD_ptr, f2cD_c, f2cD_m;
    std::vector<double> APT, PT;
    std::vector<int> c2fT_ptr, c2fT_slot;
    std::vector<double> c2fT_w;
    std::vector<int> f2cT_node, f2cT_ptr, f2cT_c;
    std::vector<double> f2cT_w;
};

// Assembles A, B for the trapezoidal step dt and the SPAI preconditioner;
// fills the interface lists.  Returns an empty string or an error message.
std::string build_coarse(int M, double L, double D, double k, double dt, int supg, const double *vnodes,
                         int overlap_elems, int N, double x0, double y0, const uint8_t *solid, int pitch,
                         CoarseHost &out, int outer_natural = 0);
// Several fine patches on one mesh (Algorithm 2): the Dirichlet rows take
// every patch's Gamma_{f->c} (indices patch by patch: patch p's run starts
// after the nodes of patches 0 .. p-1); out holds the operator and patch 0's
// lists, *more (if given) the lists of patches 1 .. n-1.
struct PatchGeom {
    int N;
    double x0, y0;
    const uint8_t *solid;
    int pitch;
};
std::string build_coarse(int M, double L, double D, double k, double dt, int supg, const double *vnodes,
                         int overlap_elems, const std::vector<PatchGeom> &patches, CoarseHost &out,
                         std::vector<CoarseHost> *more, int outer_natural = 0);
std::string patch_lists(int M, double L, const PatchGeom &g, CoarseHost &out);

// Perimeter slot <-> node mapping shared by host and device code.
__host__ __device__ inline void slot_to_node(int N, int p, int &i, int &j) {
    if (p < N) { i = p; j = 0; return; }
    if (p < 2 * N) { i = p - N; j = N - 1; return; }
    if (p < 3 * N - 2) { i = 0; j = p - 2 * N + 1; return; }
    i = N - 1;
    j = p - (3 * N - 2) + 1;
}

}  // namespace hyb
