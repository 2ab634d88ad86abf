// D2Q9 advection-diffusion-reaction lattice Boltzmann kernels for gfx950.
//
// One fine step (Sec. 4.1, eqs. LBE and Collision) is a fused pull update:
// each node gathers the post-collision populations of its upstream
// neighbours (x - e_i), replaces those whose upstream node is solid by its
// own reversed population (halfway bounce-back), closes the populations
// whose upstream node lies outside the patch with the maximum-entropy
// closure of Sec. 4.1.1 (perimeter nodes only), and relaxes towards the
// equilibrium of eq. (LBM_feq) with the first-order reaction source
// -k w_i u.  Populations are structure-of-arrays planes [9][N][pitch] in
// the storage type S (double, float, or binary16 holding the shifted and
// scaled g of Pop<_Float16>); arithmetic is in Pop<S>::T (double or float),
// the closures in FP64.
//
// Default path: two fine steps per launch (lbm_sweep2_kernel, temporal
// blocking through LDS).  Single-step kernels serve odd step counts
// (lbm_sweep_kernel, perimeter Dirichlet slots in the same launch) and
// handles with Neumann slots (lbm_bulk_kernel + lbm_perimeter_kernel, whose
// FP64 Newton solve would otherwise lower the occupancy of the sweep).
#include "hyb_impl.h"

#include <type_traits>

namespace hyb {
namespace {

// BGK collision with reaction, written as
//   f*_i = (1 - w) f_i + w_i [ w u (1 + 3 e.v + 9/2 (e.v)^2 - 3/2 v.v) - k u ],
// w = 1/tau; u = sum_i f_i (eq. LBM_Macro); the bracket's polynomial is the
// equilibrium of eq. (LBM_feq) with c_s^2 = 1/3 and the quadratic term read
// as -v.v/(2 c_s^2).  Returns u.
template <typename T>
__device__ __forceinline__ T collide(T (&f)[kQ], T vx, T vy, T omega, T k) {
    const T u = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const T A = omega * u;
    const T base = A * (T(1) - T(1.5) * (vx * vx + vy * vy)) - k * u;
    const T keep = T(1) - omega;
    const T c3 = T(3) * A;
    const T c45 = T(4.5) * A;
    const T w0 = T(kW[0]), w1 = T(kW[1]), w5 = T(kW[5]);
    const T dpp = vx + vy, dmp = vy - vx;   // e.v of (+,+) and (-,+)
    f[0] = keep * f[0] + w0 * base;
    f[1] = keep * f[1] + w1 * (base + c3 * vx + c45 * vx * vx);
    f[3] = keep * f[3] + w1 * (base - c3 * vx + c45 * vx * vx);
    f[2] = keep * f[2] + w1 * (base + c3 * vy + c45 * vy * vy);
    f[4] = keep * f[4] + w1 * (base - c3 * vy + c45 * vy * vy);
    f[5] = keep * f[5] + w5 * (base + c3 * dpp + c45 * dpp * dpp);
    f[7] = keep * f[7] + w5 * (base - c3 * dpp + c45 * dpp * dpp);
    f[6] = keep * f[6] + w5 * (base + c3 * dmp + c45 * dmp * dmp);
    f[8] = keep * f[8] + w5 * (base - c3 * dmp + c45 * dmp * dmp);
    return u;
}

__device__ __forceinline__ bool finite_val(double x) { return x - x == 0.0; }
__device__ __forceinline__ bool finite_val(float x) { return x - x == 0.0f; }

// Adds the number of active lanes whose flag is set to *ctr with one atomic
// per wavefront (the one-node-per-thread kernels).
__device__ __forceinline__ void count_lanes(unsigned long long *ctr, bool flag) {
    const unsigned long long lanes = __ballot(flag);
    if (lanes == 0ull) return;
    if (__lane_id() == __ffsll(static_cast<long long>(lanes)) - 1) atomicAdd(ctr, static_cast<unsigned long long>(__popcll(lanes)));
}

// Event counts of one lane over a whole multi-step launch.  At the patch
// edge a wavefront holds one perimeter node per round, so per-wavefront
// aggregation still leaves one atomic per event; and device-scope atomics
// on one address, issued from every XCD, serialise at the memory side and
// hold up the sweep's own loads and stores there.  The sweeps therefore
// count in registers and add to the device counters once per workgroup.
struct Tally {
    unsigned bad = 0u;          // infeasible closures at owned perimeter nodes
    unsigned nonfinite = 0u;    // owned nodes whose concentration is not finite
};

__device__ __forceinline__ unsigned wave_sum(unsigned v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Adds a workgroup's tallies to the device counters.  `edge` is uniform
// over the workgroup (whether the tile with its ring reaches the patch
// perimeter) and false where no closure ran, so only edge tiles take the
// extra barrier; a non-finite value is rare enough to count per wavefront.
template <int NT>
__device__ __forceinline__ void flush_tally(const LbmArgs &a, const Tally &t, bool edge) {
    if (__ballot(t.nonfinite != 0u) != 0ull) {
        const unsigned s = wave_sum(t.nonfinite);
        if (__lane_id() == 0) atomicAdd(&a.counters[kCntNonfinite], static_cast<unsigned long long>(s));
    }
    if (edge) {
        __shared__ unsigned part[NT / 64];
        const unsigned s = wave_sum(t.bad);
        if (__lane_id() == 0) part[threadIdx.x / 64] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long sum = 0ull;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) sum += part[w];
            if (sum != 0ull) atomicAdd(&a.counters[kCntInfeasible], sum);
        }
    }
}

// Address of the value a node pulls along q from an LDS stage: the upstream
// slot `pull` or, where the upstream node is solid (flag bit q set), the
// node's own opposite slot `back` (halfway bounce-back); both in elements
// from the node's slot.  The flag bit goes through an empty asm statement so
// that the compiler cannot see its 0/1 range: it would turn
// bit * (back - pull) into a compare and a select between two constants it
// first moves into registers (six VALU instructions per direction); as an
// opaque product it is a bit-field extract and one 24-bit multiply-add.  An
// LDS byte offset always fits the multiply's signed 24 bits.
template <typename T>
__device__ __forceinline__ const T *pull_or_back(const T *node, unsigned m, int q, int pull, int back) {
    int bit = static_cast<int>(__builtin_amdgcn_ubfe(m, static_cast<unsigned>(q), 1u));
    asm("" : "+v"(bit));
    constexpr int sz = static_cast<int>(sizeof(T));
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(node) + pull * sz +
                                       __mul24(bit, (back - pull) * sz));
}

// per-node reaction rate (k field in the arithmetic type) or the uniform one
template <typename T>
__device__ __forceinline__ T node_k(const LbmArgs &a, int n) {
    return a.kfield ? static_cast<const T *>(a.kfield)[n] : T(a.k);
}

// Perimeter slot of perimeter node (i, j) (inverse of slot_to_node).
__device__ __forceinline__ int perimeter_slot(int N, int i, int j) {
    if (j == 0) return i;
    if (j == N - 1) return N + i;
    if (i == 0) return 2 * N + j - 1;
    return 3 * N - 2 + j - 1;
}

// bit q set: the upstream node x - e_q lies outside the patch
__device__ __forceinline__ unsigned outside_bits(int N, int i, int j) {
    unsigned u = 0;
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
        const int si = i - kCx[q], sj = j - kCy[q];
        if (si < 0 || si >= N || sj < 0 || sj >= N) u |= 1u << q;
    }
    return u;
}

// Dirichlet closure of eq. (LBM_Dir): the unknowns U share the mass deficit
// R = u^p - sum_known f in proportion to w_i; sums in FP64.  u^p is the
// eq. (MTS) value (1 - lam) a + lam b of slot p.  R < 0 (no non-negative
// solution) is reported; with clamp the unknowns become 0, otherwise the
// closed form is kept.
template <typename T>
__device__ __forceinline__ bool dirichlet_close(const LbmArgs &a, T (&f)[kQ], unsigned unknown, int p,
                                                double lam) {
    double known = 0.0, wsum = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        if ((unknown >> q) & 1u) wsum += kW[q];
        else known += double(f[q]);
    }
    double R = (1.0 - lam) * a.bc_a[p] + lam * a.bc_b[p] - known;
    const bool bad = R < 0.0;
    if (bad && a.clamp) R = 0.0;
    const double scale = R / wsum;
#pragma unroll
    for (int q = 0; q < kQ; ++q)
        if ((unknown >> q) & 1u) f[q] = T(kW[q] * scale);
    return bad;
}

// Workgroups are handed to the 8 XCDs (each with its own L2) in
// round-robin order.  Tile t of T is given to workgroup b so that XCD b % 8
// sweeps one contiguous eighth of the tiles in row-major order: the lines a
// tile shares with its neighbours (pulls, halos) are then fetched into the
// same L2.
__device__ __forceinline__ int xcd_tile(int b, int T) {
    const int x = b & 7, k = b >> 3;
    const int q = T >> 3, r = T & 7;
    return x * q + (x < r ? x : r) + k;
}

// Whether the region of rows y0 - r .. y0 + h - 1 + r and columns x0 - r ..
// x0 + w - 1 + r reaches the patch perimeter (uniform across a workgroup:
// the per-node perimeter test only runs in tiles where it can hold).
__device__ __forceinline__ bool reaches_perimeter(int N, int x0, int y0, int w, int h, int r) {
    return x0 - r <= 0 || y0 - r <= 0 || x0 + w - 1 + r >= N - 1 || y0 + h - 1 + r >= N - 1;
}

// ---------------------------------------------------------------------------
// Single fine step
// ---------------------------------------------------------------------------

// Bounce-back value across a link to a solid node with the surface reaction
// of dissolving solids: (1 - kappa_s) f + kappa_s w_q c_sat (f itself when
// the reaction is off).
template <typename T>
__device__ __forceinline__ T reactive(const LbmArgs &a, T f, int q) {
    if (a.kappa_s == 0.0) return f;
    return T((1.0 - a.kappa_s) * double(f) + a.kappa_s * kW[q] * a.c_sat);
}

// Solid node n with fluid neighbours (flag bits q): the mass its reactive
// links move into the fluid during this step, sum over q of
// kappa_s (w_q c_sat - f*_opp(q)(n + e_q)), in q order, into a.flux[n].
template <typename S>
__device__ __forceinline__ void solid_link_flux(const LbmArgs &a, const S *__restrict__ src, unsigned m, int n,
                                                int plane, int P) {
    double s = 0.0;
#pragma unroll
    for (int q = 1; q < kQ; ++q)
        if ((m >> q) & 1u) {
            const int x = n + kCx[q] + kCy[q] * P;
            s += a.kappa_s * (kW[q] * a.c_sat - double(Pop<S>::ld(src[kOpp[q] * plane + x], kOpp[q], a)));
        }
    a.flux[n] = a.flux_first ? s : a.flux[n] + s;
}

__device__ int closure_neumann(double (&f)[kQ], unsigned unknown, double nx, double ny, double qp,
                               const double (&own)[kQ]);

// Interior node (1 <= i, j <= N-2): every upstream node is inside the
// patch.  The nine pulls are issued before the flag word is known;
// bounce-back values replace them afterwards.  Stores are non-temporal: the
// destination plane is not read again before the sweep has finished.
// WALL: at a node with solid upstream nodes the maximum-entropy zero-flux
// closure of eq. (LBM_Neu) with the wall's normal (a.wall_nx, a.wall_ny)
// replaces bounce-back (FP64 Newton, the perimeter's closure).
template <typename S, bool WALL = false>
__device__ __forceinline__ void interior_node(const LbmArgs &a, const S *__restrict__ src, S *__restrict__ dst,
                                              int n, int plane, int P) {
    typedef typename Pop<S>::T T;
    S raw[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) raw[q] = src[q * plane + n - kCx[q] - kCy[q] * P];
    const unsigned m = a.mask[n];
    if (m & kMaskSolid) {
        if (a.flux && (m & 0x1FEu)) solid_link_flux<S>(a, src, m, n, plane, P);
        return;
    }
    const float vx = a.vx[n], vy = a.vy[n];
    T f[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) f[q] = Pop<S>::ld(raw[q], q, a);
    if (WALL && (m & 0x1FEu)) {
        // unknowns: every population with e.n < 0 (the set M- of eq.
        // LBM_Neu), and the solid-sourced ones (bounced back where e.n >= 0)
        const double nx = double(a.wall_nx[n]), ny = double(a.wall_ny[n]);
        unsigned unknown = m & 0x1FEu;
        double fd[kQ], own[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            own[q] = double(Pop<S>::ld(src[q * plane + n], q, a));
            fd[q] = double(f[q]);
            if (q > 0 && kCx[q] * nx + kCy[q] * ny < 0.0) unknown |= 1u << q;
        }
        count_lanes(&a.counters[kCntInfeasible], closure_neumann(fd, unknown, nx, ny, 0.0, own));
#pragma unroll
        for (int q = 0; q < kQ; ++q) f[q] = T(fd[q]);
    } else if (m & 0x1FEu) {
#pragma unroll
        for (int q = 1; q < kQ; ++q)
            if ((m >> q) & 1u) f[q] = Pop<S>::ld(src[kOpp[q] * plane + n], kOpp[q], a);
        if (a.kappa_s != 0.0) {
#pragma unroll
            for (int q = 1; q < kQ; ++q)
                if ((m >> q) & 1u) f[q] = reactive<T>(a, f[q], q);
        }
    }
    const T u = collide<T>(f, T(vx), T(vy), T(a.omega), node_k<T>(a, n));
    count_lanes(&a.counters[kCntNonfinite], !finite_val(u));
#pragma unroll
    for (int q = 0; q < kQ; ++q) __builtin_nontemporal_store(Pop<S>::st(f[q], q, a), &dst[q * plane + n]);
    if (a.u_out) static_cast<T *>(a.u_out)[n] = u;
}

// Perimeter slot p with the Dirichlet closure.
template <typename S>
__device__ __forceinline__ void perimeter_dirichlet_node(const LbmArgs &a, const S *__restrict__ src,
                                                         S *__restrict__ dst, int p, int plane, int P) {
    typedef typename Pop<S>::T T;
    const int N = a.N;
    int i, j;
    slot_to_node(N, p, i, j);
    const int n = j * P + i;
    const unsigned m = a.mask[n];
    if (m & kMaskSolid) return;
    const unsigned unknown = outside_bits(N, i, j);
    T f[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        if ((unknown >> q) & 1u) f[q] = T(0);
        else if ((m >> q) & 1u) f[q] = reactive<T>(a, Pop<S>::ld(src[kOpp[q] * plane + n], kOpp[q], a), q);
        else f[q] = Pop<S>::ld(src[q * plane + (j - kCy[q]) * P + i - kCx[q]], q, a);
    }
    count_lanes(&a.counters[kCntInfeasible], dirichlet_close<T>(a, f, unknown, p, a.lam));
    const T u = collide<T>(f, T(a.vx[n]), T(a.vy[n]), T(a.omega), node_k<T>(a, n));
    count_lanes(&a.counters[kCntNonfinite], !finite_val(u));
#pragma unroll
    for (int q = 0; q < kQ; ++q) dst[q * plane + n] = Pop<S>::st(f[q], q, a);
    if (a.u_out) static_cast<T *>(a.u_out)[n] = u;
}

// One fine step over the whole patch in one launch: the first `tiles`
// workgroups take interior rows (tile t covers row 1 + t / row_blocks,
// 256 consecutive columns), the rest the 4(N-1) perimeter slots.
template <typename S>
__global__ void __launch_bounds__(256) lbm_sweep_kernel(LbmArgs a, int tiles, int row_blocks) {
    const int P = a.pitch;
    const int plane = static_cast<int>(a.plane);
    const S *__restrict__ src = static_cast<const S *>(a.src);
    S *__restrict__ dst = static_cast<S *>(a.dst);
    const int b = blockIdx.x;
    if (b >= tiles) {
        const int p = (b - tiles) * blockDim.x + threadIdx.x;
        if (p < 4 * (a.N - 1)) perimeter_dirichlet_node<S>(a, src, dst, p, plane, P);
        return;
    }
    const int t = xcd_tile(b, tiles);
    const int j = 1 + t / row_blocks;
    const int i = 1 + (t % row_blocks) * blockDim.x + threadIdx.x;
    if (i <= a.N - 2) interior_node<S>(a, src, dst, j * P + i, plane, P);
}

// Interior only (with the general perimeter kernel when some slots carry
// the Neumann closure).
template <typename S, bool WALL>
__global__ void __launch_bounds__(256) lbm_bulk_kernel(LbmArgs a, int row_blocks) {
    const int P = a.pitch;
    const int j = 1 + blockIdx.x / row_blocks;
    const int i = 1 + (blockIdx.x % row_blocks) * blockDim.x + threadIdx.x;
    if (i <= a.N - 2)
        interior_node<S, WALL>(a, static_cast<const S *>(a.src), static_cast<S *>(a.dst), j * P + i,
                               static_cast<int>(a.plane), P);
}

// ---------------------------------------------------------------------------
// Maximum-entropy closures (Sec. 4.1.1), FP64, for the general perimeter.
//
// Dirichlet, eq. (LBM_Dir): as dirichlet_close.
//
// Neumann, eq. (LBM_Neu), for a unit outward normal n (a patch edge or
// corner, or a solid wall): unknowns with e_i.n < 0 are w_i exp(-1 + g s_i),
// s_i = -e_i.n > 0, where the Lagrange multiplier g solves
//   ln sum_i w_i s_i exp(-1 + g s_i) = ln R',  R' = sum_known (e.n) f - q^p.
// The left side is convex and increasing in g; Newton from the closed-form
// start (exact when all s_i are equal, i.e. on a flat edge) converges
// monotonically after its first step.  Unknowns with e_i.n >= 0 (the
// tangential ones at a corner, links a curved wall grazes) are bounced back
// from the node's own post-collision value.
// ---------------------------------------------------------------------------
__device__ int closure_dirichlet(double (&f)[kQ], unsigned unknown, double up, int clamp) {
    double known = 0.0, wsum = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        if ((unknown >> q) & 1u) wsum += kW[q];
        else known += f[q];
    }
    double R = up - known;
    const int bad = R < 0.0;
    if (bad && clamp) R = 0.0;
    const double scale = R / wsum;
#pragma unroll
    for (int q = 0; q < kQ; ++q)
        if ((unknown >> q) & 1u) f[q] = kW[q] * scale;
    return bad;
}

__device__ int closure_neumann(double (&f)[kQ], unsigned unknown, double nx, double ny, double qp,
                               const double (&own)[kQ]) {
    unsigned out = 0;      // M-: unknowns with e.n < 0
    double flux_known = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const double dot = kCx[q] * nx + kCy[q] * ny;
        if ((unknown >> q) & 1u) {
            if (dot < 0.0) { out |= 1u << q; continue; }
            f[q] = own[kOpp[q]];
        }
        flux_known += dot * f[q];
    }
    const double Rp = flux_known - qp;
    // no population of M- to solve with: infeasible unless already met
    if (!out) return Rp != 0.0;
    if (!(Rp > 0.0)) {
#pragma unroll
        for (int q = 0; q < kQ; ++q)
            if ((out >> q) & 1u) f[q] = 0.0;
        return 1;
    }
    double sw = 0.0, sw2 = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        if ((out >> q) & 1u) {
            const double s = -(kCx[q] * nx + kCy[q] * ny);
            sw += kW[q] * s;
            sw2 += kW[q] * s * s;
        }
    }
    const double lnR = log(Rp);
    double g = (1.0 + lnR - log(sw)) / (sw2 / sw);
    for (int it = 0; it < 30; ++it) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            if ((out >> q) & 1u) {
                const double s = -(kCx[q] * nx + kCy[q] * ny);
                const double e = kW[q] * s * exp(-1.0 + g * s);
                s0 += e;
                s1 += e * s;
            }
        }
        const double step = (lnR - log(s0)) * s0 / s1;
        g += step;
        if (fabs(step) <= 4.0 * 2.220446049250313e-16 * (1.0 + fabs(g))) break;
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        if ((out >> q) & 1u) {
            const double s = -(kCx[q] * nx + kCy[q] * ny);
            f[q] = kW[q] * exp(-1.0 + g * s);
        }
    }
    return 0;
}

// perimeter nodes, Dirichlet or Neumann per slot: one thread per slot
template <typename S>
__global__ void __launch_bounds__(128) lbm_perimeter_kernel(LbmArgs a) {
    typedef typename Pop<S>::T T;
    const int N = a.N;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= 4 * (N - 1)) return;
    int i, j;
    slot_to_node(N, p, i, j);
    const int P = a.pitch;
    const int plane = static_cast<int>(a.plane);
    const int n = j * P + i;
    const unsigned m = a.mask[n];
    if (m & kMaskSolid) return;
    const S *__restrict__ src = static_cast<const S *>(a.src);
    S *__restrict__ dst = static_cast<S *>(a.dst);

    double f[kQ], own[kQ];
    unsigned unknown = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        own[q] = double(Pop<S>::ld(src[q * plane + n], q, a));
        const int si = i - kCx[q], sj = j - kCy[q];
        if (si < 0 || si >= N || sj < 0 || sj >= N) {
            unknown |= 1u << q;
            f[q] = 0.0;
        } else if ((m >> q) & 1u) {
            f[q] = double(reactive<T>(a, Pop<S>::ld(src[kOpp[q] * plane + n], kOpp[q], a), q));
        } else {
            f[q] = double(Pop<S>::ld(src[q * plane + sj * P + si], q, a));
        }
    }
    const int kind = a.bc_kind ? a.bc_kind[p] : 0;
    const double value = (1.0 - a.lam) * a.bc_a[p] + a.lam * a.bc_b[p];
    int bad;
    if (kind == 0) {
        bad = closure_dirichlet(f, unknown, value, a.clamp);
    } else {
        const int sx = (i == 0) ? -1 : (i == N - 1) ? 1 : 0;
        const int sy = (j == 0) ? -1 : (j == N - 1) ? 1 : 0;
        const double inv_norm = rsqrt(double(sx * sx + sy * sy));
        bad = closure_neumann(f, unknown, sx * inv_norm, sy * inv_norm, value, own);
    }
    count_lanes(&a.counters[kCntInfeasible], bad);

    T g[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = T(f[q]);
    const T u = collide<T>(g, T(a.vx[n]), T(a.vy[n]), T(a.omega), node_k<T>(a, n));
    count_lanes(&a.counters[kCntNonfinite], !finite_val(u));
#pragma unroll
    for (int q = 0; q < kQ; ++q) dst[q * plane + n] = Pop<S>::st(g[q], q, a);
}

// ---------------------------------------------------------------------------
// Two fine steps per launch (temporal blocking), Dirichlet closure only.
//
// A workgroup owns a TW x TH tile of the patch.  First half: every node of
// the tile grown by one ring (clipped to the patch) takes fine step j+1
// from the source buffer; the results stay in LDS (arithmetic type).
// Second half: the tile's own nodes take step j+2 from LDS and go to the
// destination buffer.  Per node the arithmetic is that of the single-step
// sweep (pull, halfway bounce-back, eq. (LBM_Dir) closure at perimeter
// nodes with u^p at lam = (j+1)/eta, then (j+2)/eta, collision).  Ring
// nodes are computed by every tile that borders them, so only the tile
// that owns a node counts its infeasible closures and non-finite values.
// HBM traffic for two steps is one read of the state (the ring-2 halo is
// mostly served by L2) and one write.
// ---------------------------------------------------------------------------

// Raw buffer access (gfx9 buffer instructions): the array base and size
// live in one SGPR resource and each lane supplies a 32-bit byte offset
// (stores add the plane offset q * plane as the scalar offset), so a pull
// or a store costs no 64-bit address arithmetic.  Offsets at or past
// num_records read as 0 without touching memory.
typedef __amdgpu_buffer_rsrc_t BufRsrc;
__device__ __forceinline__ BufRsrc buf_rsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename S> struct Buf;
template <> struct Buf<float> {
    static __device__ __forceinline__ float load(BufRsrc r, unsigned v, unsigned s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
    }
    static __device__ __forceinline__ void store_nt(float x, BufRsrc r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, 2);
    }
};
template <> struct Buf<double> {
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(BufRsrc(), 0, 0, 0)) Raw;
    static __device__ __forceinline__ double load(BufRsrc r, unsigned v, unsigned s) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
    }
    static __device__ __forceinline__ void store_nt(double x, BufRsrc r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(Raw, x), r, v, s, 2);
    }
};
template <> struct Buf<_Float16> {
    static __device__ __forceinline__ _Float16 load(BufRsrc r, unsigned v, unsigned s) {
        return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
    }
    static __device__ __forceinline__ void store_nt(_Float16 x, BufRsrc r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, 2);
    }
};

// Which tiles a two-step launch covers: all of the tiles_x x tiles_y grid
// (part 0), a rectangle [ix0, ix1] x [iy0, iy1] of tiles (part 1), or the
// other tiles (part 2).  The rectangle of depth 0 holds the tiles whose ring
// stays clear of the patch perimeter: a part-1 launch of it reads no
// interface value, so it may run while the coarse solve that produces them
// is still in flight.  The rectangle of depth d is that one shrunk by d tiles
// on every side; its tiles read (with their two-node halo) only nodes that
// the depth d-1 rectangle of the previous launch wrote, so the depth-d part 1
// of launch d+1 of a pass may run ahead of the coarse solve as well.
struct TileMap {
    int tiles_x, tiles_y;
    int part;
    int ix0, ix1, iy0, iy1;
    int count;               // tiles in this part
};

// Tile of the t-th workgroup of a launch of part PART (a template argument,
// so each part is its own kernel symbol and carries no runtime branch).
template <int PART>
__device__ __forceinline__ void tile_of(const TileMap &m, int t, int &tx, int &ty) {
    if constexpr (PART == 0) {
        tx = t % m.tiles_x;
        ty = t / m.tiles_x;
        return;
    }
    const int iw = m.ix1 - m.ix0 + 1;
    if constexpr (PART == 1) {
        tx = m.ix0 + t % iw;
        ty = m.iy0 + t / iw;
        return;
    }
    // part 2: rows below the rectangle, then its left and right margins row
    // by row, then the rows above it
    const int below = m.iy0 * m.tiles_x;
    if (t < below) {
        tx = t % m.tiles_x;
        ty = t / m.tiles_x;
        return;
    }
    t -= below;
    const int side = m.tiles_x - iw;           // margin tiles per middle row
    const int middle = (m.iy1 - m.iy0 + 1) * side;
    if (t < middle) {
        const int r = t / side, k = t % side;
        ty = m.iy0 + r;
        tx = k < m.ix0 ? k : m.ix1 + 1 + (k - m.ix0);
        return;
    }
    t -= middle;
    tx = t % m.tiles_x;
    ty = m.iy1 + 1 + t / m.tiles_x;
}

// Body of the two-step sweep.  FLUX (dissolving solids): bounce-back
// values carry the surface reaction, and every owned solid node with fluid
// neighbours adds the link fluxes of both fine steps to a.flux (step j+1
// from the source buffer, step j+2 from the first half's results in LDS).
template <typename S, int TW, int TH, int NT, int PART, bool FLUX, bool MID = false>
__device__ __forceinline__ void sweep2_body(const LbmArgs &a, const TileMap &map) {
    typedef typename Pop<S>::T T;
    constexpr int W1 = TW + 2, H1 = TH + 2, R1 = W1 * H1;
    constexpr int ROUNDS1 = (R1 + NT - 1) / NT;
    static_assert((TW * TH) % NT == 0 && NT % TW == 0, "second half: whole rows per round");
    constexpr int ROUNDS2 = TW * TH / NT;
    constexpr unsigned sz = sizeof(S);
    static_assert(sizeof(T) * kQ * R1 < (1u << 23), "pull_or_back: LDS byte offsets within 24 bits");
    __shared__ T lds[kQ][H1][W1];

    const int N = a.N;
    const int P = a.pitch;
    const unsigned SP = static_cast<unsigned>(a.plane);
    const unsigned NP = static_cast<unsigned>(N) * static_cast<unsigned>(P);
    const BufRsrc fsrc = buf_rsrc(a.src, kQ * SP * sz);
    const BufRsrc fdst = buf_rsrc(a.dst, kQ * SP * sz);
    const BufRsrc mrs = buf_rsrc(a.mask, NP * 2u);
    const BufRsrc vxr = buf_rsrc(a.vx, NP * 4u);
    const BufRsrc vyr = buf_rsrc(a.vy, NP * 4u);
    const T omega = T(a.omega);
    int tx, ty;
    tile_of<PART>(map, xcd_tile(blockIdx.x, map.count), tx, ty);
    const int x0 = tx * TW;
    const int y0 = ty * TH;
    const bool edge = reaches_perimeter(N, x0, y0, TW, TH, 1), edge2 = reaches_perimeter(N, x0, y0, TW, TH, 0);
    Tally tally;

    // ---- first half: step j+1 on the tile and its ring, into LDS --------
    // Pull x - e_q reads plane q at row j - cy_q, column i - cx_q, both
    // clamped onto the patch (values fetched for upstream nodes outside the
    // patch are replaced by the closure).  Measured against conditional
    // reloads of the bounce-back values: 11% faster at 2048^2 in FP32, 14%
    // in FP64 (no divergent branches, no second round trip).
    S raw[ROUNDS1][kQ];
    unsigned m[ROUNDS1];
    float vx1[ROUNDS1], vy1[ROUNDS1];
    // node coordinates of each round, stepped without divisions
    int rr[ROUNDS1], cc[ROUNDS1];
    rr[0] = threadIdx.x / W1;
    cc[0] = threadIdx.x - rr[0] * W1;
#pragma unroll
    for (int k = 1; k < ROUNDS1; ++k) {
        rr[k] = rr[k - 1] + NT / W1;
        cc[k] = cc[k - 1] + NT % W1;
        if (cc[k] >= W1) {
            cc[k] -= W1;
            rr[k] += 1;
        }
    }
    // flag words first; every pull then reads either its upstream value or,
    // for a solid upstream node, the node's own opposite population: the
    // byte offset is n sz + K_q + (bit_q ? D_q : 0) with K_q, D_q uniform
    // (no branch, no second load)
#pragma unroll
    for (int k = 0; k < ROUNDS1; ++k) {
        const int i = x0 - 1 + cc[k], j = y0 - 1 + rr[k];
        m[k] = kMaskSolid;
        if (rr[k] < H1 && i >= 0 && j >= 0 && i < N && j < N)
            m[k] = __builtin_amdgcn_raw_buffer_load_b16(mrs, 2u * static_cast<unsigned>(j * P + i), 0, 0);
    }
    unsigned K[kQ], D[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const unsigned pull = q * SP - static_cast<unsigned>(kCx[q] + kCy[q] * P);
        const unsigned own = kOpp[q] * SP;
        K[q] = pull * sz;
        D[q] = (own - pull) * sz;            // modulo 2^32; the sum below is exact
    }
#pragma unroll
    for (int k = 0; k < ROUNDS1; ++k) {
        if (m[k] & kMaskSolid) continue;
        const int i = x0 - 1 + cc[k], j = y0 - 1 + rr[k];
        const unsigned n = static_cast<unsigned>(j * P + i);
        vx1[k] = Buf<float>::load(vxr, 4u * n, 0);
        vy1[k] = Buf<float>::load(vyr, 4u * n, 0);
        if (i >= 1 && j >= 1 && i <= N - 2 && j <= N - 2) {
            const unsigned nb = n * sz;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const unsigned sel = 0u - ((m[k] >> q) & 1u);
                raw[k][q] = Buf<S>::load(fsrc, nb + K[q] + (sel & D[q]), 0);
            }
        } else {
            // patch edge: upstream rows and columns clamped onto the patch
            const int jm = j > 0 ? j - 1 : 0, jp = j < N - 1 ? j + 1 : N - 1;
            const int il = i > 0 ? i - 1 : 0, ir = i < N - 1 ? i + 1 : N - 1;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int sj = kCy[q] == 1 ? jm : kCy[q] == -1 ? jp : j;
                const int si = kCx[q] == 1 ? il : kCx[q] == -1 ? ir : i;
                const unsigned pull = q * SP + static_cast<unsigned>(sj * P + si);
                const unsigned own = kOpp[q] * SP + n;
                raw[k][q] = Buf<S>::load(fsrc, (((m[k] >> q) & 1u) ? own : pull) * sz, 0);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < ROUNDS1; ++k) {
        if (m[k] & kMaskSolid) continue;
        const int r = rr[k], c = cc[k];
        const int i = x0 - 1 + c, j = y0 - 1 + r;
        const unsigned n = static_cast<unsigned>(j * P + i);
        const bool owned = r >= 1 && r <= TH && c >= 1 && c <= TW;
        T f[kQ];
        // raw already holds the bounce-back values; decode with the plane
        // each value came from
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const T pulled = Pop<S>::ld(raw[k][q], q, a);
            const T own = Pop<S>::ld(raw[k][q], kOpp[q], a);
            if constexpr (FLUX) f[q] = ((m[k] >> q) & 1u) ? reactive<T>(a, own, q) : pulled;
            else f[q] = ((m[k] >> q) & 1u) ? own : pulled;
        }
        if (edge && (i == 0 || j == 0 || i == N - 1 || j == N - 1)) {
            const bool bad = dirichlet_close<T>(a, f, outside_bits(N, i, j), perimeter_slot(N, i, j), a.lam);
            tally.bad += bad && owned;
        }
        const T u = collide<T>(f, T(vx1[k]), T(vy1[k]), omega, node_k<T>(a, static_cast<int>(n)));
        tally.nonfinite += owned && !finite_val(u);
        // the second half reads the first step's result in the arithmetic
        // type (FP16 shifted storage rounds to binary16 only at the store)
#pragma unroll
        for (int q = 0; q < kQ; ++q) lds[q][r][c] = f[q];
        if constexpr (MID) {
            // a recording forward keeps the intermediate state too, and u
            if (owned) {
                const BufRsrc fmid = buf_rsrc(a.mid, kQ * SP * sz);
#pragma unroll
                for (int q = 0; q < kQ; ++q) Buf<S>::store_nt(Pop<S>::st(f[q], q, a), fmid, n * sz, q * SP * sz);
                if (a.u_out) static_cast<T *>(a.u_out)[n] = u;
            }
        }
    }

    // flags and velocities of the owned nodes, fetched before the barrier
    unsigned m2[ROUNDS2];
    float vx2[ROUNDS2], vy2[ROUNDS2];
#pragma unroll
    for (int k = 0; k < ROUNDS2; ++k) {
        const int idx = threadIdx.x + NT * k;
        const int i = x0 + idx % TW, j = y0 + idx / TW;
        m2[k] = kMaskSolid;
        if (i < N && j < N) {
            const unsigned n = static_cast<unsigned>(j * P + i);
            m2[k] = __builtin_amdgcn_raw_buffer_load_b16(mrs, 2u * n, 0, 0);
            vx2[k] = Buf<float>::load(vxr, 4u * n, 0);
            vy2[k] = Buf<float>::load(vyr, 4u * n, 0);
        }
    }
    // dissolving solids: an owned solid node with fluid neighbours needs, for
    // step j+1, the populations f*_opp(q)(x + e_q) of the source buffer (the
    // first half fetched the same lines for the bounce-back of those
    // neighbours) and its running flux sum
    S g1[FLUX ? ROUNDS2 : 1][kQ];
    double fl2[FLUX ? ROUNDS2 : 1];
    if constexpr (FLUX) {
#pragma unroll
        for (int k = 0; k < ROUNDS2; ++k) {
            if (!(m2[k] & kMaskSolid) || !(m2[k] & 0x1FEu)) continue;
            const int idx = threadIdx.x + NT * k;
            const unsigned n = static_cast<unsigned>((y0 + idx / TW) * P + x0 + idx % TW);
#pragma unroll
            for (int q = 1; q < kQ; ++q) {
                const unsigned at = kOpp[q] * SP + static_cast<unsigned>(kCx[q] + kCy[q] * P);
                g1[k][q] = Buf<S>::load(fsrc, (n + at) * sz, 0);
            }
            fl2[k] = (a.flux_first || !a.flux) ? 0.0 : a.flux[n];
        }
    }
    __syncthreads();

    // ---- second half: step j+2 on the owned nodes, from LDS ------------
#pragma unroll
    for (int k = 0; k < ROUNDS2; ++k) {
        if (m2[k] & kMaskSolid) {
            if constexpr (FLUX) {
                if ((m2[k] & 0x1FEu) && a.flux) {
                    // sum over q of kappa_s (w_q c_sat - f*_opp(q)(x + e_q)),
                    // in q order, for step j+1 then step j+2
                    const int idx = threadIdx.x + NT * k;
                    const int r = idx / TW, c = idx % TW;
                    const T *base = &lds[0][0][0] + (r + 1) * W1 + (c + 1);
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int q = 1; q < kQ; ++q)
                        if ((m2[k] >> q) & 1u) {
                            s1 += a.kappa_s * (kW[q] * a.c_sat - double(Pop<S>::ld(g1[k][q], kOpp[q], a)));
                            const T x1 = base[kOpp[q] * (H1 * W1) + kCy[q] * W1 + kCx[q]];
                            s2 += a.kappa_s * (kW[q] * a.c_sat - double(x1));
                        }
                    a.flux[(y0 + r) * P + x0 + c] = (fl2[k] + s1) + s2;
                }
            }
            continue;
        }
        const int idx = threadIdx.x + NT * k;
        const int r = idx / TW, c = idx % TW;
        const int i = x0 + c, j = y0 + r;
        const unsigned n = static_cast<unsigned>(j * P + i);
        const bool perim = edge2 && (i == 0 || j == 0 || i == N - 1 || j == N - 1);
        const unsigned unknown = perim ? outside_bits(N, i, j) : 0u;
        T g[kQ];
        {
            // one LDS read per direction at a selected address (upstream
            // value, or the node's own opposite value for a solid upstream
            // node); closure unknowns are overwritten below
            const T *base = &lds[0][0][0] + (r + 1) * W1 + (c + 1);
#pragma unroll
            for (int q = 0; q < kQ; ++q)
                g[q] = *pull_or_back(base, m2[k], q, q * (H1 * W1) - kCy[q] * W1 - kCx[q], kOpp[q] * (H1 * W1));
            if constexpr (FLUX) {
#pragma unroll
                for (int q = 1; q < kQ; ++q)
                    if ((m2[k] >> q) & 1u) g[q] = reactive<T>(a, g[q], q);
            }
        }
        if (perim) {
            const bool bad = dirichlet_close<T>(a, g, unknown, perimeter_slot(N, i, j), a.lam2);
            tally.bad += bad;
        }
        const T u = collide<T>(g, T(vx2[k]), T(vy2[k]), omega, node_k<T>(a, static_cast<int>(n)));
        tally.nonfinite += !finite_val(u);
#pragma unroll
        for (int q = 0; q < kQ; ++q) Buf<S>::store_nt(Pop<S>::st(g[q], q, a), fdst, n * sz, q * SP * sz);
        if constexpr (MID) {
            if (a.u_out2) static_cast<T *>(a.u_out2)[n] = u;
        }
    }
    flush_tally<NT>(a, tally, edge);
}

template <typename S, int TW, int TH, int NT, int PART>
__global__ void __launch_bounds__(NT) lbm_sweep2_kernel(LbmArgs a, TileMap map) {
    sweep2_body<S, TW, TH, NT, PART, false>(a, map);
}

// whole-patch two-step launch with the surface reaction of dissolving solids
template <typename S, int TW, int TH, int NT>
__global__ void __launch_bounds__(NT) lbm_sweep2_flux_kernel(LbmArgs a, TileMap map) {
    sweep2_body<S, TW, TH, NT, 0, true>(a, map);
}

// whole-patch two-step launch that also stores the intermediate state (a.mid)
template <typename S, int TW, int TH, int NT>
__global__ void __launch_bounds__(NT) lbm_sweep2_rec_kernel(LbmArgs a, TileMap map) {
    sweep2_body<S, TW, TH, NT, 0, false, true>(a, map);
}

// the same with the surface reaction of dissolving solids and its link fluxes
template <typename S, int TW, int TH, int NT>
__global__ void __launch_bounds__(NT) lbm_sweep2_flux_rec_kernel(LbmArgs a, TileMap map) {
    sweep2_body<S, TW, TH, NT, 0, true, true>(a, map);
}

// ---------------------------------------------------------------------------
// K fine steps per launch (K = 3, 4)
// ---------------------------------------------------------------------------
// A workgroup owns a TW x TH tile.  Step j+1 runs on the tile grown by
// G = K-1 rings, from HBM into LDS (as the two-step kernel's first half, with
// wider rings); each next step runs on a region one ring narrower, from LDS,
// its results held in registers across a barrier and written back over the
// values they replace; step j+K runs on the owned nodes, from LDS, stored to
// HBM.  Every node takes the single step's operations, and values pass
// through the storage format between steps, so the result equals K single
// steps up to how the compiler fuses multiply-adds in each kernel (FP64
// states measured identical to the two-step launches', FP32 ones within a
// few ulp).  The state crosses HBM once per K fine steps; the first
// stage does (TW+2G)(TH+2G) / ((TW+2)(TH+2)) of the two-step kernel's
// first-half work (1.24 at K = 3, 1.48 at K = 4 for 64 x 8).

// interface weight of stage s (1-based) of a multi-step launch
__device__ __forceinline__ double stage_lam(const LbmArgs &a, int s) {
    return s == 1 ? a.lam : s == 2 ? a.lam2 : s == 3 ? a.lam3 : s == 4 ? a.lam4 : a.lam5;
}

// Row and column of each round's node in a W-wide region of R nodes, NT
// lanes per round, stepped without divisions.
template <int W, int NT, int ROUNDS>
__device__ __forceinline__ void region_coords(int (&rr)[ROUNDS], int (&cc)[ROUNDS]) {
    rr[0] = threadIdx.x / W;
    cc[0] = threadIdx.x - rr[0] * W;
#pragma unroll
    for (int k = 1; k < ROUNDS; ++k) {
        rr[k] = rr[k - 1] + NT / W;
        cc[k] = cc[k - 1] + NT % W;
        if (cc[k] >= W) {
            cc[k] -= W;
            rr[k] += 1;
        }
    }
}

template <int TW, int TH, int NT, int RING>
struct Region {
    static constexpr int W = TW + 2 * RING, H = TH + 2 * RING, ROUNDS = (W * H + NT - 1) / NT;
};

// Flags and velocities of the nodes of the RING-ring region (solid flag for
// rounds past the region or nodes off the patch).
template <int TW, int TH, int NT, int RING>
__device__ __forceinline__ void region_fields(int N, int P, int x0, int y0, const BufRsrc &mrs, const BufRsrc &vxr,
                                              const BufRsrc &vyr, unsigned (&m)[Region<TW, TH, NT, RING>::ROUNDS],
                                              float (&vx)[Region<TW, TH, NT, RING>::ROUNDS],
                                              float (&vy)[Region<TW, TH, NT, RING>::ROUNDS],
                                              int (&rr)[Region<TW, TH, NT, RING>::ROUNDS],
                                              int (&cc)[Region<TW, TH, NT, RING>::ROUNDS]) {
    typedef Region<TW, TH, NT, RING> R;
    region_coords<R::W, NT, R::ROUNDS>(rr, cc);
#pragma unroll
    for (int k = 0; k < R::ROUNDS; ++k) {
        const int i = x0 - RING + cc[k], j = y0 - RING + rr[k];
        m[k] = kMaskSolid;
        if (rr[k] < R::H && i >= 0 && j >= 0 && i < N && j < N) {
            const unsigned n = static_cast<unsigned>(j * P + i);
            m[k] = __builtin_amdgcn_raw_buffer_load_b16(mrs, 2u * n, 0, 0);
            vx[k] = Buf<float>::load(vxr, 4u * n, 0);
            vy[k] = Buf<float>::load(vyr, 4u * n, 0);
        }
    }
}

// Stages after the first: step j + G + 1 - RING on the RING-ring region from
// LDS (LDS array of the G-ring region, W0 wide, planes PL apart).  RING > 0:
// results to registers, the next region's fields fetched, barrier, results
// written back in place, barrier, next stage.  RING = 0: the owned nodes,
// stored to HBM.
template <typename S, int TW, int TH, int NT, int G, int RING, bool FLUX, bool EDGE>
__device__ __forceinline__ void later_stages(const LbmArgs &a, typename Pop<S>::T *L0, int x0, int y0,
                                             const BufRsrc &fdst, const BufRsrc &mrs, const BufRsrc &vxr,
                                             const BufRsrc &vyr,
                                             const unsigned (&m)[Region<TW, TH, NT, RING>::ROUNDS],
                                             const float (&vx)[Region<TW, TH, NT, RING>::ROUNDS],
                                             const float (&vy)[Region<TW, TH, NT, RING>::ROUNDS],
                                             const int (&rr)[Region<TW, TH, NT, RING>::ROUNDS],
                                             const int (&cc)[Region<TW, TH, NT, RING>::ROUNDS],
                                             const unsigned (&mo)[TW * TH / NT], double (&acc)[TW * TH / NT],
                                             Tally &tally) {
    typedef typename Pop<S>::T T;
    typedef Region<TW, TH, NT, RING> R;
    constexpr int W0 = TW + 2 * G, H0 = TH + 2 * G, PL = H0 * W0;
    constexpr int OFF = G - RING;               // region origin in LDS coordinates
    constexpr int STAGE = G + 1 - RING;
    static_assert(sizeof(T) * kQ * PL < (1u << 23), "pull_or_back: LDS byte offsets within 24 bits");
    constexpr unsigned sz = sizeof(S);
    const int N = a.N;
    const int P = a.pitch;
    const unsigned SP = static_cast<unsigned>(a.plane);
    const T omega = T(a.omega);
    const double lam = stage_lam(a, STAGE);
    // EDGE false: the caller found that no stage of this tile reaches the
    // perimeter, so the node loop carries no perimeter test or closure
    const bool edge = EDGE && reaches_perimeter(N, x0, y0, TW, TH, RING);
    T h[R::ROUNDS][kQ];
#pragma unroll
    for (int k = 0; k < R::ROUNDS; ++k) {
        if (m[k] & kMaskSolid) continue;
        const int r = rr[k], c = cc[k];
        const int i = x0 - RING + c, j = y0 - RING + r;
        const unsigned n = static_cast<unsigned>(j * P + i);
        const bool owned = r >= RING && r < RING + TH && c >= RING && c < RING + TW;
        const bool perim = edge && (i == 0 || j == 0 || i == N - 1 || j == N - 1);
        // one LDS read per direction at a selected address (upstream value,
        // or the node's own opposite value for a solid upstream node);
        // closure unknowns are overwritten below
        const T *base = L0 + (r + OFF) * W0 + (c + OFF);
#pragma unroll
        for (int q = 0; q < kQ; ++q) h[k][q] = *pull_or_back(base, m[k], q, q * PL - kCy[q] * W0 - kCx[q], kOpp[q] * PL);
        if constexpr (FLUX) {
#pragma unroll
            for (int q = 1; q < kQ; ++q)
                if ((m[k] >> q) & 1u) h[k][q] = reactive<T>(a, h[k][q], q);
        }
        if (perim) {
            const bool bad = dirichlet_close<T>(a, h[k], outside_bits(N, i, j), perimeter_slot(N, i, j), lam);
            tally.bad += bad && owned;
        }
        const T u = collide<T>(h[k], T(vx[k]), T(vy[k]), omega, node_k<T>(a, static_cast<int>(n)));
        tally.nonfinite += owned && !finite_val(u);
        if constexpr (RING == 0) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) Buf<S>::store_nt(Pop<S>::st(h[k][q], q, a), fdst, n * sz, q * SP * sz);
        }
    }
    if constexpr (FLUX) {
        // link fluxes of this step at the owned solid nodes, in q order, from
        // the step's input (still in LDS: the write-back comes after the
        // barrier below)
        constexpr int RO = TW * TH / NT;
#pragma unroll
        for (int k = 0; k < RO; ++k) {
            if (!(mo[k] & kMaskSolid) || !(mo[k] & 0x1FEu)) continue;
            const int idx = threadIdx.x + NT * k;
            const T *base = L0 + (idx / TW + G) * W0 + (idx % TW + G);
            double s = 0.0;
#pragma unroll
            for (int q = 1; q < kQ; ++q)
                if ((mo[k] >> q) & 1u)
                    s += a.kappa_s * (kW[q] * a.c_sat - double(base[kOpp[q] * PL + kCy[q] * W0 + kCx[q]]));
            acc[k] += s;
            if constexpr (RING == 0) {
                if (a.flux) a.flux[(y0 + idx / TW) * P + x0 + idx % TW] = acc[k];
            }
        }
    }
    if constexpr (RING > 0) {
        typedef Region<TW, TH, NT, RING - 1> R2;
        unsigned m2[R2::ROUNDS];
        float vx2[R2::ROUNDS], vy2[R2::ROUNDS];
        int rr2[R2::ROUNDS], cc2[R2::ROUNDS];
        region_fields<TW, TH, NT, RING - 1>(N, P, x0, y0, mrs, vxr, vyr, m2, vx2, vy2, rr2, cc2);
        __syncthreads();             // every read of this stage's inputs is done
#pragma unroll
        for (int k = 0; k < R::ROUNDS; ++k) {
            if (m[k] & kMaskSolid) continue;
#pragma unroll
            for (int q = 0; q < kQ; ++q) L0[q * PL + (rr[k] + OFF) * W0 + (cc[k] + OFF)] = h[k][q];
        }
        __syncthreads();
        later_stages<S, TW, TH, NT, G, RING - 1, FLUX, EDGE>(a, L0, x0, y0, fdst, mrs, vxr, vyr, m2, vx2, vy2, rr2,
                                                            cc2, mo, acc, tally);
    }
}

template <typename S, int TW, int TH, int NT, int PART, int K, bool FLUX = false>
__device__ __forceinline__ void sweepk_body(const LbmArgs &a, const TileMap &map) {
    typedef typename Pop<S>::T T;
    static_assert(K >= 3, "two-step launches use sweep2_body");
    static_assert((TW * TH) % NT == 0 && NT % TW == 0, "last stage: whole rows per round");
    constexpr int G = K - 1;
    typedef Region<TW, TH, NT, G> R0;
    constexpr int W0 = R0::W, H0 = R0::H, ROUNDS0 = R0::ROUNDS;
    constexpr unsigned sz = sizeof(S);
    __shared__ T lds[kQ][H0][W0];

    const int N = a.N;
    const int P = a.pitch;
    const unsigned SP = static_cast<unsigned>(a.plane);
    const unsigned NP = static_cast<unsigned>(N) * static_cast<unsigned>(P);
    const BufRsrc fsrc = buf_rsrc(a.src, kQ * SP * sz);
    const BufRsrc fdst = buf_rsrc(a.dst, kQ * SP * sz);
    const BufRsrc mrs = buf_rsrc(a.mask, NP * 2u);
    const BufRsrc vxr = buf_rsrc(a.vx, NP * 4u);
    const BufRsrc vyr = buf_rsrc(a.vy, NP * 4u);
    const T omega = T(a.omega);
    int tx, ty;
    tile_of<PART>(map, xcd_tile(blockIdx.x, map.count), tx, ty);
    const int x0 = tx * TW;
    const int y0 = ty * TH;
    const bool edge = reaches_perimeter(N, x0, y0, TW, TH, G);
    Tally tally;

    // dissolving solids: flag words of the owned nodes, and for each owned
    // solid node with fluid neighbours its running flux sum (the previous
    // steps' sum unless this launch starts the pass) plus the link fluxes
    // of step j+1, from the source buffer (the lines the bounce-back of its
    // neighbours fetches)
    constexpr int RO = TW * TH / NT;
    unsigned mo[RO];
    double acc[RO];
    if constexpr (FLUX) {
#pragma unroll
        for (int k = 0; k < RO; ++k) {
            const int idx = threadIdx.x + NT * k;
            const int i = x0 + idx % TW, j = y0 + idx / TW;
            mo[k] = 0u;
            acc[k] = 0.0;
            if (i < N && j < N)
                mo[k] = __builtin_amdgcn_raw_buffer_load_b16(mrs, 2u * static_cast<unsigned>(j * P + i), 0, 0);
        }
#pragma unroll
        for (int k = 0; k < RO; ++k) {
            if (!(mo[k] & kMaskSolid) || !(mo[k] & 0x1FEu)) continue;
            const int idx = threadIdx.x + NT * k;
            const unsigned n = static_cast<unsigned>((y0 + idx / TW) * P + x0 + idx % TW);
            double s = 0.0;
#pragma unroll
            for (int q = 1; q < kQ; ++q)
                if ((mo[k] >> q) & 1u) {
                    const unsigned at = kOpp[q] * SP + static_cast<unsigned>(kCx[q] + kCy[q] * P);
                    s += a.kappa_s *
                         (kW[q] * a.c_sat - double(Pop<S>::ld(Buf<S>::load(fsrc, (n + at) * sz, 0), kOpp[q], a)));
                }
            acc[k] = ((a.flux_first || !a.flux) ? 0.0 : a.flux[n]) + s;
        }
    }

    // The stages run in one of two compiled copies: tiles whose widest
    // region reaches the perimeter take the perimeter tests, the clamped
    // patch-edge loads and the closures; every other tile (most of them) a
    // copy without them.
    auto stages = [&](auto edge_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
        // ---- stage 1: step j+1 on the tile and G rings, HBM -> LDS ----------
        S raw[ROUNDS0][kQ];
        unsigned m[ROUNDS0];
        float vx1[ROUNDS0], vy1[ROUNDS0];
        int rr[ROUNDS0], cc[ROUNDS0];
        region_coords<W0, NT, ROUNDS0>(rr, cc);
#pragma unroll
        for (int k = 0; k < ROUNDS0; ++k) {
            const int i = x0 - G + cc[k], j = y0 - G + rr[k];
            m[k] = kMaskSolid;
            if (rr[k] < H0 && (!EDGE || (i >= 0 && j >= 0 && i < N && j < N)))
                m[k] = __builtin_amdgcn_raw_buffer_load_b16(mrs, 2u * static_cast<unsigned>(j * P + i), 0, 0);
        }
        unsigned Kq[kQ], Dq[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const unsigned pull = q * SP - static_cast<unsigned>(kCx[q] + kCy[q] * P);
            const unsigned own = kOpp[q] * SP;
            Kq[q] = pull * sz;
            Dq[q] = (own - pull) * sz;           // modulo 2^32; the sum below is exact
        }
#pragma unroll
        for (int k = 0; k < ROUNDS0; ++k) {
            if (m[k] & kMaskSolid) continue;
            const int i = x0 - G + cc[k], j = y0 - G + rr[k];
            const unsigned n = static_cast<unsigned>(j * P + i);
            vx1[k] = Buf<float>::load(vxr, 4u * n, 0);
            vy1[k] = Buf<float>::load(vyr, 4u * n, 0);
            if (!EDGE || (i >= 1 && j >= 1 && i <= N - 2 && j <= N - 2)) {
                const unsigned nb = n * sz;
#pragma unroll
                for (int q = 0; q < kQ; ++q) {
                    const unsigned sel = 0u - ((m[k] >> q) & 1u);
                    raw[k][q] = Buf<S>::load(fsrc, nb + Kq[q] + (sel & Dq[q]), 0);
                }
            } else {
                const int jm = j > 0 ? j - 1 : 0, jp = j < N - 1 ? j + 1 : N - 1;
                const int il = i > 0 ? i - 1 : 0, ir = i < N - 1 ? i + 1 : N - 1;
#pragma unroll
                for (int q = 0; q < kQ; ++q) {
                    const int sj = kCy[q] == 1 ? jm : kCy[q] == -1 ? jp : j;
                    const int si = kCx[q] == 1 ? il : kCx[q] == -1 ? ir : i;
                    const unsigned pull = q * SP + static_cast<unsigned>(sj * P + si);
                    const unsigned own = kOpp[q] * SP + n;
                    raw[k][q] = Buf<S>::load(fsrc, (((m[k] >> q) & 1u) ? own : pull) * sz, 0);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ROUNDS0; ++k) {
            if (m[k] & kMaskSolid) continue;
            const int r = rr[k], c = cc[k];
            const int i = x0 - G + c, j = y0 - G + r;
            const unsigned n = static_cast<unsigned>(j * P + i);
            const bool owned = r >= G && r < G + TH && c >= G && c < G + TW;
            T f[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const T pulled = Pop<S>::ld(raw[k][q], q, a);
                const T own = Pop<S>::ld(raw[k][q], kOpp[q], a);
                if constexpr (FLUX) f[q] = ((m[k] >> q) & 1u) ? reactive<T>(a, own, q) : pulled;
                else f[q] = ((m[k] >> q) & 1u) ? own : pulled;
            }
            if (EDGE && (i == 0 || j == 0 || i == N - 1 || j == N - 1)) {
                const bool bad = dirichlet_close<T>(a, f, outside_bits(N, i, j), perimeter_slot(N, i, j), a.lam);
                tally.bad += bad && owned;
            }
            const T u = collide<T>(f, T(vx1[k]), T(vy1[k]), omega, node_k<T>(a, static_cast<int>(n)));
            tally.nonfinite += owned && !finite_val(u);
#pragma unroll
            for (int q = 0; q < kQ; ++q) lds[q][r][c] = f[q];
        }

        // the next region's flags and velocities, fetched before the barrier
        typedef Region<TW, TH, NT, G - 1> R1;
        unsigned m1[R1::ROUNDS];
        float vx2[R1::ROUNDS], vy2[R1::ROUNDS];
        int r1[R1::ROUNDS], c1[R1::ROUNDS];
        region_fields<TW, TH, NT, G - 1>(N, P, x0, y0, mrs, vxr, vyr, m1, vx2, vy2, r1, c1);
        __syncthreads();
        later_stages<S, TW, TH, NT, G, G - 1, FLUX, EDGE>(a, &lds[0][0][0], x0, y0, fdst, mrs, vxr, vyr, m1, vx2,
                                                          vy2, r1, c1, mo, acc, tally);
    };
    if (edge) stages(std::true_type{});
    else stages(std::false_type{});
    flush_tally<NT>(a, tally, edge);
}

template <typename S, int TW, int TH, int NT, int PART>
__global__ void __launch_bounds__(NT) lbm_sweep3_kernel(LbmArgs a, TileMap map) {
    sweepk_body<S, TW, TH, NT, PART, 3>(a, map);
}

template <typename S, int TW, int TH, int NT, int PART>
__global__ void __launch_bounds__(NT) lbm_sweep4_kernel(LbmArgs a, TileMap map) {
    sweepk_body<S, TW, TH, NT, PART, 4>(a, map);
}

template <typename S, int TW, int TH, int NT, int PART>
__global__ void __launch_bounds__(NT) lbm_sweep5_kernel(LbmArgs a, TileMap map) {
    sweepk_body<S, TW, TH, NT, PART, 5>(a, map);
}

// whole-patch K-step launch with the surface reaction of dissolving solids
template <typename S, int TW, int TH, int NT, int K>
__global__ void __launch_bounds__(NT) lbm_sweepk_flux_kernel(LbmArgs a, TileMap map) {
    sweepk_body<S, TW, TH, NT, 0, K, true>(a, map);
}

// ---------------------------------------------------------------------------
// initial state: f*(0) = collide(f^eq(u0)) at fluid nodes (Sec. 6.2, item i)
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256) lbm_init_kernel(LbmArgs a, const double *__restrict__ u0) {
    typedef typename Pop<S>::T T;
    const int N = a.N;
    const int j = blockIdx.x;
    const int P = a.pitch;
    const int plane = static_cast<int>(a.plane);
    S *__restrict__ dst = static_cast<S *>(a.dst);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int n = j * P + i;
        if (a.mask[n] & kMaskSolid) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) dst[q * plane + n] = S(0);
            continue;
        }
        T f[kQ];
        const T u = T(u0[j * N + i]);
        const T vx = T(a.vx[n]), vy = T(a.vy[n]);
        const T usq = T(1.5) * (vx * vx + vy * vy);
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const T ev = T(kCx[q]) * vx + T(kCy[q]) * vy;
            f[q] = T(kW[q]) * u * (T(1) + T(3) * ev + T(4.5) * ev * ev - usq);
        }
        collide<T>(f, vx, vy, T(a.omega), node_k<T>(a, n));
#pragma unroll
        for (int q = 0; q < kQ; ++q) dst[q * plane + n] = Pop<S>::st(f[q], q, a);
    }
}

// u = sum_i f*_i / (1 - k): the collision removes k u from the node's mass.
template <typename S>
__global__ void __launch_bounds__(256) lbm_conc_kernel(LbmArgs a, double *__restrict__ out) {
    typedef typename Pop<S>::T T;
    const int N = a.N;
    const int j = blockIdx.x;
    const int P = a.pitch;
    const int plane = static_cast<int>(a.plane);
    const S *__restrict__ src = static_cast<const S *>(a.src);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int n = j * P + i;
        double u = 0.0;
        if (!(a.mask[n] & kMaskSolid)) {
            for (int q = 0; q < kQ; ++q) u += double(Pop<S>::ld(src[q * plane + n], q, a));
            u /= (1.0 - double(node_k<T>(a, n)));
        }
        out[j * N + i] = u;
    }
}

template <typename S>
hipError_t step_impl(const LbmArgs &a, bool general_perimeter, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int np = 4 * (a.N - 1);
    const int row_blocks = (a.N - 2 + 255) / 256;
    const int interior_blocks = row_blocks * (a.N - 2);
    if (e0) (void)hipEventRecord(e0, s);
    if (!general_perimeter) {
        const int per_blocks = (np + 255) / 256;
        hipLaunchKernelGGL(lbm_sweep_kernel<S>, dim3(interior_blocks + per_blocks), dim3(256), 0, s, a,
                           interior_blocks, row_blocks);
        if (e1) (void)hipEventRecord(e1, s);
    } else {
        if (interior_blocks > 0) {
            if (a.wall_nx)
                hipLaunchKernelGGL((lbm_bulk_kernel<S, true>), dim3(interior_blocks), dim3(256), 0, s, a, row_blocks);
            else
                hipLaunchKernelGGL((lbm_bulk_kernel<S, false>), dim3(interior_blocks), dim3(256), 0, s, a,
                                   row_blocks);
        }
        if (e1) (void)hipEventRecord(e1, s);
        hipLaunchKernelGGL(lbm_perimeter_kernel<S>, dim3((np + 127) / 128), dim3(128), 0, s, a);
    }
    return hipGetLastError();
}

// Tile shape of the two-step sweep: LDS holds 9 planes of (TW+2) x (TH+2)
// values of the arithmetic type.  64 x 8 tiles: 23.8 KB of LDS with FP32
// arithmetic (256 lanes, six workgroups per CU), 47.5 KB in FP64 (512 lanes,
// three workgroups per CU).  Measured on the 2048^2 and 4096^2 pore
// workloads: FP32 64 x 8 ran 14% faster than 64 x 16 with 256 lanes and the
// same as 64 x 16 with 512 lanes; 64 x 24 and 64 x 32 (1024 lanes) were
// slower at 2048^2.  FP64 with 512 lanes ran 4-7% faster than with 256.
#ifndef SWEEP2_TH32
#define SWEEP2_TH32 8
#endif
#ifndef SWEEP2_NT32
#define SWEEP2_NT32 256
#endif
#ifndef SWEEP2_TH64
#define SWEEP2_TH64 8
#endif
#ifndef SWEEP2_NT64
#define SWEEP2_NT64 512
#endif
#ifndef SWEEP2_TW32
#define SWEEP2_TW32 64
#endif
#ifndef SWEEP2_TW64
#define SWEEP2_TW64 64
#endif
template <typename S> struct Tile2 { static constexpr int TW = SWEEP2_TW32, TH = SWEEP2_TH32, NT = SWEEP2_NT32; };
template <> struct Tile2<double> { static constexpr int TW = SWEEP2_TW64, TH = SWEEP2_TH64, NT = SWEEP2_NT64; };

template <typename S>
hipError_t step2_impl(const LbmArgs &a, int part, int depth, int ring, hipStream_t s) {
    constexpr int TW = Tile2<S>::TW, TH = Tile2<S>::TH, NT = Tile2<S>::NT;
    TileMap m{};
    m.tiles_x = (a.N + TW - 1) / TW;
    m.tiles_y = (a.N + TH - 1) / TH;
    m.part = part;
    // depth-0 rectangle: tiles whose ring of `ring` nodes (x0 - ring ..
    // x0 + TW - 1 + ring, likewise in y) lies within columns and rows
    // 1 .. N-2 (all full tiles); depth d shrinks it by d tiles on every side.
    // The kernel reads a one-node ring; ring 2 gives the rectangles of the
    // three-step launches of the same pass, so the rectangles of successive
    // launches nest.
    const int lx = a.N - 1 - ring - TW, ly = a.N - 1 - ring - TH;
    const bool fits = lx >= TW && ly >= TH;
    m.ix0 = 1 + depth;
    m.iy0 = 1 + depth;
    m.ix1 = (fits ? lx / TW : 0) - depth;
    m.iy1 = (fits ? ly / TH : 0) - depth;
    const bool has_rect = fits && m.ix1 >= m.ix0 && m.iy1 >= m.iy0;
    const int all = m.tiles_x * m.tiles_y;
    const int inner = has_rect ? (m.ix1 - m.ix0 + 1) * (m.iy1 - m.iy0 + 1) : 0;
    if (part != 0 && !has_rect) {
        // empty rectangle: part 1 is empty, part 2 is everything
        if (part == 1) return hipSuccess;
        m.part = 0;
    }
    m.count = m.part == 0 ? all : m.part == 1 ? inner : all - inner;
    if (m.count == 0) return hipSuccess;
    if (a.flux || a.kappa_s != 0.0) {
        // dissolving solids: whole-patch launches only
        if (m.part != 0) return hipErrorInvalidValue;
        if (a.mid)
            hipLaunchKernelGGL((lbm_sweep2_flux_rec_kernel<S, TW, TH, NT>), dim3(m.count), dim3(NT), 0, s, a, m);
        else
            hipLaunchKernelGGL((lbm_sweep2_flux_kernel<S, TW, TH, NT>), dim3(m.count), dim3(NT), 0, s, a, m);
        return hipGetLastError();
    }
    if (a.mid) {
        if (m.part != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((lbm_sweep2_rec_kernel<S, TW, TH, NT>), dim3(m.count), dim3(NT), 0, s, a, m);
        return hipGetLastError();
    }
    if (m.part == 0) hipLaunchKernelGGL((lbm_sweep2_kernel<S, TW, TH, NT, 0>), dim3(m.count), dim3(NT), 0, s, a, m);
    else if (m.part == 1) hipLaunchKernelGGL((lbm_sweep2_kernel<S, TW, TH, NT, 1>), dim3(m.count), dim3(NT), 0, s, a, m);
    else hipLaunchKernelGGL((lbm_sweep2_kernel<S, TW, TH, NT, 2>), dim3(m.count), dim3(NT), 0, s, a, m);
    return hipGetLastError();
}

// Tile of the multi-step sweeps (K = 3, 4): 64 x 8 owned nodes, 512 lanes
// (one owned node per lane in the last stage); LDS holds 9 planes of
// (TW+2K-2) x (TH+2K-2) values of the arithmetic type: 29.4 / 35.3 KB in
// FP32, 58.8 / 70.6 KB in FP64.  Measured at pore2048 FP32 (4 + 3 + 3 per
// pass): 0.783 ms per coarse step against 0.832 with 256 lanes; 64 x 16
// with 512 lanes 0.808, 64 x 12 with 384 lanes 0.854.  In FP64, 512 lanes
// cut the sweep time per pass by 4.6% against the two-step launches.
template <typename S> struct Tile3 { static constexpr int TW = 64, TH = 8, NT = 512; };

template <typename S, int K>
hipError_t stepk_impl(const LbmArgs &a, int part, int depth, int ring, hipStream_t s) {
    constexpr int TW = Tile3<S>::TW, TH = Tile3<S>::TH, NT = Tile3<S>::NT;
    TileMap m{};
    m.tiles_x = (a.N + TW - 1) / TW;
    m.tiles_y = (a.N + TH - 1) / TH;
    m.part = part;
    // depth-0 rectangle: tiles whose ring of `ring` >= K-1 nodes lies within
    // columns and rows 1 .. N-2; depth d shrinks it by d tiles on every side
    // (a tile's ring lies within its neighbour tiles, which the previous
    // launch's rectangle of depth d - 1 covers)
    if (ring < K - 1) ring = K - 1;
    const int lx = a.N - 1 - ring - TW, ly = a.N - 1 - ring - TH;
    const bool fits = lx >= TW && ly >= TH;
    m.ix0 = 1 + depth;
    m.iy0 = 1 + depth;
    m.ix1 = (fits ? lx / TW : 0) - depth;
    m.iy1 = (fits ? ly / TH : 0) - depth;
    const bool has_rect = fits && m.ix1 >= m.ix0 && m.iy1 >= m.iy0;
    const int all = m.tiles_x * m.tiles_y;
    const int inner = has_rect ? (m.ix1 - m.ix0 + 1) * (m.iy1 - m.iy0 + 1) : 0;
    if (part != 0 && !has_rect) {
        if (part == 1) return hipSuccess;
        m.part = 0;
    }
    m.count = m.part == 0 ? all : m.part == 1 ? inner : all - inner;
    if (m.count == 0) return hipSuccess;
    if (a.mid) return hipErrorInvalidValue;
    if (a.flux || a.kappa_s != 0.0) {
        // dissolving solids: whole-patch launches only
        if (m.part != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((lbm_sweepk_flux_kernel<S, TW, TH, NT, K>), dim3(m.count), dim3(NT), 0, s, a, m);
        return hipGetLastError();
    }
    if constexpr (K == 3) {
        if (m.part == 0) hipLaunchKernelGGL((lbm_sweep3_kernel<S, TW, TH, NT, 0>), dim3(m.count), dim3(NT), 0, s, a, m);
        else if (m.part == 1) hipLaunchKernelGGL((lbm_sweep3_kernel<S, TW, TH, NT, 1>), dim3(m.count), dim3(NT), 0, s, a, m);
        else hipLaunchKernelGGL((lbm_sweep3_kernel<S, TW, TH, NT, 2>), dim3(m.count), dim3(NT), 0, s, a, m);
    } else if constexpr (K == 4) {
        if (m.part == 0) hipLaunchKernelGGL((lbm_sweep4_kernel<S, TW, TH, NT, 0>), dim3(m.count), dim3(NT), 0, s, a, m);
        else if (m.part == 1) hipLaunchKernelGGL((lbm_sweep4_kernel<S, TW, TH, NT, 1>), dim3(m.count), dim3(NT), 0, s, a, m);
        else hipLaunchKernelGGL((lbm_sweep4_kernel<S, TW, TH, NT, 2>), dim3(m.count), dim3(NT), 0, s, a, m);
    } else {
        if (m.part == 0) hipLaunchKernelGGL((lbm_sweep5_kernel<S, TW, TH, NT, 0>), dim3(m.count), dim3(NT), 0, s, a, m);
        else if (m.part == 1) hipLaunchKernelGGL((lbm_sweep5_kernel<S, TW, TH, NT, 1>), dim3(m.count), dim3(NT), 0, s, a, m);
        else hipLaunchKernelGGL((lbm_sweep5_kernel<S, TW, TH, NT, 2>), dim3(m.count), dim3(NT), 0, s, a, m);
    }
    return hipGetLastError();
}

template <typename S>
hipError_t stepk_dispatch(const LbmArgs &a, int K, int part, int depth, int ring, hipStream_t s) {
    if (K == 3) return stepk_impl<S, 3>(a, part, depth, ring, s);
    if (K == 4) return stepk_impl<S, 4>(a, part, depth, ring, s);
    if (K == 5) return stepk_impl<S, 5>(a, part, depth, ring, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_lbm_stepk(const LbmArgs &a, int prec, int K, hipStream_t s, int part, int depth, int ring) {
    if (prec == HYB_FP32) return stepk_dispatch<float>(a, K, part, depth, ring, s);
    if (prec == HYB_FP16S) return stepk_dispatch<_Float16>(a, K, part, depth, ring, s);
    if (prec == HYB_FP64) return stepk_dispatch<double>(a, K, part, depth, ring, s);
    return hipErrorInvalidValue;
}

hipError_t launch_lbm_step2(const LbmArgs &a, int prec, hipStream_t s, int part, int depth, int ring) {
    if (ring < 1 || ring > 4) return hipErrorInvalidValue;
    if (prec == HYB_FP64) return step2_impl<double>(a, part, depth, ring, s);
    if (prec == HYB_FP32) return step2_impl<float>(a, part, depth, ring, s);
    return step2_impl<_Float16>(a, part, depth, ring, s);
}

hipError_t launch_lbm_step(const LbmArgs &a, int prec, bool general_perimeter, hipStream_t s,
                           hipEvent_t sweep_begin, hipEvent_t sweep_end) {
    if (prec == HYB_FP64) return step_impl<double>(a, general_perimeter, s, sweep_begin, sweep_end);
    if (prec == HYB_FP32) return step_impl<float>(a, general_perimeter, s, sweep_begin, sweep_end);
    return step_impl<_Float16>(a, general_perimeter, s, sweep_begin, sweep_end);
}

hipError_t launch_lbm_init(const LbmArgs &a, const double *u0, int prec, hipStream_t s) {
    if (prec == HYB_FP64) hipLaunchKernelGGL(lbm_init_kernel<double>, dim3(a.N), dim3(256), 0, s, a, u0);
    else if (prec == HYB_FP32) hipLaunchKernelGGL(lbm_init_kernel<float>, dim3(a.N), dim3(256), 0, s, a, u0);
    else hipLaunchKernelGGL(lbm_init_kernel<_Float16>, dim3(a.N), dim3(256), 0, s, a, u0);
    return hipGetLastError();
}

hipError_t launch_concentration(const LbmArgs &a, double *out, int prec, hipStream_t s) {
    if (prec == HYB_FP64) hipLaunchKernelGGL(lbm_conc_kernel<double>, dim3(a.N), dim3(256), 0, s, a, out);
    else if (prec == HYB_FP32) hipLaunchKernelGGL(lbm_conc_kernel<float>, dim3(a.N), dim3(256), 0, s, a, out);
    else hipLaunchKernelGGL(lbm_conc_kernel<_Float16>, dim3(a.N), dim3(256), 0, s, a, out);
    return hipGetLastError();
}

}  // namespace hyb
