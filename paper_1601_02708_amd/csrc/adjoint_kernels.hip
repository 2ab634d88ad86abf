// Reverse mode (adjoint) of the fine step, for the differentiation form of
// the lattice sub-stepping.  One fine step maps f*(t) to f*(t+1) through
// pull streaming with halfway bounce-back, the Dirichlet closure of eq.
// (LBM_Dir) at perimeter nodes, and the BGK + reaction collision; with the
// closure applied as printed the step is linear in (f*(t), u^p) for fixed
// velocity and reaction rate.  Its adjoint, given l = dJ/df*(t+1):
//
//   collision   mu_p = (1 - w) l_p + sum_q l_q w_q (w P_q(v) - k)
//               dJ/dk(x) += -u(x) sum_q w_q l_q
//   closure     G = sum_U w_U mu_U / W;  nu_K = mu_K - G;  nu_U = 0;
//               dJ/du^p += G  (G = 0 where the closure was clamped at 0)
//   streaming   dJ/df*_p(y) = nu_p(y + e_p)   if y + e_p is a fluid node
//                                             of the patch (it pulled f*_p(y))
//                           + nu_q(y), q = opp(p), if y bounced back along q
//
// (P_q(v) = 1 + 3 e.v + 9/2 (e.v)^2 - 3/2 v.v, w = 1/tau).  The first two
// are local to a node, the last gathers from the neighbours: one kernel per
// reversed step computes nu for a 64 x 8 tile and its one-node ring into LDS
// and then gathers the tile's outputs from there, so nu never goes to HBM.
// The forward states of the step come from the tape recorded by the forward
// sweep.
#include "hyb_impl.h"

#include <type_traits>

namespace hyb {
namespace {

__device__ __forceinline__ int slot_of(int N, int i, int j) {
    if (j == 0) return i;
    if (j == N - 1) return N + i;
    if (i == 0) return 2 * N + j - 1;
    return 3 * N - 2 + j - 1;
}

// Dense FP64 ends of a reversed sweep, folded into its first and last
// launches: lam_dense (or null) is read in place of the pitched cotangent
// (index (q*N + j)*N + i, converted to T as a separate packing pass would),
// out_dense (or null) receives the output in that layout (added to it when
// accumulate), in place of the pitched output.
struct AdjDense {
    const double *lam_dense;
    double *out_dense;
    int accumulate;
};

__device__ __forceinline__ size_t dense_at(int N, int q, int i, int j) {
    return ((size_t)q * N + j) * N + i;
}

// nu at node (i, j) (collision and closure transposed) from the node's
// cotangent l = dJ/df*(t+1); gradients of the closure and the reaction rate
// are accumulated when `owner` (every node has exactly one owner tile, ring
// copies recompute nu only).  The dJ/dk term of the step goes to *stash
// when given (a paired launch then adds both steps' terms at once), else
// grad_k becomes (grad_k - prior) - term: prior is the term of the reversed
// step before, held back, so the sum is that of two separate updates.
template <typename T, bool EDGE = true>
__device__ __forceinline__ void adj_nu_of(const LbmArgs &a, int i, int j, const T *__restrict__ snext,
                                          const T (&l)[kQ], bool owner, double *__restrict__ grad_a,
                                          double *__restrict__ grad_b, double *__restrict__ grad_k, T (&nu)[kQ],
                                          double *stash = nullptr, double prior = 0.0) {
    const int N = a.N, P = a.pitch;
    const int plane = static_cast<int>(a.plane);
    const int n = j * P + i;
    const unsigned m = a.mask[n];
    if (m & kMaskSolid) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) nu[q] = T(0);
        return;
    }
    const T vx = T(a.vx[n]), vy = T(a.vy[n]);
    const T k = a.kfield ? static_cast<const T *>(a.kfield)[n] : T(a.k);
    const T omega = T(a.omega);
    const T vv = T(1.5) * (vx * vx + vy * vy);
    T S = T(0), wl = T(0);
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const T ev = T(kCx[q]) * vx + T(kCy[q]) * vy;
        const T Pq = T(1) + T(3) * ev + T(4.5) * ev * ev - vv;
        S += l[q] * T(kW[q]) * (omega * Pq - k);
        wl += T(kW[q]) * l[q];
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) nu[q] = (T(1) - omega) * l[q] + S;
    if (grad_k && owner) {
        // u at the step's collision: recorded by the forward, or from the
        // next state, sum f*(t+1) = (1 - k) u
        T u;
        if (a.u_rec) {
            u = static_cast<const T *>(a.u_rec)[n];
        } else {
            T s = T(0);
#pragma unroll
            for (int q = 0; q < kQ; ++q) s += snext[q * plane + n];
            u = s / (T(1) - k);
        }
        const double term = double(u) * double(wl);
        if (stash) {
            *stash = term;
        } else {
            const size_t at = (size_t)j * N + i;
            grad_k[at] = (grad_k[at] - prior) - term;
        }
    }
    if (EDGE && (i == 0 || j == 0 || i == N - 1 || j == N - 1)) {
        unsigned unknown = 0;
#pragma unroll
        for (int q = 1; q < kQ; ++q) {
            const int si = i - kCx[q], sj = j - kCy[q];
            if (si < 0 || si >= N || sj < 0 || sj >= N) unknown |= 1u << q;
        }
        const int p = slot_of(N, i, j);
        bool active = true;
        if (a.clamp) {
            // the forward closure's R from the step's source state
            const T *__restrict__ src = static_cast<const T *>(a.src);
            double known = 0.0;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                if ((unknown >> q) & 1u) continue;
                if ((m >> q) & 1u) {
                    // bounce-back, relaxed towards w_q c_sat across a reactive link
                    const double b = double(src[kOpp[q] * plane + n]);
                    known += a.kappa_s == 0.0 ? b : (1.0 - a.kappa_s) * b + a.kappa_s * kW[q] * a.c_sat;
                } else {
                    known += double(src[q * plane + (j - kCy[q]) * P + i - kCx[q]]);
                }
            }
            active = !((1.0 - a.lam) * a.bc_a[p] + a.lam * a.bc_b[p] - known < 0.0);
        }
        double G = 0.0;
        if (active) {
            double wsum = 0.0;
#pragma unroll
            for (int q = 0; q < kQ; ++q)
                if ((unknown >> q) & 1u) {
                    G += kW[q] * double(nu[q]);
                    wsum += kW[q];
                }
            G /= wsum;
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) nu[q] = ((unknown >> q) & 1u) ? T(0) : T(double(nu[q]) - G);
        if (owner) {
            grad_a[p] += (1.0 - a.lam) * G;
            grad_b[p] += a.lam * G;
        }
    }
}

// nu at node (i, j) with the node's cotangent read from lam
template <typename T, bool EDGE = true>
__device__ __forceinline__ void adj_nu(const LbmArgs &a, int i, int j, const T *__restrict__ snext,
                                       const T *__restrict__ lam, const double *__restrict__ lam_dense, bool owner,
                                       double *__restrict__ grad_a, double *__restrict__ grad_b,
                                       double *__restrict__ grad_k, T (&nu)[kQ], double *stash = nullptr) {
    const int plane = static_cast<int>(a.plane);
    const int n = j * a.pitch + i;
    T l[kQ];
    if (a.mask[n] & kMaskSolid) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) nu[q] = T(0);
        return;
    }
    if (lam_dense) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) l[q] = T(lam_dense[dense_at(a.N, q, i, j)]);
    } else {
#pragma unroll
        for (int q = 0; q < kQ; ++q) l[q] = lam[q * plane + n];
    }
    adj_nu_of<T, EDGE>(a, i, j, snext, l, owner, grad_a, grad_b, grad_k, nu, stash);
}

// One reversed fine step.  Phase 1: nu for the tile grown by one ring (0
// outside the patch and at solid nodes), into LDS.  Phase 2, per owned
// fluid node y: dJ/df*_p(y) = nu_p(y + e_p) (zero when y + e_p is solid or
// outside: it pulled nothing from y) + (1 - kappa_s) nu_q(y), q = opp(p),
// when y bounced back along q (kappa_s: surface reaction of dissolving
// solids, 0 when off).
// inj (or null): a cotangent added to the output at fluid nodes (an
// objective that also reads the state the output belongs to).
template <typename T, int TW, int TH, int NT>
__global__ void __launch_bounds__(NT) adj_step_kernel(LbmArgs a, const T *__restrict__ snext,
                                                      const T *__restrict__ lam, T *__restrict__ out,
                                                      double *__restrict__ grad_a, double *__restrict__ grad_b,
                                                      double *__restrict__ grad_k, int tiles_x,
                                                      const T *__restrict__ inj, AdjDense dn) {
    constexpr int W1 = TW + 2, H1 = TH + 2;
    __shared__ T nus[kQ][H1][W1];
    const int N = a.N, P = a.pitch;
    const int plane = static_cast<int>(a.plane);
    const int x0 = (blockIdx.x % tiles_x) * TW, y0 = (blockIdx.x / tiles_x) * TH;
    for (int r = threadIdx.x; r < W1 * H1; r += NT) {
        const int lx = r % W1, ly = r / W1;
        const int i = x0 - 1 + lx, j = y0 - 1 + ly;
        T nu[kQ];
        if (i < 0 || j < 0 || i >= N || j >= N) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) nu[q] = T(0);
        } else {
            const bool owner = lx >= 1 && lx <= TW && ly >= 1 && ly <= TH;
            adj_nu<T>(a, i, j, snext, lam, dn.lam_dense, owner, grad_a, grad_b, grad_k, nu);
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) nus[q][ly][lx] = nu[q];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < TW * TH; r += NT) {
        const int lx = 1 + r % TW, ly = 1 + r / TW;
        const int i = x0 + lx - 1, j = y0 + ly - 1;
        if (i >= N || j >= N) continue;
        const int n = j * P + i;
        const unsigned m = a.mask[n];
        if (m & kMaskSolid) {
            if (dn.out_dense) {
                if (!dn.accumulate)
#pragma unroll
                    for (int q = 0; q < kQ; ++q) dn.out_dense[dense_at(N, q, i, j)] = 0.0;
            } else {
#pragma unroll
                for (int q = 0; q < kQ; ++q) out[q * plane + n] = T(0);
            }
            continue;
        }
        // a reactive link returns 1 - kappa_s of the population (1 when off)
        const T keep = T(1.0 - a.kappa_s);
#pragma unroll
        for (int p = 0; p < kQ; ++p) {
            T acc = nus[p][ly + kCy[p]][lx + kCx[p]];
            const int q = kOpp[p];
            if ((m >> q) & 1u) acc += keep * nus[q][ly][lx];
            if (inj) acc += inj[p * plane + n];
            if (dn.out_dense) {
                const size_t d = dense_at(N, p, i, j);
                dn.out_dense[d] = dn.accumulate ? dn.out_dense[d] + double(acc) : double(acc);
            } else {
                out[p * plane + n] = acc;
            }
        }
    }
}

// Two reversed fine steps in one launch: step t (a1: its source state and
// interface weight; snext1 = f*(t+1)) and then step t-1 (a2; snext2 =
// f*(t)), from lam = dJ/df*(t+1) to out = dJ/df*(t-1).  Phase 1: nu of step
// t for the tile grown by two rings, into LDS.  Phase 2: dJ/df*(t) gathered
// for the tile grown by one ring (as one reversed step's output), and from
// it nu of step t-1, held in registers across a barrier and written back in
// place.  Phase 3: the owned nodes gather their outputs.  Every node takes
// the single reversed step's operations (dJ/df*(t) never leaves the chip),
// so the result equals two adj_step_kernel launches; gradients are added by
// the owner of each node, step t before step t-1 (in FP64 the dJ/dk terms
// of both steps in one update, (g - term_t) - term_t-1, as two updates
// would leave it).  inj_mid, inj_out (or null): cotangents added at fluid
// nodes to dJ/df*(t) (on chip) and to the output dJ/df*(t-1).
template <typename T, int TW, int TH, int NT>
__global__ void __launch_bounds__(NT) adj_step2_kernel(LbmArgs a1, LbmArgs a2, const T *__restrict__ snext1,
                                                       const T *__restrict__ snext2, const T *__restrict__ lam,
                                                       T *__restrict__ out, double *__restrict__ grad_a,
                                                       double *__restrict__ grad_b, double *__restrict__ grad_k,
                                                       int tiles_x, const T *__restrict__ inj_mid,
                                                       const T *__restrict__ inj_out, AdjDense dn) {
    constexpr int W2 = TW + 4, H2 = TH + 4, W1 = TW + 2, H1 = TH + 2;
    constexpr int R1 = (W1 * H1 + NT - 1) / NT;
    // FP64: the owned nodes' dJ/dk terms of step t wait in LDS and step
    // t-1 adds both (one read-modify-write of grad_k per pair)
    constexpr bool STASH = sizeof(T) == 8;
    __shared__ T nus[kQ][H2][W2];
    __shared__ double kst[STASH ? TH : 1][STASH ? TW : 1];
    const int N = a1.N, P = a1.pitch;
    const int plane = static_cast<int>(a1.plane);
    const int x0 = (blockIdx.x % tiles_x) * TW, y0 = (blockIdx.x / tiles_x) * TH;
    // Two compiled copies: a tile whose two-ring region reaches the patch
    // perimeter (or its end) takes the bounds tests and the closure's
    // transpose; every other tile (most of them) a copy without them.
    const bool edge = x0 - 2 <= 0 || y0 - 2 <= 0 || x0 + TW + 1 >= N - 1 || y0 + TH + 1 >= N - 1;
    auto phases = [&](auto edge_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
        // ---- phase 1: nu of step t, two rings ---------------------------------
        for (int r = threadIdx.x; r < W2 * H2; r += NT) {
            const int lx = r % W2, ly = r / W2;
            const int i = x0 - 2 + lx, j = y0 - 2 + ly;
            T nu[kQ];
            if (EDGE && (i < 0 || j < 0 || i >= N || j >= N)) {
#pragma unroll
                for (int q = 0; q < kQ; ++q) nu[q] = T(0);
            } else {
                const bool owner = lx >= 2 && lx <= TW + 1 && ly >= 2 && ly <= TH + 1;
                adj_nu<T, EDGE>(a1, i, j, snext1, lam, dn.lam_dense, owner, grad_a, grad_b, grad_k, nu,
                          STASH && owner ? &kst[STASH ? ly - 2 : 0][STASH ? lx - 2 : 0] : nullptr);
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) nus[q][ly][lx] = nu[q];
        }
        __syncthreads();
        // ---- phase 2: dJ/df*(t) on one ring, then nu of step t-1 --------------
        const T keep = T(1.0 - a1.kappa_s);
        T h[R1][kQ];
#pragma unroll
        for (int k = 0; k < R1; ++k) {
            const int r = threadIdx.x + NT * k;
            const int lx = 1 + r % W1, ly = 1 + r / W1;      // ring-2 coordinates of the one-ring node
            const int i = x0 - 2 + lx, j = y0 - 2 + ly;
#pragma unroll
            for (int q = 0; q < kQ; ++q) h[k][q] = T(0);
            if (r >= W1 * H1 || (EDGE && (i < 0 || j < 0 || i >= N || j >= N))) continue;
            const int n = j * P + i;
            const unsigned m = a1.mask[n];
            if (m & kMaskSolid) continue;
            T l[kQ];
#pragma unroll
            for (int p = 0; p < kQ; ++p) {
                T acc = nus[p][ly + kCy[p]][lx + kCx[p]];
                const int q = kOpp[p];
                if ((m >> q) & 1u) acc += keep * nus[q][ly][lx];
                if (inj_mid) acc += inj_mid[p * plane + n];
                l[p] = acc;
            }
            const bool owner = lx >= 2 && lx <= TW + 1 && ly >= 2 && ly <= TH + 1;
            adj_nu_of<T, EDGE>(a2, i, j, snext2, l, owner, grad_a, grad_b, grad_k, h[k], nullptr,
                         STASH && owner ? kst[STASH ? ly - 2 : 0][STASH ? lx - 2 : 0] : 0.0);
        }
        __syncthreads();             // every read of step t's nu is done
#pragma unroll
        for (int k = 0; k < R1; ++k) {
            const int r = threadIdx.x + NT * k;
            if (r >= W1 * H1) continue;
            const int lx = 1 + r % W1, ly = 1 + r / W1;
#pragma unroll
            for (int q = 0; q < kQ; ++q) nus[q][ly][lx] = h[k][q];
        }
        __syncthreads();
        // ---- phase 3: the owned nodes' dJ/df*(t-1) -----------------------------
        const T keep2 = T(1.0 - a2.kappa_s);
        for (int r = threadIdx.x; r < TW * TH; r += NT) {
            const int lx = 2 + r % TW, ly = 2 + r / TW;
            const int i = x0 + lx - 2, j = y0 + ly - 2;
            if (EDGE && (i >= N || j >= N)) continue;
            const int n = j * P + i;
            const unsigned m = a2.mask[n];
            if (m & kMaskSolid) {
                if (dn.out_dense) {
                    if (!dn.accumulate)
#pragma unroll
                        for (int q = 0; q < kQ; ++q) dn.out_dense[dense_at(N, q, i, j)] = 0.0;
                } else {
#pragma unroll
                    for (int q = 0; q < kQ; ++q) out[q * plane + n] = T(0);
                }
                continue;
            }
#pragma unroll
            for (int p = 0; p < kQ; ++p) {
                T acc = nus[p][ly + kCy[p]][lx + kCx[p]];
                const int q = kOpp[p];
                if ((m >> q) & 1u) acc += keep2 * nus[q][ly][lx];
                if (inj_out) acc += inj_out[p * plane + n];
                if (dn.out_dense) {
                    const size_t d = dense_at(N, p, i, j);
                    dn.out_dense[d] = dn.accumulate ? dn.out_dense[d] + double(acc) : double(acc);
                } else {
                    out[p * plane + n] = acc;
                }
            }
        }
    };
    if (edge) phases(std::true_type{});
    else phases(std::false_type{});
}

// dense FP64 [9][N][N] <-> pitched planes of T
template <typename T>
__global__ void __launch_bounds__(256) adj_pack_kernel(LbmArgs a, const double *__restrict__ dense, T *__restrict__ pitched,
                                                      int row_blocks) {
    const int N = a.N, P = a.pitch;
    const int plane = static_cast<int>(a.plane);
    const int j = blockIdx.x / row_blocks;
    const int i = (blockIdx.x % row_blocks) * blockDim.x + threadIdx.x;
    if (i >= N) return;
#pragma unroll
    for (int q = 0; q < kQ; ++q) pitched[q * plane + j * P + i] = T(dense[((size_t)q * N + j) * N + i]);
}

template <typename T>
__global__ void __launch_bounds__(256) adj_unpack_kernel(LbmArgs a, const T *__restrict__ pitched, double *__restrict__ dense,
                                                        int row_blocks, int accumulate) {
    const int N = a.N, P = a.pitch;
    const int plane = static_cast<int>(a.plane);
    const int j = blockIdx.x / row_blocks;
    const int i = (blockIdx.x % row_blocks) * blockDim.x + threadIdx.x;
    if (i >= N) return;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const size_t d = ((size_t)q * N + j) * N + i;
        const double v = double(pitched[q * plane + j * P + i]);
        dense[d] = accumulate ? dense[d] + v : v;
    }
}

// Lanes per workgroup: 512 in FP64, whose LDS tile (two rings of nu, 58.8 KB
// for the paired kernel) allows two workgroups per CU -- 16 waves rather than
// the 8 of 256-lane groups; 256 in FP32 (29.4 KB, five groups per CU).
template <typename T>
constexpr int adj_lanes() { return sizeof(T) == 8 ? 512 : 256; }

template <typename T>
hipError_t adjoint_step_impl(const LbmArgs &a, const void *snext, const void *lam, void *out, double *grad_a,
                             double *grad_b, double *grad_k, const void *inj, AdjDense dn, hipStream_t s) {
    constexpr int TW = 64, TH = 8, NT = adj_lanes<T>();
    const int tiles_x = (a.N + TW - 1) / TW, tiles_y = (a.N + TH - 1) / TH;
    hipLaunchKernelGGL((adj_step_kernel<T, TW, TH, NT>), dim3(tiles_x * tiles_y), dim3(NT), 0, s, a,
                       static_cast<const T *>(snext), static_cast<const T *>(lam), static_cast<T *>(out), grad_a,
                       grad_b, grad_k, tiles_x, static_cast<const T *>(inj), dn);
    return hipGetLastError();
}

template <typename T>
hipError_t adjoint_step2_impl(const LbmArgs &a1, const LbmArgs &a2, const void *snext1, const void *snext2,
                              const void *lam, void *out, double *grad_a, double *grad_b, double *grad_k,
                              const void *inj_mid, const void *inj_out, AdjDense dn, hipStream_t s) {
    constexpr int TW = 64, TH = 8, NT = adj_lanes<T>();
    const int tiles_x = (a1.N + TW - 1) / TW, tiles_y = (a1.N + TH - 1) / TH;
    hipLaunchKernelGGL((adj_step2_kernel<T, TW, TH, NT>), dim3(tiles_x * tiles_y), dim3(NT), 0, s, a1, a2,
                       static_cast<const T *>(snext1), static_cast<const T *>(snext2), static_cast<const T *>(lam),
                       static_cast<T *>(out), grad_a, grad_b, grad_k, tiles_x, static_cast<const T *>(inj_mid),
                       static_cast<const T *>(inj_out), dn);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_step2(const LbmArgs &a1, const LbmArgs &a2, int prec, const void *snext1,
                                const void *snext2, const void *lam, void *out, double *grad_a, double *grad_b,
                                double *grad_k, hipStream_t s, const void *inj_mid, const void *inj_out,
                                const double *lam_dense, double *out_dense, bool accumulate) {
    const AdjDense dn{lam_dense, out_dense, accumulate ? 1 : 0};
    if (prec == HYB_FP64)
        return adjoint_step2_impl<double>(a1, a2, snext1, snext2, lam, out, grad_a, grad_b, grad_k, inj_mid, inj_out,
                                          dn, s);
    return adjoint_step2_impl<float>(a1, a2, snext1, snext2, lam, out, grad_a, grad_b, grad_k, inj_mid, inj_out, dn,
                                     s);
}

hipError_t launch_adjoint_step(const LbmArgs &a, int prec, const void *snext, const void *lam, void *nu, void *out,
                               double *grad_a, double *grad_b, double *grad_k, hipStream_t s, const void *inj,
                               const double *lam_dense, double *out_dense, bool accumulate) {
    (void)nu;    // scratch of the two-kernel form; the fused kernel keeps nu in LDS
    const AdjDense dn{lam_dense, out_dense, accumulate ? 1 : 0};
    if (prec == HYB_FP64) return adjoint_step_impl<double>(a, snext, lam, out, grad_a, grad_b, grad_k, inj, dn, s);
    return adjoint_step_impl<float>(a, snext, lam, out, grad_a, grad_b, grad_k, inj, dn, s);
}

hipError_t launch_adjoint_pack(const LbmArgs &a, int prec, const double *dense, void *pitched, bool to_pitched,
                               hipStream_t s, bool accumulate) {
    const int rb = (a.N + 255) / 256;
    const dim3 grid(a.N * rb), block(256);
    if (to_pitched) {
        if (prec == HYB_FP64)
            hipLaunchKernelGGL(adj_pack_kernel<double>, grid, block, 0, s, a, dense, static_cast<double *>(pitched), rb);
        else
            hipLaunchKernelGGL(adj_pack_kernel<float>, grid, block, 0, s, a, dense, static_cast<float *>(pitched), rb);
    } else {
        if (prec == HYB_FP64)
            hipLaunchKernelGGL(adj_unpack_kernel<double>, grid, block, 0, s, a, static_cast<const double *>(pitched),
                               const_cast<double *>(dense), rb, accumulate ? 1 : 0);
        else
            hipLaunchKernelGGL(adj_unpack_kernel<float>, grid, block, 0, s, a, static_cast<const float *>(pitched),
                               const_cast<double *>(dense), rb, accumulate ? 1 : 0);
    }
    return hipGetLastError();
}

}  // namespace hyb
