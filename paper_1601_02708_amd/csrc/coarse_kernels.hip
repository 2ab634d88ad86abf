// Coarse-scale kernels: the trapezoidal FEM step (Sec. 6.1, eq.
// FEM_discrete with theta = 1/2) solved by right-preconditioned BiCGSTAB in
// FP64, and the two grid transfers of Sec. 6.2, item ii.
//
// The coarse system is tiny (at most a few 10^4 unknowns) and needs a few
// dozen dependent passes per solve, so it is latency-bound.  The two
// kernels that apply A P give each mesh row eight lanes (one stencil row
// each) to put eight times more waves in flight; the others use one lane
// per row.  Stencil products read zero-halo padded vectors; dot
// products are reduced deterministically (each workgroup writes a partial,
// the next kernel sums all partials in block order); the preconditioner P
// (a sparse approximate inverse computed on the host) is folded into the
// operator A P.  One BiCGSTAB iteration is two kernels with one reduction
// each; device-side flags turn the launches after convergence into no-ops.
#include "hyb_impl.h"

namespace hyb {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int padded_index(const CoarseDev &c, int node) {
    const int m1 = c.M + 1;
    const int k = node % m1, l = node / m1;
    return (l + kCoarseHalo) * c.S + (k + kCoarseHalo);
}

// Stencil product of row `node` (width W, radius W/2) with padded vector x;
// coefficients are offset-major (coef[o * n + node]).
template <int W>
__device__ __forceinline__ double stencil_row(const double *__restrict__ coef, int n, int node, int pidx, int S,
                                              const double *__restrict__ x) {
    constexpr int R = W / 2;
    double acc = 0.0;
#pragma unroll
    for (int dl = -R; dl <= R; ++dl) {
#pragma unroll
        for (int dk = -R; dk <= R; ++dk)
            acc += coef[(size_t)((dl + R) * W + (dk + R)) * n + node] * x[pidx + dl * S + dk];
    }
    return acc;
}

// A P times padded vector x at row `node`, computed by the eight lanes of
// a group: lane g < 7 takes stencil row dl = g - 3 (seven contiguous
// coefficients, seven contiguous vector entries), lane 7 adds zero; the
// xor butterfly leaves the same (bit-identical) total in all eight lanes.
__device__ __forceinline__ double ap_row8(const CoarseDev &c, int node, int pidx, int g, bool valid,
                                          const double *__restrict__ x) {
    constexpr int W = kApW, R = W / 2;
    double acc = 0.0;
    if (valid && g < W) {
        const double *__restrict__ cr = c.AP + (size_t)node * (W * W) + g * W;
        const double *__restrict__ xr = x + pidx + (g - R) * c.S - R;
#pragma unroll
        for (int dk = 0; dk < W; ++dk) acc += cr[dk] * xr[dk];
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    return acc;
}

// The same product for the vector s - omega t, formed entry by entry from
// two complete vectors (the entries equal what the row owners compute).
__device__ __forceinline__ double ap_row8_diff(const CoarseDev &c, int node, int pidx, int g, bool valid,
                                               const double *__restrict__ s, const double *__restrict__ t,
                                               double omega) {
    constexpr int W = kApW, R = W / 2;
    double acc = 0.0;
    if (valid && g < W) {
        const double *__restrict__ cr = c.AP + (size_t)node * (W * W) + g * W;
        const size_t o = pidx + (g - R) * c.S - R;
#pragma unroll
        for (int dk = 0; dk < W; ++dk) acc += cr[dk] * (s[o + dk] - omega * t[o + dk]);
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    return acc;
}

// Dense part of the shadow residual: the MurmurHash3 32-bit finaliser of
// the node index, mapped to [-1, 1).
__device__ __forceinline__ double shadow_hash(int node) {
    unsigned x = static_cast<unsigned>(node) * 0x9E3779B9u + 0x7F4A7C15u;
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return double(x) * (2.0 / 4294967296.0) - 1.0;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
    // wave reduction then across the waves of the block
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        v[k] = x;
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[wave * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / 64;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += lds[w * NV + k];
            v[k] = s;
        }
    }
}

// Reduction partials: every kernel of the solve writes one partial per block
// into its own slot; the next kernel sums all blocks in block order, so the
// scalars are bit-identical in every block (deterministic).
__device__ __forceinline__ double *slot_ptr(const CoarseDev &c, int slot) {
    return c.partials + (size_t)slot * kPartialValues * c.pstride;
}
template <int NV>
__device__ __forceinline__ void write_partials(const CoarseDev &c, int slot, double (&v)[NV], double *lds) {
    block_sum<NV>(v, lds);
    if (threadIdx.x == 0) {
        double *s = slot_ptr(c, slot);
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k * c.pstride + blockIdx.x] = v[k];
    }
}
// Sums of the `blocks` per-block partials of an earlier kernel, computed by
// the first wave of the block (lanes stride over the blocks, then a fixed
// shuffle tree), so every block obtains bit-identical values; broadcast via
// LDS.
template <int NV>
__device__ __forceinline__ void read_sums(const CoarseDev &c, int slot, int blocks, double (&out)[NV],
                                          double *lds) {
    if (threadIdx.x < 64) {
        const double *s = slot_ptr(c, slot);
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            // batches of 16 independent loads per lane (one memory round
            // trip per 1024 partials), summed in a fixed order
            double acc = 0.0;
            for (int base = 0; base < blocks; base += 1024) {
                double part[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int b = base + threadIdx.x + 64 * u;
                    part[u] = b < blocks ? s[(size_t)k * c.pstride + b] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) acc += part[u];
            }
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
            if (threadIdx.x == 0) lds[16 + k] = acc;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = lds[16 + k];
    __syncthreads();
}

enum Slot { kSlotRhs = 0, kSlotA = 1, kSlotB = 2 };

// b = B d(t_n) on free rows, a_ii times the prescribed value on Dirichlet
// rows; r0 = b - A x0 (x0 = initial guess).  Initialises the Krylov
// vectors and the solver state for the kernels that follow; partials
// b.b, r0.r0 and h.r0 (h = shadow_hash).
__global__ void __launch_bounds__(kBlock) coarse_rhs_kernel(CoarseDev c, const double *__restrict__ guess) {
    __shared__ double lds[32];
    double red[3] = {0.0, 0.0, 0.0};
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node < c.n) {
        const int pidx = padded_index(c, node);
        const int kind = c.dkind[node];
        double b;
        if (kind == -1) b = stencil_row<3>(c.B9, c.n, node, pidx, c.S, c.xn);
        else b = c.A9[(size_t)4 * c.n + node] * (kind == -2 ? c.outer_value : c.ufc[kind]);
        const double r0 = b - stencil_row<3>(c.A9, c.n, node, pidx, c.S, guess);
        c.r[pidx] = r0;
        c.p[pidx] = 0.0;
        c.v[pidx] = 0.0;
        c.z[pidx] = 0.0;
        c.y[pidx] = 0.0;
        red[0] = b * b;
        red[1] = r0 * r0;
        red[2] = shadow_hash(node) * r0;
    }
    write_partials<3>(c, kSlotRhs, red, lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        KrylovState &st = *c.state;
        st.rho = 1.0;
        st.alpha = 1.0;
        st.iters = 0;
        st.done = 0;
        st.brk = 0;
        st.skip = 0;
    }
}

// r0 = rhs (a given padded vector, first guess 0): the rhs kernel of a
// solve of (c.AP) y = rhs, with the same partials and state as
// coarse_rhs_kernel.
__global__ void __launch_bounds__(kBlock) coarse_rhs_given_kernel(CoarseDev c, const double *__restrict__ rhs) {
    __shared__ double lds[32];
    double red[3] = {0.0, 0.0, 0.0};
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node < c.n) {
        const int pidx = padded_index(c, node);
        const double r0 = rhs[pidx];
        c.r[pidx] = r0;
        c.p[pidx] = 0.0;
        c.v[pidx] = 0.0;
        c.z[pidx] = 0.0;
        c.y[pidx] = 0.0;
        red[0] = r0 * r0;
        red[1] = r0 * r0;
        red[2] = shadow_hash(node) * r0;
    }
    write_partials<3>(c, kSlotRhs, red, lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        KrylovState &st = *c.state;
        st.rho = 1.0;
        st.alpha = 1.0;
        st.iters = 0;
        st.done = 0;
        st.brk = 0;
        st.skip = 0;
    }
}

// Right-preconditioned BiCGSTAB on (A P) y = r0, x = x0 + P y, two kernels
// per iteration; every cross-block dependency is a kernel boundary (the
// device-scope cache maintenance happens once per launch instead of once per
// block and barrier).  Iteration k:
//
//   A(k): finish iteration k-1 -- omega = t.s / t.t, y += alpha p + omega s,
//         r = s - omega t -- with rho_k = rh.r = rh.s - omega rh.t from
//         B(k-1)'s sums; beta = (rho_k / rho_{k-1}) (alpha / omega);
//         w = A P r (from the neighbours' s - omega t); p = r + beta (p -
//         omega v); v' = A P p = w + beta (v - omega z); partials rh.v', r.r.
//   B(k): stop if ||r_k|| <= tol ||b|| (the explicit r.r of A(k)), at a
//         breakdown, or at k = max_iter; else alpha = rho_k / rh.v';
//         s = r - alpha v'; z = A P v'; t = A P s = w - alpha z; partials
//         t.s, t.t, rh.s, rh.t.
//
// A(0) starts from r0 and sets the shadow residual rh = r0 + gamma h, with
// h = shadow_hash and gamma = ||r0|| / sqrt(n) (rho_0 = r0.r0 + gamma h.r0).
// The dense part matters: a warm start leaves r0 on the Dirichlet rows,
// which A P maps almost onto themselves, and with rh = r0 the later rh.r
// would be rounding noise (a near breakdown that the folded rho = rh.s -
// omega rh.t cannot survive).  The state block is read by every block of a
// kernel and written (by block 0) only under names that kernel does not
// read: A writes rho_next, brk, skip and (A(0)) bb = b.b; B writes rho,
// alpha and done.
__global__ void __launch_bounds__(kBlock) coarse_iter_a(CoarseDev c, int k) {
    __shared__ double lds[32];
    KrylovState &st = *c.state;
    if (st.done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st.skip = 1;
        return;
    }
    const bool first = k == 0;
    double rho, omega = 0.0, gamma = 0.0, bb = 0.0;
    if (first) {
        double rs[3];
        read_sums<3>(c, kSlotRhs, c.grid, rs, lds);
        bb = rs[0];
        gamma = sqrt(rs[1] / c.n);
        rho = rs[1] + gamma * rs[2];
    } else {
        double bs[4];
        read_sums<4>(c, kSlotB, c.grid8, bs, lds);
        omega = bs[1] > 0.0 ? bs[0] / bs[1] : 0.0;
        rho = bs[2] - omega * bs[3];
    }
    const bool breakdown = !first && (omega == 0.0 || rho == 0.0);
    const double alpha = st.alpha;
    const double beta = (first || breakdown) ? 0.0 : (rho / st.rho) * (alpha / omega);
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int node = gt >> 3, g = gt & 7;
    const bool valid = node < c.n;
    const int pi = valid ? padded_index(c, node) : 0;
    // r_k at this row; lane 0 of the row's eight also folds iteration k-1
    double r = 0.0;
    if (valid) {
        if (first) {
            r = c.r[pi];
        } else {
            const double sv = c.s[pi];
            r = sv - omega * c.t[pi];
            if (g == 0) {
                c.y[pi] += alpha * c.p[pi] + omega * sv;
                c.r[pi] = r;
            }
        }
    }
    const double w = first ? ap_row8(c, node, pi, g, valid, c.r) : ap_row8_diff(c, node, pi, g, valid, c.s, c.t, omega);
    double red[2] = {0.0, 0.0};
    if (valid && g == 0) {
        double rh;
        if (first) {
            rh = r + gamma * shadow_hash(node);
            c.rh[pi] = rh;
        } else {
            rh = c.rh[pi];
        }
        c.p[pi] = r + beta * (c.p[pi] - omega * c.v[pi]);
        const double vn = w + beta * (c.v[pi] - omega * c.z[pi]);
        c.w[pi] = w;
        c.v[pi] = vn;
        red[0] = rh * vn;
        red[1] = r * r;
    }
    write_partials<2>(c, kSlotA, red, lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.rho_next = rho;
        st.brk = breakdown ? 1 : 0;
        st.skip = 0;
        if (first) st.bb = bb;
    }
}

__global__ void __launch_bounds__(kBlock) coarse_iter_b(CoarseDev c, int k, double tol, int max_iter) {
    __shared__ double lds[32];
    KrylovState &st = *c.state;
    if (st.skip) return;
    double as[2];
    read_sums<2>(c, kSlotA, c.grid8, as, lds);
    const double bnorm = sqrt(st.bb);
    const double rnorm = sqrt(as[1]);
    const bool converged = rnorm <= tol * (bnorm > 0.0 ? bnorm : 1.0);
    if (converged || st.brk || k >= max_iter || !(rnorm == rnorm)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st.done = 1;
            st.converged = converged ? 1 : 0;
            st.rnorm = rnorm;
            st.bnorm = bnorm;
            st.iters = k;
        }
        return;
    }
    const double rho = st.rho_next;
    const double alpha = rho / as[0];
    double red[4] = {0.0, 0.0, 0.0, 0.0};
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int node = gt >> 3, g = gt & 7;
    const bool valid = node < c.n;
    const int pi = valid ? padded_index(c, node) : 0;
    const double zn = ap_row8(c, node, pi, g, valid, c.v);
    if (valid && g == 0) {
        const double sv = c.r[pi] - alpha * c.v[pi];
        const double tv = c.w[pi] - alpha * zn;
        const double rh = c.rh[pi];
        c.s[pi] = sv;
        c.z[pi] = zn;
        c.t[pi] = tv;
        red[0] = tv * sv;
        red[1] = tv * tv;
        red[2] = rh * sv;
        red[3] = rh * tv;
    }
    write_partials<4>(c, kSlotB, red, lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.rho = rho;
        st.alpha = alpha;
    }
}

// x = x0 + P y; records iterations, convergence and ||r|| / ||b|| (the
// state was closed by the final convergence test).
__global__ void __launch_bounds__(kBlock) coarse_finish(CoarseDev c, const double *__restrict__ guess) {
    const KrylovState &st = *c.state;
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node < c.n) {
        const int pi = padded_index(c, node);
        c.x1[pi] = guess[pi] + stencil_row<kSpaiW>(c.P, c.n, node, pi, c.S, c.y);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c.result->iters = st.iters;
        c.result->converged = st.converged;
        c.result->relres = st.bnorm > 0.0 ? st.rnorm / st.bnorm : st.rnorm;
    }
}

// out = y (the solution of a solve from y = 0 without a right
// preconditioner); records iterations, convergence and ||r|| / ||b||.
__global__ void __launch_bounds__(kBlock) coarse_take_kernel(CoarseDev c, double *__restrict__ out) {
    const KrylovState &st = *c.state;
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node < c.n) {
        const int pi = padded_index(c, node);
        out[pi] = c.y[pi];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c.result->iters = st.iters;
        c.result->converged = st.converged;
        c.result->relres = st.bnorm > 0.0 ? st.rnorm / st.bnorm : st.rnorm;
    }
}

// First guess of a coarse step's first solve: the linear extrapolation
// 2 d(t_n) - d(t_{n-1}) in time, written to x1.
__global__ void coarse_extrapolate_kernel(CoarseDev c, int len) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len) c.x1[k] = 2.0 * c.xn[k] - c.xprev[k];
}

// a[p] = interpolant of xa, b[p] = interpolant of xb at perimeter slot p.
__global__ void c2f_kernel(const int *__restrict__ idx, const double *__restrict__ w, int nslots,
                           const double *__restrict__ xa, const double *__restrict__ xb, double *__restrict__ a,
                           double *__restrict__ b) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nslots) return;
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int k = idx[4 * p + c];
        const double wc = w[4 * p + c];
        sa += wc * xa[k];
        sb += wc * xb[k];
    }
    a[p] = sa;
    b[p] = sb;
}

// ufc[c] = sum of the four weighted lattice concentrations around Gamma_{f->c}
// node c.  Every index is a valid lattice node (dropped corners carry weight
// 0), so all 36 population loads are issued at once; zero weights are
// selected out rather than multiplied, so no value stored at a solid node can
// reach the sum.
template <typename S>
__global__ void f2c_kernel(LbmArgs lat, const int *__restrict__ idx, const double *__restrict__ w, int nfc,
                           double *__restrict__ ufc) {
    typedef typename Pop<S>::T T;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nfc) return;
    const S *__restrict__ src = static_cast<const S *>(lat.src);
    const int plane = static_cast<int>(lat.plane);
    int n[4];
    double wm[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        n[m] = idx[4 * c + m];
        wm[m] = w[4 * c + m];
    }
    S raw[4][kQ];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < kQ; ++q) raw[m][q] = src[q * plane + n[m]];
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double u = 0.0;
#pragma unroll
        for (int q = 0; q < kQ; ++q) u += double(Pop<S>::ld(raw[m][q], q, lat));
        const double k = lat.kfield ? double(static_cast<const T *>(lat.kfield)[n[m]]) : lat.k;
        acc += wm[m] != 0.0 ? wm[m] * (u / (1.0 - k)) : 0.0;
    }
    ufc[c] = acc;
}

}  // namespace

hipError_t launch_coarse_rhs(const CoarseDev &c, const double *guess, hipStream_t s) {
    hipLaunchKernelGGL(coarse_rhs_kernel, dim3(c.grid), dim3(kBlock), 0, s, c, guess);
    return hipGetLastError();
}

hipError_t launch_coarse_solve(const CoarseDev &c, const double *guess, int iterations, int max_iter, double tol,
                               hipStream_t s) {
    for (int k = 0; k < iterations; ++k) {
        hipLaunchKernelGGL(coarse_iter_a, dim3(c.grid8), dim3(kBlock), 0, s, c, k);
        hipLaunchKernelGGL(coarse_iter_b, dim3(c.grid8), dim3(kBlock), 0, s, c, k, tol, max_iter);
    }
    // closing pair: finishes the last enqueued iteration and tests it
    hipLaunchKernelGGL(coarse_iter_a, dim3(c.grid8), dim3(kBlock), 0, s, c, iterations);
    hipLaunchKernelGGL(coarse_iter_b, dim3(c.grid8), dim3(kBlock), 0, s, c, iterations, tol, 0);
    hipLaunchKernelGGL(coarse_finish, dim3(c.grid), dim3(kBlock), 0, s, c, guess);
    return hipGetLastError();
}

hipError_t launch_coarse_solve_given(const CoarseDev &c, const double *rhs, double *out, int iterations, int max_iter,
                                     double tol, hipStream_t s) {
    hipLaunchKernelGGL(coarse_rhs_given_kernel, dim3(c.grid), dim3(kBlock), 0, s, c, rhs);
    for (int k = 0; k < iterations; ++k) {
        hipLaunchKernelGGL(coarse_iter_a, dim3(c.grid8), dim3(kBlock), 0, s, c, k);
        hipLaunchKernelGGL(coarse_iter_b, dim3(c.grid8), dim3(kBlock), 0, s, c, k, tol, max_iter);
    }
    hipLaunchKernelGGL(coarse_iter_a, dim3(c.grid8), dim3(kBlock), 0, s, c, iterations);
    hipLaunchKernelGGL(coarse_iter_b, dim3(c.grid8), dim3(kBlock), 0, s, c, iterations, tol, 0);
    hipLaunchKernelGGL(coarse_take_kernel, dim3(c.grid), dim3(kBlock), 0, s, c, out);
    return hipGetLastError();
}

hipError_t launch_coarse_extrapolate(const CoarseDev &c, hipStream_t s) {
    const int len = c.S * c.S;
    hipLaunchKernelGGL(coarse_extrapolate_kernel, dim3((len + 255) / 256), dim3(256), 0, s, c, len);
    return hipGetLastError();
}

hipError_t launch_c2f(const int *idx, const double *w, int nslots, const double *xa, const double *xb, double *a,
                      double *b, hipStream_t s) {
    hipLaunchKernelGGL(c2f_kernel, dim3((nslots + 255) / 256), dim3(256), 0, s, idx, w, nslots, xa, xb, a, b);
    return hipGetLastError();
}

hipError_t launch_f2c(const LbmArgs &lat, const int *idx, const double *w, int nfc, double *ufc, int prec,
                      hipStream_t s) {
    if (nfc == 0) return hipSuccess;
    // one wave per block: the few thousand coarse nodes spread over as many
    // CUs as possible (every lane's 36 loads touch different cache lines)
    const dim3 grid((nfc + 63) / 64), block(64);
    if (prec == HYB_FP64) hipLaunchKernelGGL(f2c_kernel<double>, grid, block, 0, s, lat, idx, w, nfc, ufc);
    else if (prec == HYB_FP32) hipLaunchKernelGGL(f2c_kernel<float>, grid, block, 0, s, lat, idx, w, nfc, ufc);
    else hipLaunchKernelGGL(f2c_kernel<_Float16>, grid, block, 0, s, lat, idx, w, nfc, ufc);
    return hipGetLastError();
}

}  // namespace hyb
