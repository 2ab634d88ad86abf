// Coarse-scale kernels: the trapezoidal FEM step (Sec. 6.1, eq.
// FEM_discrete with theta = 1/2) solved by right-preconditioned BiCGSTAB in
// FP64, and the two grid transfers of Sec. 6.2, item ii.
//
// The coarse system is tiny (at most a few 10^4 unknowns) and needs a few
// dozen dependent passes per solve, so it is latency-bound.  The whole
// solve is one persistent cooperative kernel: every workgroup owns a
// contiguous range of mesh nodes, stencil products read the padded vectors
// directly, dot products are reduced deterministically (each workgroup
// writes a partial, every workgroup sums all partials in the same order
// after a grid barrier), and the preconditioner P (a sparse approximate
// inverse computed on the host) is folded into the operator A P so one
// iteration needs two stencil products and five grid barriers.
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

// Grid-wide barrier for a cooperative launch.  Each block publishes the
// round it has reached in its own flag word (no contended atomics); the
// first wave of every block then polls all flags until each has reached
// the round.  One thread per block fences to device scope on either side
// (release of the block's writes, acquire of the others'), bracketed by
// workgroup barriers.  The wait is bounded: a timeout is recorded and the
// caller abandons the solve.
__device__ bool grid_barrier(const CoarseDev &c, unsigned &round) {
    __syncthreads();
    if (gridDim.x == 1) return true;
    round += 1;
    __shared__ int failed;
    if (threadIdx.x < 64) {
        if (threadIdx.x == 0) {
            __threadfence();
            __hip_atomic_store(&c.flags[blockIdx.x], round, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        unsigned spins = 0;
        int st = 0;
        for (;;) {
            int reached = 1;
            for (int b = threadIdx.x; b < (int)gridDim.x; b += 64)
                reached &= __hip_atomic_load(&c.flags[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= round;
            if (__all(reached)) break;
            if (++spins > (1u << 26) ||
                __hip_atomic_load(&c.result->barrier_timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                st = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (threadIdx.x == 0) {
            __threadfence();
            if (st) atomicOr(&c.result->barrier_timeout, 1u);
            failed = st;
        }
    }
    __syncthreads();
    return failed == 0;
}

// Reduce NV per-thread values over the grid; the result is returned to
// every thread.  Partials are double-buffered by `parity` so a fast block
// cannot overwrite values a slow block is still summing.
template <int NV>
__device__ bool grid_sum(const CoarseDev &c, double (&v)[NV], unsigned &round, int &parity, double *lds) {
    block_sum<NV>(v, lds);
    double *slot = c.partials + (size_t)parity * gridDim.x * 4;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) slot[blockIdx.x * 4 + k] = v[k];
    }
    if (!grid_barrier(c, round)) return false;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int b = 0; b < (int)gridDim.x; ++b) s += slot[b * 4 + k];
        v[k] = s;
    }
    parity ^= 1;
    return true;
}

// b = B d(t_n) on free rows, a_ii times the prescribed value on Dirichlet rows;
// r0 = b - A x0 (x0 = initial guess); also writes ||b||^2 partials and
// resets the barrier flags and result block for the solve that follows.
__global__ void __launch_bounds__(kBlock) coarse_rhs_kernel(CoarseDev c, const double *__restrict__ guess) {
    __shared__ double lds[16];
    if (blockIdx.x == 0) {
        for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) c.flags[b] = 0u;
        if (threadIdx.x == 0) c.result->barrier_timeout = 0u;
    }
    double bb[1] = {0.0};
    for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < c.n; node += gridDim.x * blockDim.x) {
        const int pidx = padded_index(c, node);
        const int kind = c.dkind[node];
        double b;
        if (kind == -1) b = stencil_row<3>(c.B9, c.n, node, pidx, c.S, c.xn);
        else b = c.A9[(size_t)4 * c.n + node] * (kind == -2 ? c.outer_value : c.ufc[kind]);
        const double r0 = b - stencil_row<3>(c.A9, c.n, node, pidx, c.S, guess);
        c.r[pidx] = r0;
        bb[0] += b * b;
    }
    block_sum<1>(bb, lds);
    if (threadIdx.x == 0) c.partials[2 * gridDim.x * 4 + blockIdx.x] = bb[0];
}

// Right-preconditioned BiCGSTAB on (A P) y = r0, x = x0 + P y.
__global__ void __launch_bounds__(kBlock) coarse_bicgstab_kernel(CoarseDev c, const double *__restrict__ guess,
                                                                 int max_iter, double tol) {
    __shared__ double lds[64];
    unsigned round = 0;
    int parity = 0;
    const int stride = gridDim.x * blockDim.x;
    const int first = blockIdx.x * blockDim.x + threadIdx.x;

    double bnorm2 = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) bnorm2 += c.partials[2 * gridDim.x * 4 + b];
    const double bnorm = sqrt(bnorm2);

    double red[2] = {0.0, 0.0};
    for (int node = first; node < c.n; node += stride) {
        const int pi = padded_index(c, node);
        const double r = c.r[pi];
        c.rh[pi] = r;
        c.p[pi] = 0.0;
        c.v[pi] = 0.0;
        c.y[pi] = 0.0;
        red[0] += r * r;
        red[1] += r * r;
    }
    bool ok = grid_sum<2>(c, red, round, parity, lds);
    double rnorm = sqrt(red[0]);
    double rho = 1.0, alpha = 1.0, omega = 1.0, rho1 = red[1];
    int it = 0;
    const double target = tol * (bnorm > 0.0 ? bnorm : 1.0);
    bool converged = rnorm <= target;
    while (ok && !converged && it < max_iter) {
        ++it;
        const double beta = (rho1 / rho) * (alpha / omega);
        rho = rho1;
        for (int node = first; node < c.n; node += stride) {
            const int pi = padded_index(c, node);
            c.p[pi] = c.r[pi] + beta * (c.p[pi] - omega * c.v[pi]);
        }
        if (!(ok = grid_barrier(c, round))) break;
        double d1[1] = {0.0};
        for (int node = first; node < c.n; node += stride) {
            const int pi = padded_index(c, node);
            const double vv = stencil_row<kApW>(c.AP, c.n, node, pi, c.S, c.p);
            c.v[pi] = vv;
            d1[0] += c.rh[pi] * vv;
        }
        if (!(ok = grid_sum<1>(c, d1, round, parity, lds))) break;
        alpha = rho / d1[0];
        for (int node = first; node < c.n; node += stride) {
            const int pi = padded_index(c, node);
            c.s[pi] = c.r[pi] - alpha * c.v[pi];
        }
        if (!(ok = grid_barrier(c, round))) break;
        double d2[2] = {0.0, 0.0};
        for (int node = first; node < c.n; node += stride) {
            const int pi = padded_index(c, node);
            const double tt = stencil_row<kApW>(c.AP, c.n, node, pi, c.S, c.s);
            c.t[pi] = tt;
            d2[0] += tt * c.s[pi];
            d2[1] += tt * tt;
        }
        if (!(ok = grid_sum<2>(c, d2, round, parity, lds))) break;
        omega = d2[1] > 0.0 ? d2[0] / d2[1] : 0.0;
        double d3[2] = {0.0, 0.0};
        for (int node = first; node < c.n; node += stride) {
            const int pi = padded_index(c, node);
            const double sv = c.s[pi];
            c.y[pi] += alpha * c.p[pi] + omega * sv;
            const double rn = sv - omega * c.t[pi];
            c.r[pi] = rn;
            d3[0] += rn * rn;
            d3[1] += c.rh[pi] * rn;
        }
        if (!(ok = grid_sum<2>(c, d3, round, parity, lds))) break;
        rnorm = sqrt(d3[0]);
        rho1 = d3[1];
        converged = rnorm <= target;
        if (omega == 0.0 || rho1 == 0.0) break;
    }
    if (ok) ok = grid_barrier(c, round);
    if (ok) {
        for (int node = first; node < c.n; node += stride) {
            const int pi = padded_index(c, node);
            c.x1[pi] = guess[pi] + stencil_row<kSpaiW>(c.P, c.n, node, pi, c.S, c.y);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c.result->iters = it;
        c.result->converged = (ok && converged) ? 1 : 0;
        c.result->relres = bnorm > 0.0 ? rnorm / bnorm : rnorm;
    }
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

// ufc[c] = sum of the four weighted lattice concentrations around Gamma_{f->c} node c.
template <typename T>
__global__ void f2c_kernel(LbmArgs lat, const int *__restrict__ idx, const double *__restrict__ w, int nfc,
                           double *__restrict__ ufc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nfc) return;
    const T *__restrict__ src = static_cast<const T *>(lat.src);
    const int S = static_cast<int>(lat.plane);
    double acc = 0.0;
    for (int m = 0; m < 4; ++m) {
        const double wm = w[4 * c + m];
        if (wm == 0.0) continue;
        const int n = idx[4 * c + m];
        double u = 0.0;
        for (int q = 0; q < kQ; ++q) u += double(src[q * S + n]);
        const double k = lat.kfield ? double(static_cast<const T *>(lat.kfield)[n]) : lat.k;
        acc += wm * (u / (1.0 - k));
    }
    ufc[c] = acc;
}

}  // namespace

hipError_t launch_coarse_rhs(const CoarseDev &c, const double *guess, hipStream_t s) {
    hipLaunchKernelGGL(coarse_rhs_kernel, dim3(c.grid), dim3(kBlock), 0, s, c, guess);
    return hipGetLastError();
}

hipError_t launch_coarse_solve(const CoarseDev &c, const double *guess, int max_iter, double tol,
                               hipStream_t s) {
    if (c.grid == 1) {
        hipLaunchKernelGGL(coarse_bicgstab_kernel, dim3(1), dim3(kBlock), 0, s, c, guess, max_iter, tol);
        return hipGetLastError();
    }
    CoarseDev cc = c;
    const double *g = guess;
    void *args[] = {&cc, &g, &max_iter, &tol};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(coarse_bicgstab_kernel), dim3(c.grid),
                                      dim3(kBlock), args, 0, s);
}

hipError_t launch_c2f(const int *idx, const double *w, int nslots, const double *xa, const double *xb, double *a,
                      double *b, hipStream_t s) {
    hipLaunchKernelGGL(c2f_kernel, dim3((nslots + 255) / 256), dim3(256), 0, s, idx, w, nslots, xa, xb, a, b);
    return hipGetLastError();
}

hipError_t launch_f2c(const LbmArgs &lat, const int *idx, const double *w, int nfc, double *ufc, bool fp64,
                      hipStream_t s) {
    if (nfc == 0) return hipSuccess;
    if (fp64) hipLaunchKernelGGL(f2c_kernel<double>, dim3((nfc + 255) / 256), dim3(256), 0, s, lat, idx, w, nfc, ufc);
    else hipLaunchKernelGGL(f2c_kernel<float>, dim3((nfc + 255) / 256), dim3(256), 0, s, lat, idx, w, nfc, ufc);
    return hipGetLastError();
}

}  // namespace hyb
