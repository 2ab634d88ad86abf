// Reverse mode of one coarse step's coarse half: the transposes of the
// coarse-to-fine interpolation (Sec. 6.2, item i), of the trapezoidal step
// with strong Dirichlet rows (eq. FEM_discrete) and of the fine-to-coarse
// transfer (Sec. 6.2, item ii).  Every transpose is a gather over lists or
// stencils built on the host, so each output element is written by one lane
// (or one wavefront) and summed in a fixed order (deterministic, no
// atomics).
#include "hyb_impl.h"

namespace hyb {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int pad_of(const CoarseDev &c, int node) {
    const int m1 = c.M + 1;
    return (node / m1 + kCoarseHalo) * c.S + (node % m1 + kCoarseHalo);
}

// lam_dn += C^T ga, lam_d1 = C^T gb (+ lam_d_dense) at every mesh node
// One wavefront per mesh node: a node of an element the patch perimeter
// crosses gathers thousands of slots, so lane l sums entries l, l + 64, ...
// of the node's list and the lanes combine in a fixed tree (deterministic).
constexpr int kGatherLanes = 64;
__global__ void __launch_bounds__(kGatherLanes)
    c2f_transpose_kernel(CoarseDev c, const int *__restrict__ ptr, const int *__restrict__ slot,
                         const double *__restrict__ w, const double *__restrict__ ga, const double *__restrict__ gb,
                         const double *__restrict__ lam_d_dense, double *__restrict__ lam_dn,
                         double *__restrict__ lam_d1) {
    const int node = blockIdx.x;
    const int lane = threadIdx.x;
    double sa = 0.0, sb = 0.0;
    for (int e = ptr[node] + lane; e < ptr[node + 1]; e += kGatherLanes) {
        sa += w[e] * ga[slot[e]];
        sb += w[e] * gb[slot[e]];
    }
#pragma unroll
    for (int off = kGatherLanes / 2; off > 0; off >>= 1) {
        sa += __shfl_down(sa, off, kGatherLanes);
        sb += __shfl_down(sb, off, kGatherLanes);
    }
    if (lane == 0) {
        const int pi = pad_of(c, node);
        lam_dn[pi] += sa;
        lam_d1[pi] = lam_d_dense ? sb + lam_d_dense[node] : sb;
    }
}

// out = S in at every mesh node, S offset-major of width W (halo >= W/2)
template <int W>
__global__ void stencil_kernel(CoarseDev c, const double *__restrict__ coef, const double *__restrict__ in,
                               double *__restrict__ out) {
    constexpr int R = W / 2;
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= c.n) return;
    const int pi = pad_of(c, node);
    double acc = 0.0;
#pragma unroll
    for (int dl = -R; dl <= R; ++dl)
#pragma unroll
        for (int dk = -R; dk <= R; ++dk)
            acc += coef[(size_t)((dl + R) * W + (dk + R)) * c.n + node] * in[pi + dl * c.S + dk];
    out[pi] = acc;
}

// lam_dn[i] += sum over free rows j next to i of B(j, i) mu[j]; the
// Gamma_{f->c} row of index t receives lam_ufc[t] = a_ii mu[row] (its
// right-hand side is a_ii times the transferred value); an outer-edge row
// adds a_ii mu to grad_outer (its right-hand side is a_ii times the
// prescribed value)
__global__ void rhs_transpose_kernel(CoarseDev c, const int *__restrict__ fc_row, int nfc,
                                     const double *__restrict__ mu, double *__restrict__ lam_dn,
                                     double *__restrict__ lam_ufc, double *__restrict__ grad_outer) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= c.n) return;
    const int m1 = c.M + 1;
    const int kk = t % m1, l = t / m1;
    double s = 0.0;
#pragma unroll
    for (int dl = -1; dl <= 1; ++dl)
#pragma unroll
        for (int dk = -1; dk <= 1; ++dk) {
            const int nk = kk + dk, nl = l + dl;
            if (nk < 0 || nk > c.M || nl < 0 || nl > c.M) continue;
            const int j = nl * m1 + nk;
            if (c.dkind[j] != -1) continue;
            // B(j, t): row j at offset (-dk, -dl)
            s += c.B9[(size_t)((1 - dl) * 3 + (1 - dk)) * c.n + j] * mu[pad_of(c, j)];
        }
    lam_dn[pad_of(c, t)] += s;
    if (grad_outer && c.dkind[t] == -2) grad_outer[t] += c.A9[(size_t)4 * c.n + t] * mu[pad_of(c, t)];
    if (t < nfc) {
        const int row = fc_row[t];
        lam_ufc[t] = c.A9[(size_t)4 * c.n + row] * mu[pad_of(c, row)];
    }
}

template <typename T>
__global__ void f2c_transpose_kernel(LbmArgs lat, const int *__restrict__ node, const int *__restrict__ ptr,
                                     const int *__restrict__ cidx, const double *__restrict__ w, int ntouched,
                                     const double *__restrict__ lam_ufc, const T *__restrict__ g,
                                     T *__restrict__ lam_pitched, double *__restrict__ lam_dense,
                                     double *__restrict__ grad_k) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntouched) return;
    const int n = node[t];
    const int plane = static_cast<int>(lat.plane);
    double lam_u = 0.0;
    for (int e = ptr[t]; e < ptr[t + 1]; ++e) lam_u += w[e] * lam_ufc[cidx[e]];
    const double k = lat.kfield ? double(static_cast<const T *>(lat.kfield)[n]) : lat.k;
    const double inv = 1.0 / (1.0 - k);
    const int i = n % lat.pitch, j = n / lat.pitch;
    if (lam_pitched) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) lam_pitched[q * plane + n] += T(lam_u * inv);
    } else {
#pragma unroll
        for (int q = 0; q < kQ; ++q) lam_dense[((size_t)q * lat.N + j) * lat.N + i] += lam_u * inv;
    }
    if (grad_k) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kQ; ++q) s += double(g[q * plane + n]);
        grad_k[(size_t)j * lat.N + i] += lam_u * s * inv * inv;
    }
}

__global__ void repad_kernel(CoarseDev c, const double *__restrict__ from, double *__restrict__ to, int to_dense) {
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= c.n) return;
    const int pi = pad_of(c, node);
    if (to_dense) to[node] = from[pi];
    else to[pi] = from[node];
}

int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

hipError_t launch_c2f_transpose(const CoarseDev &c, const int *ptr, const int *slot, const double *w, const double *ga,
                                const double *gb, const double *lam_d_dense, double *lam_dn, double *lam_d1,
                                hipStream_t s) {
    hipLaunchKernelGGL(c2f_transpose_kernel, dim3(c.n), dim3(kGatherLanes), 0, s, c, ptr, slot, w, ga, gb,
                       lam_d_dense, lam_dn, lam_d1);
    return hipGetLastError();
}

hipError_t launch_coarse_stencil(const CoarseDev &c, const double *coef, int W, const double *in, double *out,
                                 hipStream_t s) {
    if (W != kSpaiW) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stencil_kernel<kSpaiW>, dim3(blocks_for(c.n)), dim3(kBlock), 0, s, c, coef, in, out);
    return hipGetLastError();
}

hipError_t launch_coarse_rhs_transpose(const CoarseDev &c, const int *fc_row, int nfc, const double *mu,
                                       double *lam_dn, double *lam_ufc, double *grad_outer, hipStream_t s) {
    hipLaunchKernelGGL(rhs_transpose_kernel, dim3(blocks_for(c.n)), dim3(kBlock), 0, s, c, fc_row, nfc, mu, lam_dn,
                       lam_ufc, grad_outer);
    return hipGetLastError();
}

hipError_t launch_f2c_transpose(const LbmArgs &lat, int prec, const int *node, const int *ptr, const int *cidx,
                                const double *w, int ntouched, const double *lam_ufc, const void *g_state,
                                void *lam_pitched, double *lam_dense, double *grad_k, hipStream_t s) {
    if (ntouched == 0) return hipSuccess;
    if (prec == HYB_FP64)
        hipLaunchKernelGGL(f2c_transpose_kernel<double>, dim3(blocks_for(ntouched)), dim3(kBlock), 0, s, lat, node,
                           ptr, cidx, w, ntouched, lam_ufc, static_cast<const double *>(g_state),
                           static_cast<double *>(lam_pitched), lam_dense, grad_k);
    else if (prec == HYB_FP32)
        hipLaunchKernelGGL(f2c_transpose_kernel<float>, dim3(blocks_for(ntouched)), dim3(kBlock), 0, s, lat, node,
                           ptr, cidx, w, ntouched, lam_ufc, static_cast<const float *>(g_state),
                           static_cast<float *>(lam_pitched), lam_dense, grad_k);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_coarse_repad(const CoarseDev &c, const double *from, double *to, bool to_dense, hipStream_t s) {
    hipLaunchKernelGGL(repad_kernel, dim3(blocks_for(c.n)), dim3(kBlock), 0, s, c, from, to, to_dense ? 1 : 0);
    return hipGetLastError();
}

}  // namespace hyb
