// Diagnostics of a lattice state on the device: the mass readout, the
// smallest population and the H function of eq. (BH) (Sec. 4.1), reduced in
// two passes with a fixed order so that the result does not depend on
// timing.
#include "hyb_impl.h"

namespace hyb {
namespace {

__device__ __forceinline__ bool finite_val(double x) { return x - x == 0.0; }

// per-node reaction rate (k field in the arithmetic type) or the uniform one
template <typename T>
__device__ __forceinline__ T node_k(const LbmArgs &a, int n) {
    return a.kfield ? static_cast<const T *>(a.kfield)[n] : T(a.k);
}

// Diagnostics of a lattice state (Sec. 4.1, eqs. LBM_Macro and BH), first
// pass: workgroup j reduces row j's fluid nodes to four partials,
//   part[4j + 0] = sum of u = sum_q f*_q / (1 - k)   (the concentration readout),
//   part[4j + 1] = min over q of f*_q,
//   part[4j + 2] = sum over q with f*_q > 0 of f*_q ln(f*_q / w_q)  (eq. BH),
//   part[4j + 3] = number of nodes with a non-finite population,
// all in FP64 from the decoded stored values.  Each lane takes the nodes
// i = lane, lane + 256, ... in order and the lanes combine in a fixed tree,
// so the result does not depend on timing.
template <typename S>
__global__ void __launch_bounds__(256) lbm_diag_rows_kernel(LbmArgs a, double *__restrict__ part) {
    typedef typename Pop<S>::T T;
    __shared__ double red[4][256];
    const int N = a.N;
    const int j = blockIdx.x;
    const int P = a.pitch;
    const S *__restrict__ src = static_cast<const S *>(a.src);
    double m = 0.0, h = 0.0, bad = 0.0, mn = __builtin_inf();
    // ln(f / w) as ln f - ln w: one logarithm and no division per value
    double lnw[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) lnw[q] = log(kW[q]);
    // every node's values are loaded before its flag decides (no branch
    // between the loads of successive nodes, so they overlap)
#pragma unroll 4
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int n = j * P + i;
        S v[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) v[q] = src[q * a.plane + n];
        if (a.mask[n] & kMaskSolid) continue;
        double sum = 0.0;
        bool fin = true;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const double f = double(Pop<S>::ld(v[q], q, a));
            sum += f;
            fin = fin && finite_val(f);
            mn = f < mn ? f : mn;
            if (f > 0.0) h += f * (log(f) - lnw[q]);
        }
        m += sum / (1.0 - double(node_k<T>(a, n)));
        bad += fin ? 0.0 : 1.0;
    }
    const int t = threadIdx.x;
    red[0][t] = m;
    red[1][t] = mn;
    red[2][t] = h;
    red[3][t] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] = red[1][t + w] < red[1][t] ? red[1][t + w] : red[1][t];
            red[2][t] += red[2][t + w];
            red[3][t] += red[3][t + w];
        }
        __syncthreads();
    }
    if (t < 4) part[4 * j + t] = red[t][0];
}

// Second pass: one workgroup sums the rows' partials (lane t takes rows t,
// t + 256, ... in order, then a fixed tree) into out[0..3].
__global__ void __launch_bounds__(256) lbm_diag_finish_kernel(const double *__restrict__ part, int rows,
                                                              double *__restrict__ out) {
    __shared__ double red[4][256];
    const int t = threadIdx.x;
    double m = 0.0, h = 0.0, bad = 0.0, mn = __builtin_inf();
    for (int r = t; r < rows; r += blockDim.x) {
        m += part[4 * r + 0];
        mn = part[4 * r + 1] < mn ? part[4 * r + 1] : mn;
        h += part[4 * r + 2];
        bad += part[4 * r + 3];
    }
    red[0][t] = m;
    red[1][t] = mn;
    red[2][t] = h;
    red[3][t] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] = red[1][t + w] < red[1][t] ? red[1][t + w] : red[1][t];
            red[2][t] += red[2][t + w];
            red[3][t] += red[3][t + w];
        }
        __syncthreads();
    }
    if (t < 4) out[t] = red[t][0];
}

}  // namespace

hipError_t launch_diagnostics(const LbmArgs &a, int prec, double *part, double *out, hipStream_t s) {
    if (prec == HYB_FP64) hipLaunchKernelGGL(lbm_diag_rows_kernel<double>, dim3(a.N), dim3(256), 0, s, a, part);
    else if (prec == HYB_FP32) hipLaunchKernelGGL(lbm_diag_rows_kernel<float>, dim3(a.N), dim3(256), 0, s, a, part);
    else hipLaunchKernelGGL(lbm_diag_rows_kernel<_Float16>, dim3(a.N), dim3(256), 0, s, a, part);
    hipLaunchKernelGGL(lbm_diag_finish_kernel, dim3(1), dim3(256), 0, s, part, a.N, out);
    return hipGetLastError();
}

}  // namespace hyb
