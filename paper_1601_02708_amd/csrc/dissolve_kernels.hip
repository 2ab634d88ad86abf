// Dissolving solids: the commit of the pore geometry at the end of a coarse
// step and the fine-to-coarse transfer over the current fluid corners.
//
// The paper's pore-scale example (Sec. 7.4) keeps its solids fixed; the
// model here extends its halfway bounce-back (Sec. 4.1) with a first-order
// surface reaction: a population returned across a fluid-solid link relaxes
// towards w_q c_sat at rate kappa_s, and the mass that moves into the fluid
// is taken from the solid node.  The fine steps sum that mass per solid node
// (the sweep kernels, LbmArgs::flux); the kernels below act at the commit:
// masses are debited, exhausted solids become fluid with the equilibrium of
// their fluid neighbours' mean concentration at zero velocity, and the flag
// words are rebuilt -- three streams over the patch, no atomics.  The fine-to-coarse transfer (Sec. 6.2, item ii) then
// weights the current fluid corners.
#include "hyb_impl.h"

namespace hyb {
namespace {

constexpr int kBlock = 256;

template <typename S>
__device__ __forceinline__ double node_conc(const LbmArgs &a, const S *__restrict__ f, int n, int plane) {
    typedef typename Pop<S>::T T;
    double u = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) u += double(Pop<S>::ld(f[q * plane + n], q, a));
    const double k = a.kfield ? double(static_cast<const T *>(a.kfield)[n]) : a.k;
    return u / (1.0 - k);
}

// One lane per node of the patch.  Reads the flag words as they were
// before the commit (bit 15: solid) and writes only solid[] and, at nodes
// that convert, their populations and mass, so no lane reads what another
// writes: a converted node's neighbours that enter its mean are fluid.
// Loads are unconditional (neighbour coordinates clamped onto the patch,
// values of solid or outside neighbours discarded afterwards), so each lane
// waits for memory twice at most instead of once per neighbour.
// Commit, first kernel (one lane per node, a stream over the flag words):
// solid nodes with fluid neighbours lose their link-flux sum (the others
// moved nothing this step; their flux entry is not maintained); a node
// whose mass is then <= 0 becomes fluid (solid[] cleared, mass 0).  No
// atomics: one counter taking ~30k conversions per commit serialised them
// (0.8 ms), so converted nodes are counted on the host from solid[].
__global__ void __launch_bounds__(kBlock) dissolve_decide_kernel(LbmArgs a, double *__restrict__ mass,
                                                                  uint8_t *__restrict__ solid) {
    const int N = a.N, P = a.pitch;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int j = t / N, i = t - j * N;
    const int n = j * P + i;
    const unsigned m = a.mask[n];
    if (!(m & kMaskSolid)) return;
    const double held = mass[n], moved = a.flux[n];
    const double left = held - ((m & 0x1FEu) ? moved : 0.0);
    if (!(left <= 0.0)) {
        mass[n] = left;
    } else {
        mass[n] = 0.0;
        solid[n] = 0;
    }
}

// Commit, second kernel (one lane per node; the nodes whose flag word says
// solid and whose solid[] entry the first kernel cleared convert): f*_q =
// w_q (1 - k) u_mean into a.dst, u_mean the mean concentration of the
// node's fluid 8-neighbours (flag words before the commit) in q order.
// Neighbour flags and populations are loaded at clamped coordinates first
// and the values of solid or outside neighbours discarded, so a lane waits
// for memory twice.
template <typename S>
__global__ void __launch_bounds__(kBlock) dissolve_convert_kernel(LbmArgs a, const uint8_t *__restrict__ solid) {
    const int N = a.N, P = a.pitch;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int j = t / N, i = t - j * N;
    const int n = j * P + i;
    if (!(a.mask[n] & kMaskSolid) || solid[n]) return;
    S *__restrict__ f = static_cast<S *>(a.dst);
    const int plane = static_cast<int>(a.plane);
    int x[kQ];
    bool use[kQ];
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
        const int xi = i + kCx[q], xj = j + kCy[q];
        const bool inside = xi >= 0 && xi < N && xj >= 0 && xj < N;
        x[q] = min(max(xj, 0), N - 1) * P + min(max(xi, 0), N - 1);
        use[q] = inside && !(a.mask[x[q]] & kMaskSolid);
    }
    double sum = 0.0;
    int cnt = 0;
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
        const double u = node_conc<S>(a, f, x[q], plane);
        if (use[q]) {
            sum += u;
            cnt += 1;
        }
    }
    const double ubar = cnt ? sum / cnt : 0.0;
    const double k = a.kfield ? double(static_cast<const typename Pop<S>::T *>(a.kfield)[n]) : a.k;
#pragma unroll
    for (int q = 0; q < kQ; ++q) f[q * plane + n] = Pop<S>::st(typename Pop<S>::T(kW[q] * ubar * (1.0 - k)), q, a);
}

// Flag words from solid[]: a solid node carries bit 15 and a bit for every
// fluid neighbour x + e_q; a fluid node a bit for every solid upstream
// neighbour x - e_q inside the patch.
__global__ void __launch_bounds__(kBlock) mask_rebuild_kernel(int N, int P, const uint8_t *__restrict__ solid,
                                                               uint16_t *__restrict__ mask) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int j = t / N, i = t - j * N;
    const bool self = solid[j * P + i] != 0;
    // all eight neighbour flags are loaded at clamped coordinates first
    uint8_t other[kQ];
    bool inside[kQ];
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
        const int di = self ? kCx[q] : -kCx[q], dj = self ? kCy[q] : -kCy[q];
        const int xi = i + di, xj = j + dj;
        inside[q] = xi >= 0 && xi < N && xj >= 0 && xj < N;
        other[q] = solid[min(max(xj, 0), N - 1) * P + min(max(xi, 0), N - 1)];
    }
    unsigned m = self ? kMaskSolid : 0u;
#pragma unroll
    for (int q = 1; q < kQ; ++q)
        if (inside[q] && self != (other[q] != 0)) m |= 1u << q;
    mask[j * P + i] = static_cast<uint16_t>(m);
}

// ufc[c] = sum over fluid corners of w_m u_m, divided by the sum of their
// weights (both in corner order); the fallback node's concentration when
// no fluid corner carries weight.
template <typename S>
__global__ void f2c_dynamic_kernel(LbmArgs lat, const int *__restrict__ idx, const double *__restrict__ w,
                                   const int *__restrict__ fb, int nfc, double *__restrict__ ufc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nfc) return;
    const S *__restrict__ src = static_cast<const S *>(lat.src);
    const int plane = static_cast<int>(lat.plane);
    double acc = 0.0, wsum = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int n = idx[4 * c + m];
        if (lat.mask[n] & kMaskSolid) continue;
        const double wm = w[4 * c + m];
        acc += wm * node_conc<S>(lat, src, n, plane);
        wsum += wm;
    }
    if (wsum > 0.0) {
        ufc[c] = acc / wsum;
    } else {
        const int n = fb[c];
        ufc[c] = n >= 0 ? node_conc<S>(lat, src, n, plane) : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Reverse mode of a dissolving coarse step.  With its converting set fixed
// the commit maps the state before it linearly: a converted node n takes
// f*_q(n) = w_q (1 - k_n) ubar_n, ubar_n = (1/c_n) sum_{x in F(n)} u_x,
// u_x = sum_p f*_p(x) / (1 - k_x) over its c_n fluid neighbours F(n).  For
// the cotangent lam of the committed state: every fluid x gets
// sum_{n converted, x in F(n)} h_n / (1 - k_x) on all nine populations with
// h_n = (1 - k_n) sum_q w_q lam_q(n) / c_n; dJ/dk_n -= ubar_n sum_q w_q
// lam_q(n); dJ/dk_x += sum h_n u_x / (1 - k_x); lam(n) is cleared (the
// state before the commit at a solid node is not read).
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool converted_at(const LbmArgs &a, const uint8_t *__restrict__ after, int n) {
    return (a.mask[n] & kMaskSolid) && !after[n];
}

template <typename T>
__device__ __forceinline__ double conc_of(const LbmArgs &a, const T *__restrict__ f, int n, int plane) {
    double u = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) u += double(f[q * plane + n]);
    const double k = a.kfield ? double(static_cast<const T *>(a.kfield)[n]) : a.k;
    return u / (1.0 - k);
}

// per converted node: h_n into H, its own rate term into grad_k
template <typename T>
__global__ void __launch_bounds__(kBlock) conversion_t_nodes(LbmArgs a, const uint8_t *__restrict__ after,
                                                              const T *__restrict__ pre, const T *__restrict__ lam,
                                                              double *__restrict__ H, double *__restrict__ grad_k) {
    const int N = a.N, P = a.pitch;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int j = t / N, i = t - j * N;
    const int n = j * P + i;
    if (!converted_at(a, after, n)) return;
    const int plane = static_cast<int>(a.plane);
    double sum = 0.0;
    int cnt = 0;
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
        const int xi = i + kCx[q], xj = j + kCy[q];
        if (xi < 0 || xi >= N || xj < 0 || xj >= N) continue;
        const int x = xj * P + xi;
        if (a.mask[x] & kMaskSolid) continue;
        sum += conc_of<T>(a, pre, x, plane);
        cnt += 1;
    }
    double lw = 0.0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) lw += kW[q] * double(lam[q * plane + n]);
    const double k = a.kfield ? double(static_cast<const T *>(a.kfield)[n]) : a.k;
    H[n] = cnt ? (1.0 - k) * lw / cnt : 0.0;
    if (grad_k) grad_k[(size_t)j * N + i] -= (cnt ? sum / cnt : 0.0) * lw;
}

// per node: converted nodes clear their cotangent, fluid nodes next to
// converted ones receive their h_n (in place; each lane writes its node)
template <typename T>
__global__ void __launch_bounds__(kBlock) conversion_t_gather(LbmArgs a, const uint8_t *__restrict__ after,
                                                               const T *__restrict__ pre, T *__restrict__ lam,
                                                               const double *__restrict__ H,
                                                               double *__restrict__ grad_k) {
    const int N = a.N, P = a.pitch;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int j = t / N, i = t - j * N;
    const int n = j * P + i;
    const int plane = static_cast<int>(a.plane);
    const unsigned m = a.mask[n];
    if (m & kMaskSolid) {
        if (!after[n]) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) lam[q * plane + n] = T(0);
        }
        return;
    }
    // neighbours' flags first (clamped coordinates), then their h_n
    bool conv[kQ];
    int x[kQ];
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
        const int xi = i + kCx[q], xj = j + kCy[q];
        const bool inside = xi >= 0 && xi < N && xj >= 0 && xj < N;
        x[q] = min(max(xj, 0), N - 1) * P + min(max(xi, 0), N - 1);
        conv[q] = inside && converted_at(a, after, x[q]);
    }
    bool any = false;
#pragma unroll
    for (int q = 1; q < kQ; ++q) any |= conv[q];
    if (!any) return;
    double acc = 0.0;
#pragma unroll
    for (int q = 1; q < kQ; ++q)
        if (conv[q]) acc += H[x[q]];
    const double k = a.kfield ? double(static_cast<const T *>(a.kfield)[n]) : a.k;
    const double add = acc / (1.0 - k);
#pragma unroll
    for (int q = 0; q < kQ; ++q) lam[q * plane + n] = T(double(lam[q * plane + n]) + add);
    if (grad_k) grad_k[(size_t)j * N + i] += acc * conc_of<T>(a, pre, n, plane) / (1.0 - k);
}

// transposed dynamic fine-to-coarse transfer: per touched lattice node, the
// cotangents of the Gamma_{f->c} nodes that read it with their weights under
// the step's flag words
template <typename T>
__global__ void f2c_dynamic_transpose_kernel(LbmArgs lat, const int *__restrict__ node, const int *__restrict__ ptr,
                                             const int *__restrict__ cidx, const int *__restrict__ slot, int ntouched,
                                             const int *__restrict__ fcr_idx, const double *__restrict__ fcr_w,
                                             const double *__restrict__ lam_ufc, const T *__restrict__ g,
                                             T *__restrict__ lam_pitched, double *__restrict__ lam_dense,
                                             double *__restrict__ grad_k) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntouched) return;
    const int n = node[t];
    if (lat.mask[n] & kMaskSolid) return;
    double lam_u = 0.0;
    for (int e = ptr[t]; e < ptr[t + 1]; ++e) {
        const int c = cidx[e], m = slot[e];
        double wsum = 0.0;
#pragma unroll
        for (int mm = 0; mm < 4; ++mm)
            if (!(lat.mask[fcr_idx[4 * c + mm]] & kMaskSolid)) wsum += fcr_w[4 * c + mm];
        const double w = m < 4 ? (wsum > 0.0 ? fcr_w[4 * c + m] / wsum : 0.0) : (wsum > 0.0 ? 0.0 : 1.0);
        lam_u += w * lam_ufc[c];
    }
    const int plane = static_cast<int>(lat.plane);
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

int blocks_for(long long n) { return (int)((n + kBlock - 1) / kBlock); }

template <typename S>
hipError_t commit_impl(const LbmArgs &a, double *mass, uint8_t *solid, uint16_t *mask, hipStream_t s) {
    const dim3 grid(blocks_for((long long)a.N * a.N)), block(kBlock);
    hipLaunchKernelGGL(dissolve_decide_kernel, grid, block, 0, s, a, mass, solid);
    hipLaunchKernelGGL(dissolve_convert_kernel<S>, grid, block, 0, s, a, solid);
    hipLaunchKernelGGL(mask_rebuild_kernel, grid, block, 0, s, a.N, a.pitch, solid, mask);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dissolve_commit(const LbmArgs &a, int prec, double *mass, uint8_t *solid, uint16_t *mask,
                                  hipStream_t s) {
    if (!a.flux || !a.dst || !mass || !solid || !mask) return hipErrorInvalidValue;
    if (prec == HYB_FP64) return commit_impl<double>(a, mass, solid, mask, s);
    if (prec == HYB_FP32) return commit_impl<float>(a, mass, solid, mask, s);
    return commit_impl<_Float16>(a, mass, solid, mask, s);
}

hipError_t launch_f2c_dynamic(const LbmArgs &lat, const int *idx, const double *w, const int *fb, int nfc,
                              double *ufc, int prec, hipStream_t s) {
    if (nfc == 0) return hipSuccess;
    const dim3 grid((nfc + 63) / 64), block(64);
    if (prec == HYB_FP64) hipLaunchKernelGGL(f2c_dynamic_kernel<double>, grid, block, 0, s, lat, idx, w, fb, nfc, ufc);
    else if (prec == HYB_FP32) hipLaunchKernelGGL(f2c_dynamic_kernel<float>, grid, block, 0, s, lat, idx, w, fb, nfc, ufc);
    else hipLaunchKernelGGL(f2c_dynamic_kernel<_Float16>, grid, block, 0, s, lat, idx, w, fb, nfc, ufc);
    return hipGetLastError();
}

hipError_t launch_mask_rebuild(int N, int pitch, const uint8_t *solid, uint16_t *mask, hipStream_t s) {
    hipLaunchKernelGGL(mask_rebuild_kernel, dim3(blocks_for((long long)N * N)), dim3(kBlock), 0, s, N, pitch, solid,
                       mask);
    return hipGetLastError();
}

hipError_t launch_conversion_transpose(const LbmArgs &a, int prec, const uint8_t *after, const void *pre, void *lam,
                                       double *H, double *grad_k, hipStream_t s) {
    const dim3 grid(blocks_for((long long)a.N * a.N)), block(kBlock);
    if (prec == HYB_FP64) {
        hipLaunchKernelGGL(conversion_t_nodes<double>, grid, block, 0, s, a, after, static_cast<const double *>(pre),
                           static_cast<const double *>(lam), H, grad_k);
        hipLaunchKernelGGL(conversion_t_gather<double>, grid, block, 0, s, a, after, static_cast<const double *>(pre),
                           static_cast<double *>(lam), H, grad_k);
    } else if (prec == HYB_FP32) {
        hipLaunchKernelGGL(conversion_t_nodes<float>, grid, block, 0, s, a, after, static_cast<const float *>(pre),
                           static_cast<const float *>(lam), H, grad_k);
        hipLaunchKernelGGL(conversion_t_gather<float>, grid, block, 0, s, a, after, static_cast<const float *>(pre),
                           static_cast<float *>(lam), H, grad_k);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_f2c_dynamic_transpose(const LbmArgs &lat, int prec, const int *node, const int *ptr,
                                        const int *cidx, const int *slot, int ntouched, const int *fcr_idx,
                                        const double *fcr_w, const double *lam_ufc, const void *g_state,
                                        void *lam_pitched, double *lam_dense, double *grad_k, hipStream_t s) {
    if (ntouched == 0) return hipSuccess;
    const dim3 grid(blocks_for(ntouched)), block(kBlock);
    if (prec == HYB_FP64)
        hipLaunchKernelGGL(f2c_dynamic_transpose_kernel<double>, grid, block, 0, s, lat, node, ptr, cidx, slot,
                           ntouched, fcr_idx, fcr_w, lam_ufc, static_cast<const double *>(g_state),
                           static_cast<double *>(lam_pitched), lam_dense, grad_k);
    else if (prec == HYB_FP32)
        hipLaunchKernelGGL(f2c_dynamic_transpose_kernel<float>, grid, block, 0, s, lat, node, ptr, cidx, slot,
                           ntouched, fcr_idx, fcr_w, lam_ufc, static_cast<const float *>(g_state),
                           static_cast<float *>(lam_pitched), lam_dense, grad_k);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace hyb
