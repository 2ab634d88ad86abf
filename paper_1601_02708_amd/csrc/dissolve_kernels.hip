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
// words are rebuilt.  The fine-to-coarse transfer (Sec. 6.2, item ii) then
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
template <typename S>
__global__ void __launch_bounds__(kBlock) dissolve_commit_kernel(LbmArgs a, double *__restrict__ mass,
                                                                  uint8_t *__restrict__ solid) {
    const int N = a.N, P = a.pitch;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int i = t % N, j = t / N;
    const int n = j * P + i;
    const unsigned m = a.mask[n];
    if (!(m & kMaskSolid)) return;
    // solid nodes without fluid neighbours moved nothing this step
    const double left = mass[n] - ((m & 0x1FEu) ? a.flux[n] : 0.0);
    if (!(left <= 0.0)) {
        mass[n] = left;
        return;
    }
    S *__restrict__ f = static_cast<S *>(a.dst);
    const int plane = static_cast<int>(a.plane);
    double sum = 0.0;
    int cnt = 0;
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
        const int xi = i + kCx[q], xj = j + kCy[q];
        if (xi < 0 || xi >= N || xj < 0 || xj >= N) continue;
        const int x = xj * P + xi;
        if (a.mask[x] & kMaskSolid) continue;
        sum += node_conc<S>(a, f, x, plane);
        cnt += 1;
    }
    const double ubar = cnt ? sum / cnt : 0.0;
    const double k = a.kfield ? double(static_cast<const typename Pop<S>::T *>(a.kfield)[n]) : a.k;
#pragma unroll
    for (int q = 0; q < kQ; ++q) f[q * plane + n] = Pop<S>::st(typename Pop<S>::T(kW[q] * ubar * (1.0 - k)), q, a);
    mass[n] = 0.0;
    solid[n] = 0;
    atomicAdd(&a.counters[kCntConverted], 1ull);
}

// Flag words from solid[]: a solid node carries bit 15 and a bit for every
// fluid neighbour x + e_q; a fluid node a bit for every solid upstream
// neighbour x - e_q inside the patch.
__global__ void __launch_bounds__(kBlock) mask_rebuild_kernel(int N, int P, const uint8_t *__restrict__ solid,
                                                               uint16_t *__restrict__ mask) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int i = t % N, j = t / N;
    const bool self = solid[j * P + i] != 0;
    unsigned m = self ? kMaskSolid : 0u;
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
        const int di = self ? kCx[q] : -kCx[q], dj = self ? kCy[q] : -kCy[q];
        const int xi = i + di, xj = j + dj;
        if (xi < 0 || xi >= N || xj < 0 || xj >= N) continue;
        const bool other = solid[xj * P + xi] != 0;
        if (self != other) m |= 1u << q;
    }
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

int blocks_for(long long n) { return (int)((n + kBlock - 1) / kBlock); }

template <typename S>
hipError_t commit_impl(const LbmArgs &a, double *mass, uint8_t *solid, uint16_t *mask, hipStream_t s) {
    const long long nodes = (long long)a.N * a.N;
    hipLaunchKernelGGL(dissolve_commit_kernel<S>, dim3(blocks_for(nodes)), dim3(kBlock), 0, s, a, mass, solid);
    hipLaunchKernelGGL(mask_rebuild_kernel, dim3(blocks_for(nodes)), dim3(kBlock), 0, s, a.N, a.pitch, solid, mask);
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

}  // namespace hyb
