// One-dimensional hybrid of Sec. 7.1 (D1Q2 lattice Boltzmann coupled to
// linear Galerkin elements by Algorithm 1, Sec. 6.2) behind include/hyb1d.h.
//
// The problem is small (at most 2048 fine and 1024 coarse nodes) and every
// step depends on the previous one, so the whole run lives in one
// workgroup: the fine populations and the coarse solution stay in LDS for
// all coarse steps of a call, the fine steps are separated by workgroup
// barriers, and the tridiagonal coarse solve is the Thomas recurrence on
// one lane with the factorisation of A prepared at set-up.  Arithmetic is
// FP64 and, in the lattice and the right-hand side, in the order of the
// formulas (no contraction into fused multiply-adds).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "hyb.h"
#include "hyb1d.h"

namespace {

constexpr int kMaxF = 2048;
constexpr int kMaxC = 1024;
constexpr int kThreads = 1024;
constexpr size_t kAlign = 256;

struct Dev1D {
    int nf, nc, eta, max_iter;
    int ic;                     // coarse node at the fine subdomain's left end
    int iff;                    // fine node at the coarse subdomain's right end
    double vl, tau;             // D1Q2 lattice velocity and relaxation time
    const double *bl, *bd, *bu; // rows of B: sub-, main and super-diagonal [nc]
    const double *ta, *tinv, *tc;   // A = LU (Thomas): sub-diagonal, 1 / pivot, c' [nc]
    double *fstar;              // [2][nf] committed post-collision populations (+, -)
    double *d;                  // [nc] committed coarse solution
};

__device__ __forceinline__ void collide(double &fp, double &fm, double vl, double tau) {
#pragma clang fp contract(off)
    const double u = fp + fm;
    const double ep = 0.5 * u * (1.0 + vl), em = 0.5 * u * (1.0 - vl);
    fp = fp + (ep - fp) / tau;
    fm = fm + (em - fm) / tau;
}

__global__ void __launch_bounds__(kThreads) hyb1d_init_kernel(Dev1D h, const double *__restrict__ u0) {
    for (int i = threadIdx.x; i < h.nf; i += blockDim.x) {
#pragma clang fp contract(off)
        const double u = u0[i];
        double fp = 0.5 * u * (1.0 + h.vl), fm = 0.5 * u * (1.0 - h.vl);
        collide(fp, fm, h.vl, h.tau);
        h.fstar[i] = fp;
        h.fstar[h.nf + i] = fm;
    }
}

// n_steps coarse steps of Algorithm 1.  Every Schwarz iteration restarts
// the fine steps from the committed populations; the first takes the
// fine-to-coarse value from them, later ones from the previous iteration's
// result; fine step j of eta receives u^p = (1 - j/eta) a + (j/eta) b.
__global__ void __launch_bounds__(kThreads) hyb1d_run_kernel(Dev1D h, int n_steps) {
#pragma clang fp contract(off)
    __shared__ double sf[2][kMaxF];      // committed populations (with the rest, 112 KB of LDS)
    __shared__ double sF[2][kMaxF];      // populations of the running iteration
    __shared__ double sd[kMaxC], sd1[kMaxC], sr[kMaxC];
    __shared__ double sta[kMaxC], stinv[kMaxC], stc[kMaxC];   // the factorisation of A, read by one lane
    const int nf = h.nf, nc = h.nc, tid = threadIdx.x;
    for (int i = tid; i < nc; i += kThreads) {
        sta[i] = h.ta[i];
        stinv[i] = h.tinv[i];
        stc[i] = h.tc[i];
    }
    for (int i = tid; i < nf; i += kThreads) {
        sf[0][i] = h.fstar[i];
        sf[1][i] = h.fstar[nf + i];
    }
    for (int i = tid; i < nc; i += kThreads) sd[i] = h.d[i];
    __syncthreads();
    for (int step = 0; step < n_steps; ++step) {
        double ufc = sf[0][h.iff] + sf[1][h.iff];
        const double a = sd[h.ic];
        for (int it = 0; it < h.max_iter; ++it) {
            // right-hand side B d, Dirichlet row last
            for (int i = tid; i < nc; i += kThreads) {
                double r = 0.0;
                if (i > 0) r += h.bl[i] * sd[i - 1];
                r += h.bd[i] * sd[i];
                if (i < nc - 1) r += h.bu[i] * sd[i + 1];
                sr[i] = i == nc - 1 ? ufc : r;
            }
            __syncthreads();
            if (tid == 0) {
                // the recurrences from LDS, unrolled so that the next
                // coefficients load while the previous element finishes
                double y = sr[0] * stinv[0];
                sd1[0] = y;
#pragma unroll 8
                for (int i = 1; i < nc; ++i) {
                    y = (sr[i] - sta[i] * y) * stinv[i];
                    sd1[i] = y;
                }
                double x = y;
#pragma unroll 8
                for (int i = nc - 2; i >= 0; --i) {
                    x = sd1[i] - stc[i] * x;
                    sd1[i] = x;
                }
            }
            for (int i = tid; i < nf; i += kThreads) {
                sF[0][i] = sf[0][i];
                sF[1][i] = sf[1][i];
            }
            __syncthreads();
            const double b = sd1[h.ic];
            for (int j = 1; j <= h.eta; ++j) {
                const double lam = (double)j / (double)h.eta;
                const double up = (1.0 - lam) * a + lam * b;
                // pull: + moves right, - moves left; closures at both ends
                double fp[kMaxF / kThreads], fm[kMaxF / kThreads];
#pragma unroll
                for (int k = 0; k < kMaxF / kThreads; ++k) {
                    const int i = tid + k * kThreads;
                    if (i >= nf) continue;
                    fm[k] = i < nf - 1 ? sF[1][i + 1] : sF[0][nf - 2];
                    fp[k] = i > 0 ? sF[0][i - 1] : up - sF[1][1];
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < kMaxF / kThreads; ++k) {
                    const int i = tid + k * kThreads;
                    if (i >= nf) continue;
                    collide(fp[k], fm[k], h.vl, h.tau);
                    sF[0][i] = fp[k];
                    sF[1][i] = fm[k];
                }
                __syncthreads();
            }
            ufc = sF[0][h.iff] + sF[1][h.iff];
        }
        // commit the last iteration
        for (int i = tid; i < nf; i += kThreads) {
            sf[0][i] = sF[0][i];
            sf[1][i] = sF[1][i];
        }
        for (int i = tid; i < nc; i += kThreads) sd[i] = sd1[i];
        __syncthreads();
    }
    for (int i = tid; i < nf; i += kThreads) {
        h.fstar[i] = sf[0][i];
        h.fstar[nf + i] = sf[1][i];
    }
    for (int i = tid; i < nc; i += kThreads) h.d[i] = sd[i];
}

__global__ void hyb1d_conc_kernel(Dev1D h, double *__restrict__ u) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < h.nf; i += gridDim.x * blockDim.x)
        u[i] = h.fstar[i] + h.fstar[h.nf + i];
}

struct Sizes {
    int nc = 0, nf = 0, eta = 0, ic = 0, iff = 0;
    double xf0 = 0.0, dt_c = 0.0, dt_f = 0.0;
    size_t off_b = 0, off_t = 0, off_f = 0, off_d = 0, off_u = 0, total = 0;
};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool near_int(double x, int &n) {
    n = (int)std::lround(x);
    return std::fabs(x - n) < 1e-9 * std::max(1.0, std::fabs(x));
}

// the discretisation of the 1-D set-up, or an empty string when it is invalid
std::string sizes_of(const hyb1d_params *p, Sizes &S) {
    if (!p || !(p->h_c > 0.0) || !(p->h_f > 0.0) || !(p->D > 0.0) || !(p->L_ov > 0.0) || p->L_ov >= 1.0 ||
        p->max_iter < 1 || !std::isfinite(p->v))
        return "invalid parameters";
    S.dt_c = p->h_c * p->h_c / (2.0 * p->D);
    S.dt_f = p->h_f * p->h_f / (2.0 * p->D);
    if (!near_int(S.dt_c / S.dt_f, S.eta) || S.eta < 1) return "(h_c / h_f)^2 must be an integer";
    const double xc_end = 0.5 + 0.5 * p->L_ov, xf_start = 0.5 - 0.5 * p->L_ov;
    int nc, nf, ic, iff;
    if (!near_int(xc_end / p->h_c, nc) || std::fabs(nc * p->h_c - xc_end) > 1e-9)
        return "1/2 + L_ov/2 must be a multiple of h_c";
    if (!near_int((1.0 - xf_start) / p->h_f, nf) || std::fabs(nf * p->h_f - (1.0 - xf_start)) > 1e-9)
        return "1/2 - L_ov/2 must leave a whole number of fine cells";
    if (!near_int(xf_start / p->h_c, ic) || std::fabs(ic * p->h_c - xf_start) > 1e-9)
        return "the fine subdomain must start at a coarse node";
    if (!near_int((xc_end - xf_start) / p->h_f, iff) || std::fabs(xf_start + iff * p->h_f - xc_end) > 1e-9)
        return "the coarse subdomain must end at a fine node";
    S.nc = nc + 1;
    S.nf = nf + 1;
    S.ic = ic;
    S.iff = iff;
    S.xf0 = xf_start;
    if (S.nf > kMaxF || S.nc > kMaxC || S.nf < 3 || S.nc < 3) return "at most 2048 fine and 1024 coarse nodes";
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    S.off_b = take(3 * (size_t)S.nc * 8);
    S.off_t = take(3 * (size_t)S.nc * 8);
    S.off_f = take(2 * (size_t)S.nf * 8);
    S.off_d = take((size_t)S.nc * 8);
    S.off_u = take((size_t)S.nf * 8);
    S.total = off;
    return std::string();
}

}  // namespace

struct hyb1d_handle {
    Dev1D dev{};
    Sizes S;
    hipStream_t stream = nullptr;
    double *ubuf = nullptr;
};

extern "C" {

int hyb1d_query(const hyb1d_params *p, int *nc, int *nf, int *eta, double *xf0, size_t *ws_bytes) {
    Sizes S;
    if (!sizes_of(p, S).empty()) return HYB_EINVAL;
    if (nc) *nc = S.nc;
    if (nf) *nf = S.nf;
    if (eta) *eta = S.eta;
    if (xf0) *xf0 = S.xf0;
    if (ws_bytes) *ws_bytes = S.total;
    return HYB_OK;
}

int hyb1d_create(const hyb1d_params *p, const double *d0, const double *u0, void *workspace, void *stream,
                 hyb1d_handle **out) {
    if (!out) return HYB_EINVAL;
    *out = nullptr;
    Sizes S;
    const std::string msg = sizes_of(p, S);
    if (!msg.empty()) {
        std::fprintf(stderr, "hyb1d_create: %s\n", msg.c_str());
        return HYB_EINVAL;
    }
    if (!d0 || !u0 || !workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign) return HYB_EINVAL;
    const int nc = S.nc, nf = S.nf;
    // coarse matrices: consistent mass, Galerkin advection and diffusion
    std::vector<double> Ml(nc, 0.0), Md(nc, 0.0), Mu(nc, 0.0), Kl(nc, 0.0), Kd(nc, 0.0), Ku(nc, 0.0);
    const double hc = p->h_c;
    const double me[2][2] = {{hc / 6.0 * 2.0, hc / 6.0}, {hc / 6.0, hc / 6.0 * 2.0}};
    const double ke[2][2] = {{-p->v / 2.0 + p->D / hc, p->v / 2.0 - p->D / hc},
                             {-p->v / 2.0 - p->D / hc, p->v / 2.0 + p->D / hc}};
    for (int e = 0; e < nc - 1; ++e) {
        Md[e] += me[0][0];
        Mu[e] += me[0][1];
        Ml[e + 1] += me[1][0];
        Md[e + 1] += me[1][1];
        Kd[e] += ke[0][0];
        Ku[e] += ke[0][1];
        Kl[e + 1] += ke[1][0];
        Kd[e + 1] += ke[1][1];
    }
    const double hdt = 0.5 * S.dt_c;
    std::vector<double> host(3 * (size_t)nc * 2, 0.0);
    double *bl = host.data(), *bd = bl + nc, *bu = bd + nc;
    double *ta = bu + nc, *tinv = ta + nc, *tc = tinv + nc;
    std::vector<double> al(nc), ad(nc), au(nc);
    for (int i = 0; i < nc; ++i) {
        bl[i] = Ml[i] - hdt * Kl[i];
        bd[i] = Md[i] - hdt * Kd[i];
        bu[i] = Mu[i] - hdt * Ku[i];
        al[i] = Ml[i] + hdt * Kl[i];
        ad[i] = Md[i] + hdt * Kd[i];
        au[i] = Mu[i] + hdt * Ku[i];
    }
    al[nc - 1] = 0.0;                       // Dirichlet row: identity
    ad[nc - 1] = 1.0;
    au[nc - 1] = 0.0;
    for (int i = 0; i < nc; ++i) {
        const double piv = ad[i] - (i > 0 ? al[i] * tc[i - 1] : 0.0);
        if (!(std::fabs(piv) > 0.0)) return HYB_EINVAL;
        tinv[i] = 1.0 / piv;
        tc[i] = au[i] * tinv[i];
        ta[i] = al[i];
    }
    hyb1d_handle *h = new hyb1d_handle();
    h->S = S;
    h->stream = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    Dev1D &d = h->dev;
    d.nf = nf;
    d.nc = nc;
    d.eta = S.eta;
    d.max_iter = p->max_iter;
    d.ic = S.ic;
    d.iff = S.iff;
    d.vl = p->v * S.dt_f / p->h_f;
    d.tau = 0.5 + p->D * S.dt_f / (p->h_f * p->h_f);
    double *B = reinterpret_cast<double *>(ws + S.off_b);
    double *T = reinterpret_cast<double *>(ws + S.off_t);
    d.bl = B;
    d.bd = B + nc;
    d.bu = B + 2 * nc;
    d.ta = T;
    d.tinv = T + nc;
    d.tc = T + 2 * nc;
    d.fstar = reinterpret_cast<double *>(ws + S.off_f);
    d.d = reinterpret_cast<double *>(ws + S.off_d);
    h->ubuf = reinterpret_cast<double *>(ws + S.off_u);
    auto fail = [&](hipError_t e) {
        std::fprintf(stderr, "hyb1d_create: %s\n", hipGetErrorString(e));
        delete h;
        return HYB_EHIP;
    };
    hipError_t e;
    if ((e = hipMemcpyAsync(B, bl, 3 * (size_t)nc * 8, hipMemcpyHostToDevice, h->stream)) != hipSuccess) return fail(e);
    if ((e = hipMemcpyAsync(T, ta, 3 * (size_t)nc * 8, hipMemcpyHostToDevice, h->stream)) != hipSuccess) return fail(e);
    if ((e = hipMemcpyAsync(d.d, d0, (size_t)nc * 8, hipMemcpyHostToDevice, h->stream)) != hipSuccess) return fail(e);
    if ((e = hipMemcpyAsync(h->ubuf, u0, (size_t)nf * 8, hipMemcpyHostToDevice, h->stream)) != hipSuccess) return fail(e);
    hipLaunchKernelGGL(hyb1d_init_kernel, dim3(1), dim3(kThreads), 0, h->stream, d, h->ubuf);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return fail(e);
    *out = h;
    return HYB_OK;
}

int hyb1d_run(hyb1d_handle *h, int n_steps) {
    if (!h || n_steps < 0) return HYB_EINVAL;
    if (n_steps == 0) return HYB_OK;
    hipLaunchKernelGGL(hyb1d_run_kernel, dim3(1), dim3(kThreads), 0, h->stream, h->dev, n_steps);
    return hipGetLastError() == hipSuccess ? HYB_OK : HYB_EHIP;
}

int hyb1d_state(hyb1d_handle *h, double *d, double *u) {
    if (!h) return HYB_EINVAL;
    hipLaunchKernelGGL(hyb1d_conc_kernel, dim3(4), dim3(256), 0, h->stream, h->dev, h->ubuf);
    if (hipGetLastError() != hipSuccess) return HYB_EHIP;
    if (d && hipMemcpyAsync(d, h->dev.d, (size_t)h->S.nc * 8, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return HYB_EHIP;
    if (u && hipMemcpyAsync(u, h->ubuf, (size_t)h->S.nf * 8, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return HYB_EHIP;
    return hipStreamSynchronize(h->stream) == hipSuccess ? HYB_OK : HYB_EHIP;
}

void hyb1d_destroy(hyb1d_handle *h) { delete h; }

}  // extern "C"
