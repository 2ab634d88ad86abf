/* One-dimensional hybrid (Sec. 7.1): D1Q2 lattice Boltzmann on the fine
 * subdomain (1/2 - L_ov/2, 1), two-node linear Galerkin finite elements on
 * the coarse subdomain (0, 1/2 + L_ov/2), coupled by Algorithm 1 (Sec. 6.2)
 * with the multi-time-step interface value of eq. (MTS).  The whole run
 * executes on the GPU in one workgroup per handle, its state resident in
 * LDS between coarse steps of one call.
 *
 * Model (the paper's 1-D set-up):
 *   - time steps dt = h^2 / (2 D) on both grids, so eta = (h_c / h_f)^2
 *     fine steps per coarse step (must be an integer);
 *   - D1Q2: velocities +-h_f/dt_f, weights 1/2, f_i^eq = (u/2)(1 + e_i v'),
 *     v' = v dt_f / h_f, BGK with tau = 1/2 + D dt_f / h_f^2, stored state
 *     the post-collision f*;
 *   - fine boundaries: at x = 1/2 - L_ov/2 the incoming population closes
 *     eq. (LBM_Dir) with one unknown, f_+ = u^p - f_-; at x = 1 zero flux,
 *     f_- = f_+;
 *   - coarse: linear elements, consistent mass, Galerkin advection-
 *     diffusion, trapezoidal rule A d1 = B d0 (A = M + dt_c/2 K,
 *     B = M - dt_c/2 K), zero flux at x = 0 (natural), Dirichlet at the
 *     right end from the lattice;
 *   - transfers: the interface points are nodes of the other grid (both
 *     1/2 -+ L_ov/2 must be multiples of h_c and h_f), so they are nodal.
 *
 * All functions return 0 or a negative HYB_* code of hyb.h (HYB_EINVAL for
 * a set-up that violates the conditions above or exceeds 2048 fine or 1024
 * coarse nodes).
 */
#ifndef HYB1D_H
#define HYB1D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hyb1d_handle hyb1d_handle;

typedef struct {
    double h_c, h_f;        /* coarse and fine spacings */
    double L_ov;            /* overlap length */
    int max_iter;           /* Schwarz iterations per coarse step, >= 1 */
    double v, D;            /* advection velocity and diffusion coefficient, D > 0 */
} hyb1d_params;

/* Sizes of a set-up: coarse nodes nc (x_k = k h_c), fine nodes nf
 * (x_i = xf0 + i h_f), eta, and the device workspace in bytes. */
int hyb1d_query(const hyb1d_params *p, int *nc, int *nf, int *eta, double *xf0, size_t *ws_bytes);

/* Create a handle: d0 host [nc] initial coarse nodal values, u0 host [nf]
 * initial fine concentration (f*(0) = collide(f^eq(u0)) on the device),
 * workspace: device memory of ws_bytes, 256-byte aligned, owned by the
 * caller; stream: hipStream_t or NULL.  Synchronises. */
int hyb1d_create(const hyb1d_params *p, const double *d0, const double *u0, void *workspace, void *stream,
                 hyb1d_handle **out);

/* Enqueue n_steps coarse steps (each max_iter Schwarz iterations of eta
 * fine steps) in one launch; returns without waiting. */
int hyb1d_run(hyb1d_handle *h, int n_steps);

/* Current coarse nodal values (host [nc]) and fine concentration f_+ + f_-
 * (host [nf]); either may be NULL.  Synchronises. */
int hyb1d_state(hyb1d_handle *h, double *d, double *u);

void hyb1d_destroy(hyb1d_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* HYB1D_H */
