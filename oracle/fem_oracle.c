/*
 * CPU FP64 oracle, coarse-scale part: bilinear (Q1) finite elements for the
 * advection-diffusion-reaction equation, trapezoidal time stepping, a banded
 * LU solve, and the grid-transfer operators between the coarse mesh and the
 * fine lattice.  TEST INFRASTRUCTURE ONLY (see lbm_oracle.c).
 *
 *   - weak forms: Galerkin, eq. (Galerkin); SUPG, eqs. (SUPG) and (SUPG_tau)
 *   - semi-discrete system M u' + K u = s, eq. (FEM_semi); generalized
 *     trapezoid with theta = 1/2, eqs. (FEM_notation) and (FEM_discrete),
 *     written for the nodal values d:  (M + dt/2 K) d1 = (M - dt/2 K) d0
 *   - strong Dirichlet conditions (Sec. 3.1)
 *   - coarse-to-fine transfer: FEM interpolant of the containing element,
 *     and fine-to-coarse transfer: bilinear interpolation of the four
 *     surrounding lattice nodes (Secs. 5.1 and 6.2, item ii)
 *
 * Mesh: M x M squares of side h = Lside/M on [0, Lside]^2; node (k, l) at
 * (k h, l h) has index l*(M+1) + k.  Element (ex, ey) has local nodes
 * 0:(ex,ey) 1:(ex+1,ey) 2:(ex+1,ey+1) 3:(ex,ey+1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Upwind function of eq. (SUPG_tau): chi(a) = coth(a) - 1/a.  For small a
 * the two terms cancel, so below a = 0.1 the Laurent series of coth minus
 * 1/a is summed through a^9 (truncation < 7e-16 relative there):
 *   chi(a) = a/3 - a^3/45 + 2a^5/945 - a^7/4725 + 2a^9/93555 - ...          */
double orc_supg_chi(double a) {
    if (a < 0.1) {
        double a2 = a * a;
        return a * (1.0 / 3.0 + a2 * (-1.0 / 45.0 + a2 * (2.0 / 945.0 + a2 * (-1.0 / 4725.0 + a2 * (2.0 / 93555.0)))));
    }
    return 1.0 / tanh(a) - 1.0 / a;
}

/* Element matrices on one square element.  vn: nodal velocities [4][2] of
 * the element's local nodes (the velocity inside the element is their
 * bilinear interpolant).  Outputs (4x4, row a = test function N_a):
 *   Me = int N_a N_b,   Ke = int N_a v.grad N_b + D grad N_a . grad N_b + k N_a N_b
 *   Mse = int tau (v.grad N_a) N_b,   Kse = int tau (v.grad N_a)(v.grad N_b + k N_b)
 * using 2 x 2 Gauss quadrature.  tau is evaluated at each quadrature point
 * with h_e = h, p = 1 and |v| the local speed; tau = 0 where v = 0 or when
 * supg == 0.  The SUPG residual has no diffusion term because the
 * Laplacian of a bilinear function vanishes. */
void orc_fem_element(double h, double D, double k, int supg, const double *vn,
                     double *Me, double *Ke, double *Mse, double *Kse) {
    static const double XI[4] = {-1.0, 1.0, 1.0, -1.0};
    static const double ETA[4] = {-1.0, -1.0, 1.0, 1.0};
    double g = 1.0 / sqrt(3.0);
    double gp[2] = {-g, g};
    double detJ = (h / 2.0) * (h / 2.0);
    memset(Me, 0, 16 * sizeof(double));
    memset(Ke, 0, 16 * sizeof(double));
    memset(Mse, 0, 16 * sizeof(double));
    memset(Kse, 0, 16 * sizeof(double));
    for (int gi = 0; gi < 2; ++gi) {
        for (int gj = 0; gj < 2; ++gj) {
            double xi = gp[gi], eta = gp[gj];
            double N[4], dNx[4], dNy[4];
            for (int a = 0; a < 4; ++a) {
                N[a] = 0.25 * (1.0 + xi * XI[a]) * (1.0 + eta * ETA[a]);
                dNx[a] = 0.25 * XI[a] * (1.0 + eta * ETA[a]) * (2.0 / h);
                dNy[a] = 0.25 * (1.0 + xi * XI[a]) * ETA[a] * (2.0 / h);
            }
            double vx = 0.0, vy = 0.0;
            for (int a = 0; a < 4; ++a) {
                vx += N[a] * vn[2 * a];
                vy += N[a] * vn[2 * a + 1];
            }
            double tau = 0.0;
            double speed = sqrt(vx * vx + vy * vy);
            if (supg && speed > 0.0) {
                double Pe = speed * h / (2.0 * 1.0 * D);
                tau = h / (2.0 * 1.0 * speed) * orc_supg_chi(Pe);
            }
            for (int a = 0; a < 4; ++a) {
                double vga = vx * dNx[a] + vy * dNy[a];
                for (int b = 0; b < 4; ++b) {
                    double vgb = vx * dNx[b] + vy * dNy[b];
                    Me[4 * a + b] += N[a] * N[b] * detJ;
                    Ke[4 * a + b] += (N[a] * vgb + D * (dNx[a] * dNx[b] + dNy[a] * dNy[b]) +
                                      k * N[a] * N[b]) * detJ;
                    Mse[4 * a + b] += tau * vga * N[b] * detJ;
                    Kse[4 * a + b] += tau * vga * (vgb + k * N[b]) * detJ;
                }
            }
        }
    }
}

/* Global node indices of element (ex, ey). */
static void elem_nodes(int M, int ex, int ey, int *nd) {
    int s = M + 1;
    nd[0] = ey * s + ex;
    nd[1] = ey * s + ex + 1;
    nd[2] = (ey + 1) * s + ex + 1;
    nd[3] = (ey + 1) * s + ex;
}

/* ------------------------------------------------------------------------ */
/* Banded storage (LAPACK general-band layout, 0-based): for kl sub- and ku */
/* super-diagonals, A(i, j) lives at ab[j*ldab + kl + ku + i - j] with      */
/* ldab = 2 kl + ku + 1; the extra kl rows hold fill-in from pivoting.       */
/* ------------------------------------------------------------------------ */
#define AB(ab, ldab, kv, i, j) ((ab)[(size_t)(j) * (ldab) + (kv) + (i) - (j)])

/* Assemble the trapezoidal pair for time step dt:
 *   A = (M + Ms) + dt/2 (K + Ks),   B = (M + Ms) - dt/2 (K + Ks)
 * into band arrays a_band, b_band of size (M+1)^2 * ldab each (zeroed here),
 * with kl = ku = M + 2.  vnodes: [(M+1)^2][2] nodal velocity. */
void orc_fem_assemble(int M, double Lside, double D, double k, double dt, int supg,
                      const double *vnodes, double *a_band, double *b_band) {
    int n = (M + 1) * (M + 1);
    int kl = M + 2, ku = M + 2, ldab = 2 * kl + ku + 1, kv = kl + ku;
    double h = Lside / M;
    memset(a_band, 0, (size_t)n * ldab * sizeof(double));
    memset(b_band, 0, (size_t)n * ldab * sizeof(double));
    for (int ey = 0; ey < M; ++ey) {
        for (int ex = 0; ex < M; ++ex) {
            int nd[4];
            elem_nodes(M, ex, ey, nd);
            double vn[8];
            for (int a = 0; a < 4; ++a) {
                vn[2 * a] = vnodes[2 * nd[a]];
                vn[2 * a + 1] = vnodes[2 * nd[a] + 1];
            }
            double Me[16], Ke[16], Mse[16], Kse[16];
            orc_fem_element(h, D, k, supg, vn, Me, Ke, Mse, Kse);
            for (int a = 0; a < 4; ++a) {
                for (int b = 0; b < 4; ++b) {
                    double cap = Me[4 * a + b] + Mse[4 * a + b];
                    double tr = Ke[4 * a + b] + Kse[4 * a + b];
                    AB(a_band, ldab, kv, nd[a], nd[b]) += cap + 0.5 * dt * tr;
                    AB(b_band, ldab, kv, nd[a], nd[b]) += cap - 0.5 * dt * tr;
                }
            }
        }
    }
}

/* Replace the rows of the listed nodes by identity rows (strong Dirichlet). */
void orc_band_dirichlet_rows(int M, double *a_band, const int *rows, int nrows) {
    int n = (M + 1) * (M + 1);
    int kl = M + 2, ku = M + 2, ldab = 2 * kl + ku + 1, kv = kl + ku;
    for (int t = 0; t < nrows; ++t) {
        int r = rows[t];
        int j0 = r - ku < 0 ? 0 : r - ku;
        int j1 = r + ku > n - 1 ? n - 1 : r + ku;
        for (int j = j0; j <= j1; ++j) AB(a_band, ldab, kv, r, j) = 0.0;
        AB(a_band, ldab, kv, r, r) = 1.0;
    }
}

/* y = B x for a band matrix with kl = ku = M + 2 (no fill-in used). */
void orc_band_matvec(int M, const double *b_band, const double *x, double *y) {
    int n = (M + 1) * (M + 1);
    int kl = M + 2, ku = M + 2, ldab = 2 * kl + ku + 1, kv = kl + ku;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        int j0 = i - kl < 0 ? 0 : i - kl;
        int j1 = i + ku > n - 1 ? n - 1 : i + ku;
        for (int j = j0; j <= j1; ++j) s += AB(b_band, ldab, kv, i, j) * x[j];
        y[i] = s;
    }
}

/* Dense copy of a band matrix (for small-mesh tests). */
void orc_band_to_dense(int M, const double *band, double *dense) {
    int n = (M + 1) * (M + 1);
    int kl = M + 2, ku = M + 2, ldab = 2 * kl + ku + 1, kv = kl + ku;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            dense[(size_t)i * n + j] = (j - i <= ku && i - j <= kl) ? AB(band, ldab, kv, i, j) : 0.0;
}

/* Gaussian elimination with partial (row) pivoting on the band matrix, in
 * place: L multipliers below the diagonal, U (bandwidth kl + ku) above.
 * Returns 0, or j + 1 if a zero pivot was met in column j. */
int orc_band_lu(int M, double *ab, int *ipiv) {
    int n = (M + 1) * (M + 1);
    int kl = M + 2, ku = M + 2, ldab = 2 * kl + ku + 1, kv = kl + ku;
    int ju = 0;
    for (int j = 0; j < n; ++j) {
        int km = kl < n - 1 - j ? kl : n - 1 - j;
        int jp = 0;
        double best = fabs(AB(ab, ldab, kv, j, j));
        for (int t = 1; t <= km; ++t) {
            double v = fabs(AB(ab, ldab, kv, j + t, j));
            if (v > best) { best = v; jp = t; }
        }
        ipiv[j] = j + jp;
        if (best == 0.0) return j + 1;
        int lim = j + ku + jp < n - 1 ? j + ku + jp : n - 1;
        if (lim > ju) ju = lim;
        if (jp != 0) {
            for (int c = j; c <= ju; ++c) {
                double t = AB(ab, ldab, kv, j, c);
                AB(ab, ldab, kv, j, c) = AB(ab, ldab, kv, j + jp, c);
                AB(ab, ldab, kv, j + jp, c) = t;
            }
        }
        double piv = AB(ab, ldab, kv, j, j);
        for (int t = 1; t <= km; ++t) AB(ab, ldab, kv, j + t, j) /= piv;
        for (int c = j + 1; c <= ju; ++c) {
            double ujc = AB(ab, ldab, kv, j, c);
            if (ujc == 0.0) continue;
            for (int t = 1; t <= km; ++t) AB(ab, ldab, kv, j + t, c) -= AB(ab, ldab, kv, j + t, j) * ujc;
        }
    }
    return 0;
}

/* Solve A x = b with the factors from orc_band_lu; b is overwritten by x. */
void orc_band_solve(int M, const double *ab, const int *ipiv, double *b) {
    int n = (M + 1) * (M + 1);
    int kl = M + 2, ku = M + 2, ldab = 2 * kl + ku + 1, kv = kl + ku;
    for (int j = 0; j < n - 1; ++j) {
        int km = kl < n - 1 - j ? kl : n - 1 - j;
        int p = ipiv[j];
        if (p != j) { double t = b[j]; b[j] = b[p]; b[p] = t; }
        for (int t = 1; t <= km; ++t) b[j + t] -= AB(ab, ldab, kv, j + t, j) * b[j];
    }
    for (int j = n - 1; j >= 0; --j) {
        b[j] /= AB(ab, ldab, kv, j, j);
        int i0 = j - kv < 0 ? 0 : j - kv;
        for (int i = i0; i < j; ++i) b[i] -= AB(ab, ldab, kv, i, j) * b[j];
    }
}

/* ------------------------------------------------------------------------ */
/* Coarse-to-fine transfer (Sec. 6.2, item ii): the FEM interpolant of d at  */
/* point (X, Y), evaluated in the element that contains the point (element  */
/* index clamped to the mesh).                                              */
/* ------------------------------------------------------------------------ */
double orc_fem_interpolate(int M, double Lside, const double *d, double X, double Y) {
    double h = Lside / M;
    double sx = X / h, sy = Y / h;
    int ex = (int)floor(sx), ey = (int)floor(sy);
    if (ex < 0) ex = 0;
    if (ex > M - 1) ex = M - 1;
    if (ey < 0) ey = 0;
    if (ey > M - 1) ey = M - 1;
    double xi = sx - ex, et = sy - ey;
    int nd[4];
    elem_nodes(M, ex, ey, nd);
    return (1.0 - xi) * (1.0 - et) * d[nd[0]] + xi * (1.0 - et) * d[nd[1]] +
           xi * et * d[nd[2]] + (1.0 - xi) * et * d[nd[3]];
}

/* ------------------------------------------------------------------------ */
/* Fine-to-coarse transfer (Sec. 6.2, item ii): at a coarse node with        */
/* lattice coordinates (px, py) = (X - x0, Y - y0), take the lattice square */
/* with lower-left node (i0, j0) = floor(px, py) (clamped to N - 2) and     */
/*   u5 = u1 (1-gx)(1-gy) + u2 gx (1-gy) + u3 gx gy + u4 (1-gx) gy,          */
/* u1..u4 at (i0,j0), (i0+1,j0), (i0+1,j0+1), (i0,j0+1).  Solid corners     */
/* carry no concentration: the weights of the fluid corners are rescaled to */
/* sum to one, and when all four corners are solid the nearest fluid node   */
/* is used (ties broken by the lowest index j*N + i).                       */
/* ------------------------------------------------------------------------ */
static int nearest_fluid(int N, const uint8_t *solid, double px, double py) {
    int ci = (int)floor(px + 0.5), cj = (int)floor(py + 0.5);
    for (int r = 1; r <= 2 * N; ++r) {
        int best = -1;
        double bd = 0.0;
        int i0 = ci - r, i1 = ci + r, j0 = cj - r, j1 = cj + r;
        for (int j = j0 < 0 ? 0 : j0; j <= (j1 > N - 1 ? N - 1 : j1); ++j)
            for (int i = i0 < 0 ? 0 : i0; i <= (i1 > N - 1 ? N - 1 : i1); ++i) {
                if (solid[j * N + i]) continue;
                double d2 = (i - px) * (i - px) + (j - py) * (j - py);
                if (best < 0 || d2 < bd) { best = j * N + i; bd = d2; }
            }
        /* every node outside the searched square is farther than r - 0.5 */
        if (best >= 0 && sqrt(bd) <= r - 0.5) return best;
    }
    return -1;
}

double orc_fine_to_coarse(int N, const uint8_t *solid, const double *u, double px, double py) {
    int i0 = (int)floor(px), j0 = (int)floor(py);
    if (i0 < 0) i0 = 0;
    if (i0 > N - 2) i0 = N - 2;
    if (j0 < 0) j0 = 0;
    if (j0 > N - 2) j0 = N - 2;
    double gx = px - i0, gy = py - j0;
    int nd[4] = {j0 * N + i0, j0 * N + i0 + 1, (j0 + 1) * N + i0 + 1, (j0 + 1) * N + i0};
    double w[4] = {(1.0 - gx) * (1.0 - gy), gx * (1.0 - gy), gx * gy, (1.0 - gx) * gy};
    if (!solid) return w[0] * u[nd[0]] + w[1] * u[nd[1]] + w[2] * u[nd[2]] + w[3] * u[nd[3]];
    double wsum = 0.0, s = 0.0;
    for (int c = 0; c < 4; ++c)
        if (!solid[nd[c]]) { wsum += w[c]; s += w[c] * u[nd[c]]; }
    if (wsum > 0.0) return s / wsum;
    int nf = nearest_fluid(N, solid, px, py);
    return nf >= 0 ? u[nf] : 0.0;
}
