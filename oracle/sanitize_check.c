/*
 * Host sanitizer run of the CPU oracle (test infrastructure).  Built by
 * tests/test_oracle_sanitizers.py with gcc's AddressSanitizer and
 * UndefinedBehaviorSanitizer; includes the two oracle sources whole so the
 * driver uses their own definitions, and drives every entry point on small
 * problems with solids, Neumann slots, wall normals, periodic and
 * non-periodic edges, the reverse mode, the FEM assembly, the banded solve
 * and both transfers.  Exits 0 when every call returned; the sanitizers
 * abort on an invalid access or undefined operation.
 */
#include "lbm_oracle.c"
#include "fem_oracle.c"

#include <stdio.h>

static double frand(unsigned *s) {
    *s = *s * 1664525u + 1013904223u;
    return (*s >> 8) * (1.0 / 16777216.0);
}

int main(void) {
    unsigned seed = 12345u;
    for (int N = 3; N <= 21; N += 9) {
        size_t NN = (size_t)N * N;
        uint8_t *solid = calloc(NN, 1);
        double *vx = malloc(NN * 8), *vy = malloc(NN * 8), *k = malloc(NN * 8), *u0 = malloc(NN * 8);
        double *nx = calloc(NN, 8), *ny = calloc(NN, 8);
        int8_t *kind = malloc(4 * (N - 1));
        for (size_t n = 0; n < NN; ++n) {
            vx[n] = 0.05 * (frand(&seed) - 0.5);
            vy[n] = 0.05 * (frand(&seed) - 0.5);
            k[n] = 1e-3 * frand(&seed);
            u0[n] = 0.2 + frand(&seed);
        }
        if (N > 6) {      /* a solid block inside, wall normals around it */
            for (int j = N / 2 - 1; j <= N / 2 + 1; ++j)
                for (int i = N / 2 - 1; i <= N / 2 + 1; ++i) solid[j * N + i] = 1;
            for (int j = 1; j < N - 1; ++j)
                for (int i = 1; i < N - 1; ++i) {
                    double dx = N / 2 - i, dy = N / 2 - j, r = sqrt(dx * dx + dy * dy);
                    if (r > 0) { nx[j * N + i] = dx / r; ny[j * N + i] = dy / r; }
                }
        }
        for (int p = 0; p < 4 * (N - 1); ++p) kind[p] = (int8_t)(p % 3 == 0);
        double *work = malloc(9 * NN * 8);
        uint16_t *unk = malloc(NN * 2);
        for (int variant = 0; variant < 4; ++variant) {
            orc_lattice L = {N, variant == 3, variant == 3, 0.6, solid, vx, vy, variant ? k : NULL, 1e-3,
                             variant == 1 ? kind : NULL, variant == 2, variant == 2 ? 0.1 : 0.0, 1.0,
                             variant == 0 ? NULL : work, variant == 0 ? NULL : unk,
                             variant == 1 ? nx : NULL, variant == 1 ? ny : NULL};
            double *fa = malloc(9 * NN * 8), *fb = malloc(9 * NN * 8), *u = malloc(NN * 8);
            double *bc = malloc(4 * (N - 1) * 8);
            for (int p = 0; p < 4 * (N - 1); ++p) bc[p] = (kind[p] && variant == 1) ? -0.01 : frand(&seed);
            orc_lbm_init(&L, u0, fa);
            for (int step = 0; step < 3; ++step) {
                orc_lbm_substep(&L, fa, fb, bc);
                orc_lbm_substep(&L, fb, fa, bc);
            }
            orc_concentration(&L, fa, u);
            volatile double h = orc_h_function(&L, fa);
            (void)h;
            if (variant != 1) {
                double *lin = malloc(9 * NN * 8), *lout = malloc(9 * NN * 8), *gbc = calloc(4 * (N - 1), 8);
                double *gk = calloc(NN, 8);
                for (size_t n = 0; n < 9 * NN; ++n) lin[n] = frand(&seed) - 0.5;
                if (orc_lbm_adjoint_substep(&L, fa, bc, lin, lout, gbc, gk) != 0) return 2;
                free(lin); free(lout); free(gbc); free(gk);
            }
            free(fa); free(fb); free(u); free(bc);
        }
        free(work); free(unk); free(solid); free(vx); free(vy); free(k); free(u0); free(nx); free(ny); free(kind);
    }
    /* single-node closures, edge and curved normals, infeasible cases */
    for (int t = 0; t < 64; ++t) {
        double f[9], fs[9];
        for (int q = 0; q < 9; ++q) { f[q] = frand(&seed); fs[q] = frand(&seed); }
        unsigned unknown = 1u + (unsigned)(frand(&seed) * 510.0);
        orc_maxent_dirichlet(f, unknown & 0x1FEu, frand(&seed) - 0.3, t & 1);
        double a = 6.283185307179586 * frand(&seed);
        orc_maxent_neumann_normal(f, unknown & 0x1FEu, cos(a), sin(a), frand(&seed) - 0.5, fs);
        orc_maxent_neumann(f, 0x122u, -1, 0, -0.02, fs);
    }
    /* FEM: assembly, Dirichlet rows, banded LU and solve, interpolation, transfer */
    for (int M = 2; M <= 6; M += 4) {
        int n = (M + 1) * (M + 1), ldab = 2 * (M + 2) + (M + 2) + 1;
        double *vn = malloc((size_t)n * 2 * 8), *A = calloc((size_t)n * ldab, 8), *B = calloc((size_t)n * ldab, 8);
        double *x = malloc((size_t)n * 8), *y = malloc((size_t)n * 8);
        int *ipiv = malloc((size_t)n * 4), rows[4] = {0, M, n - 1 - M, n - 1};
        for (int i = 0; i < 2 * n; ++i) vn[i] = 0.1 * (frand(&seed) - 0.5);
        for (int i = 0; i < n; ++i) x[i] = frand(&seed);
        orc_fem_assemble(M, 10.0, 0.02, 1e-3, 2.0, 1, vn, A, B);
        orc_band_dirichlet_rows(M, A, rows, 4);
        orc_band_matvec(M, B, x, y);
        if (orc_band_lu(M, A, ipiv) != 0) return 3;
        orc_band_solve(M, A, ipiv, y);
        volatile double s = orc_fem_interpolate(M, 10.0, y, 3.3, 10.0) + orc_supg_chi(1e-5) + orc_supg_chi(3.0);
        (void)s;
        free(vn); free(A); free(B); free(x); free(y); free(ipiv);
    }
    {
        int N = 12;
        uint8_t solid[144] = {0};
        double u[144];
        for (int i = 0; i < 144; ++i) { u[i] = frand(&seed); solid[i] = (i % 7 == 3); }
        volatile double v = orc_fine_to_coarse(N, solid, u, 4.3, 7.9) + orc_fine_to_coarse(N, solid, u, 11.0, 11.0) +
                            orc_fine_to_coarse(N, NULL, u, 0.0, 5.5);
        (void)v;
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
