/*
 * CPU FP64 oracle for the hybrid FEM/LBM transport method of Karimi and
 * Nakshatrala (arXiv:1601.02708).  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path may link, load or call this file; only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Plain, slow and literal: each part of the method is a separate loop over
 * the lattice or the mesh, written in the order the paper states it.  No
 * SIMD, no blocking, no fusion.  Build: gcc -O2 -ffp-contract=off -fopenmp.
 * The loops whose nodes are independent (streaming, collision, readout,
 * initialisation) are split over rows between OpenMP threads; every node is
 * still computed by one thread with the same operations in the same order,
 * so the results do not depend on the thread count.  Loops that sum over
 * nodes or scatter into shared entries stay serial.
 *
 * Lattice-unit conventions: fine spacing 1, fine step 1; node (i, j) of an
 * N x N lattice is stored at n = j*N + i; populations are planes [9][N*N].
 * The stored state between sub-steps is the POST-collision population f*.
 *
 * Parts and the passages they follow:
 *   - D2Q9 velocities and weights with c_s^2 = 1/3            (Sec. 4.1)
 *   - equilibrium, eq. (LBM_feq), with the quadratic term read as
 *     -v.v/(2 c_s^2) (the printed -v.v/c_s^2 would not conserve mass)
 *   - BGK collision, eqs. (LBE) and (Collision); first-order reaction
 *     source -k w_i u added to the collision (not in the paper's LBM)
 *   - macroscopic moments, eq. (LBM_Macro)
 *   - maximum-entropy Dirichlet closure, eq. (LBM_Dir), and Neumann
 *     closure, eq. (LBM_Neu)                                   (Sec. 4.1.1)
 *   - Q1 finite elements, Galerkin eq. (Galerkin) and SUPG eqs. (SUPG),
 *     (SUPG_tau), trapezoidal time stepping eq. (FEM_discrete)  (Secs. 3, 6.1)
 *   - coarse-to-fine and fine-to-coarse transfers               (Secs. 5.1, 6.2)
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* D2Q9 lattice (Sec. 4.1): rest, 4 axis, 4 diagonal velocities.            */
/* ------------------------------------------------------------------------ */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0;

void orc_d2q9(int *ex, int *ey, double *w, int *opp) {
    for (int i = 0; i < 9; ++i) {
        ex[i] = EX[i];
        ey[i] = EY[i];
        w[i] = WT[i];
        opp[i] = OPP[i];
    }
}

/* Threads used by the row-parallel loops (n >= 1; the default is OpenMP's,
 * OMP_NUM_THREADS when set). */
void orc_set_threads(int n) {
    if (n >= 1) omp_set_num_threads(n);
}
int orc_get_threads(void) { return omp_get_max_threads(); }

/* Equilibrium, eq. (LBM_feq):
 *   f_i^eq = w_i u (1 + e.v/c_s^2 + (e.v)^2/(2 c_s^4) - v.v/(2 c_s^2)). */
void orc_feq(double u, double vx, double vy, double *feq) {
    double vv = vx * vx + vy * vy;
    for (int i = 0; i < 9; ++i) {
        double ev = EX[i] * vx + EY[i] * vy;
        feq[i] = WT[i] * u * (1.0 + ev / CS2 + (ev * ev) / (2.0 * CS2 * CS2) - vv / (2.0 * CS2));
    }
}

/* ------------------------------------------------------------------------ */
/* Lattice description                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int N;                       /* nodes per side */
    int periodic_x, periodic_y;  /* 1: sources beyond that edge wrap (test mode) */
    double tau;                  /* BGK relaxation time */
    const uint8_t *solid;        /* [N*N] 1 = solid node, or NULL */
    const double *vx, *vy;       /* [N*N] advection velocity */
    const double *k;             /* [N*N] reaction rate per node, or NULL */
    double kval;                 /* uniform reaction rate when k == NULL */
    const int8_t *bc_kind;       /* [4(N-1)] 0 Dirichlet, 1 Neumann, or NULL (all Dirichlet) */
    int clamp;                   /* Dirichlet closure: 0 as printed, 1 clamp unknowns at 0 */
    double kappa_s;              /* surface reaction at fluid-solid links (0: plain bounce-back) */
    double c_sat;                /* concentration the surface reaction drives towards */
    double *work_f;              /* [9*N*N] scratch of orc_lbm_substep, or NULL (allocated per call) */
    uint16_t *work_unknown;      /* [N*N] scratch of orc_lbm_substep, or NULL */
    const double *wall_nx;       /* [N*N] unit outward normal of the fluid domain at solid walls */
    const double *wall_ny;       /*   (towards the solid), or NULL: halfway bounce-back at walls */
} orc_lattice;

static int is_solid(const orc_lattice *L, int n) { return L->solid && L->solid[n]; }
static double kat(const orc_lattice *L, int n) { return L->k ? L->k[n] : L->kval; }

/* Perimeter slot of node (i, j), or -1 for interior nodes.  Slots run along
 * the bottom row (j = 0, i = 0..N-1), the top row (j = N-1, i = 0..N-1), the
 * left column (i = 0, j = 1..N-2) and the right column (i = N-1, j = 1..N-2). */
int orc_perimeter_slot(int N, int i, int j) {
    if (j == 0) return i;
    if (j == N - 1) return N + i;
    if (i == 0) return 2 * N + (j - 1);
    if (i == N - 1) return 2 * N + (N - 2) + (j - 1);
    return -1;
}

void orc_perimeter_node(int N, int p, int *i, int *j) {
    if (p < N) { *i = p; *j = 0; return; }
    if (p < 2 * N) { *i = p - N; *j = N - 1; return; }
    if (p < 3 * N - 2) { *i = 0; *j = p - 2 * N + 1; return; }
    *i = N - 1; *j = p - (3 * N - 2) + 1;
}

/* Outward normal direction (unnormalised, components in {-1,0,1}) of a
 * perimeter node; corners take the sum of their two edges' normals. */
static void outward_dir(int N, int i, int j, int *sx, int *sy) {
    *sx = (i == 0) ? -1 : (i == N - 1) ? 1 : 0;
    *sy = (j == 0) ? -1 : (j == N - 1) ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Initialisation (Sec. 6.2, item i): f_i(x, 0) = f_i^eq(u_0(x)); the stored  */
/* state is the post-collision value of that field.                         */
/* ------------------------------------------------------------------------ */
void orc_collide(const orc_lattice *L, const double *f, double *fstar);

void orc_lbm_init(const orc_lattice *L, const double *u0, double *fstar) {
    int N = L->N;
    size_t NN = (size_t)N * N;
    double *f = (double *)calloc(9 * NN, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int n = 0; n < (int)NN; ++n) {
        if (is_solid(L, n)) continue;
        double feq[9];
        orc_feq(u0[n], L->vx[n], L->vy[n], feq);
        for (int i = 0; i < 9; ++i) f[i * NN + n] = feq[i];
    }
    orc_collide(L, f, fstar);
    free(f);
}

/* ------------------------------------------------------------------------ */
/* Streaming, eq. (LBE), written as a pull: the population arriving at x     */
/* along e_i left x - e_i one step earlier.  A source that is a solid node   */
/* returns the population that x itself sent towards it (halfway bounce-    */
/* back); with a surface reaction of rate kappa_s at that link, the         */
/* returned population relaxes towards w_i c_sat:                           */
/*   f_i(x) = (1 - kappa_s) f*_opp(i)(x) + kappa_s w_i c_sat                */
/* (the link adds kappa_s (w_i c_sat - f*_opp(i)(x)) to the fluid).  A      */
/* source outside the patch (non-periodic edge) leaves f_i unknown and      */
/* flags it in unknown[n] (bit i).                                          */
/* ------------------------------------------------------------------------ */
void orc_stream(const orc_lattice *L, const double *fstar, double *f, uint16_t *unknown) {
    int N = L->N;
    size_t NN = (size_t)N * N;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < N; ++j) {
        for (int i = 0; i < N; ++i) {
            int n = j * N + i;
            unknown[n] = 0;
            if (is_solid(L, n)) {
                for (int q = 0; q < 9; ++q) f[q * NN + n] = 0.0;
                continue;
            }
            for (int q = 0; q < 9; ++q) {
                int si = i - EX[q], sj = j - EY[q];
                int outside = 0;
                if (si < 0 || si >= N) {
                    if (L->periodic_x) si = (si + N) % N; else outside = 1;
                }
                if (sj < 0 || sj >= N) {
                    if (L->periodic_y) sj = (sj + N) % N; else outside = 1;
                }
                if (outside) {
                    f[q * NN + n] = 0.0;
                    unknown[n] |= (uint16_t)(1u << q);
                    continue;
                }
                int s = sj * N + si;
                if (is_solid(L, s))
                    f[q * NN + n] = L->kappa_s == 0.0 ? fstar[OPP[q] * NN + n]
                                                      : (1.0 - L->kappa_s) * fstar[OPP[q] * NN + n] +
                                                            L->kappa_s * WT[q] * L->c_sat;
                else
                    f[q * NN + n] = fstar[q * NN + s];
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Maximum-entropy Dirichlet closure, eq. (LBM_Dir):                         */
/*   f_i = w_i / (sum_{j in U} w_j) * (u^p - sum_{k not in U} f_k),  i in U, */
/* the minimiser of H over the unknowns under sum_i f_i = u^p.  The result  */
/* is non-negative only when the bracket R is >= 0.  When R < 0 no          */
/* non-negative closure meets the constraint; the node is counted (return  */
/* 1) and, with clamp == 0, the closed form is applied as printed (the      */
/* constraint holds exactly, the unknowns are negative); with clamp != 0    */
/* the unknowns are set to 0 instead (non-negativity kept, constraint       */
/* missed).                                                                 */
/* ------------------------------------------------------------------------ */
int orc_maxent_dirichlet(double *f, unsigned unknown, double up, int clamp) {
    double known = 0.0, wsum = 0.0;
    for (int q = 0; q < 9; ++q) {
        if (unknown & (1u << q)) wsum += WT[q];
        else known += f[q];
    }
    double R = up - known;
    int infeasible = R < 0.0;
    if (infeasible && clamp) R = 0.0;
    for (int q = 0; q < 9; ++q) if (unknown & (1u << q)) f[q] = WT[q] / wsum * R;
    return infeasible;
}

/* ------------------------------------------------------------------------ */
/* Maximum-entropy Neumann closure, eq. (LBM_Neu).  With n the unit outward  */
/* normal and M- = {i unknown : e_i.n < 0}, the unknowns are                */
/*   f_i = w_i exp(-1 - gamma e_i.n),                                       */
/* where gamma solves                                                       */
/*   sum_{i in M-} w_i (e_i.n) exp(-1 - gamma e_i.n)                        */
/*        = q^p - sum_{j not in M-} (e_j.n) f_j .                           */
/* The left side is negative and strictly decreasing in gamma, so a root   */
/* exists iff the right side is negative; it is found by bisection.  At a   */
/* patch corner (diagonal normal) two unknowns have e_i.n = 0; they carry   */
/* no flux and are set by bounce-back from the node's own post-collision    */
/* populations.  Returns 1 when infeasible (unknowns of M- set to 0).       */
/* ------------------------------------------------------------------------ */
static double neumann_lhs(const double *a, unsigned set, double gamma) {
    double s = 0.0;
    for (int q = 0; q < 9; ++q)
        if (set & (1u << q)) s += WT[q] * a[q] * exp(-1.0 - gamma * a[q]);
    return s;
}

/* The same closure for any unit outward normal (nx, ny): unknowns with
 * e_i.n < 0 are the maxent unknowns, the other unknowns (e_i.n >= 0, e.g.
 * the tangential ones at a corner or where a curved wall grazes a link)
 * are bounced back from the node's own post-collision populations. */
int orc_maxent_neumann_normal(double *f, unsigned unknown, double nx, double ny, double qp,
                              const double *fstar_self) {
    double a[9];
    unsigned mminus = 0;
    for (int q = 0; q < 9; ++q) {
        a[q] = EX[q] * nx + EY[q] * ny;
        if (unknown & (1u << q)) {
            if (a[q] < 0.0) mminus |= 1u << q;
            else f[q] = fstar_self[OPP[q]];
        }
    }
    double rhs = qp;
    for (int q = 0; q < 9; ++q)
        if (!(mminus & (1u << q))) rhs -= a[q] * f[q];
    /* no population of M- to solve with: infeasible unless already met */
    if (!mminus) return rhs != 0.0;
    if (!(rhs < 0.0)) {
        for (int q = 0; q < 9; ++q) if (mminus & (1u << q)) f[q] = 0.0;
        return 1;
    }
    /* bracket: lhs(lo) > rhs > lhs(hi) */
    double lo = -1.0, hi = 1.0;
    while (neumann_lhs(a, mminus, lo) <= rhs) lo *= 2.0;
    while (neumann_lhs(a, mminus, hi) >= rhs) hi *= 2.0;
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (neumann_lhs(a, mminus, mid) > rhs) lo = mid; else hi = mid;
    }
    double gamma = 0.5 * (lo + hi);
    for (int q = 0; q < 9; ++q)
        if (mminus & (1u << q)) f[q] = WT[q] * exp(-1.0 - gamma * a[q]);
    return 0;
}

/* Patch-edge form: outward direction (sx, sy), components in {-1, 0, 1}. */
int orc_maxent_neumann(double *f, unsigned unknown, int sx, int sy, double qp,
                       const double *fstar_self) {
    double nrm = sqrt((double)(sx * sx + sy * sy));
    return orc_maxent_neumann_normal(f, unknown, sx / nrm, sy / nrm, qp, fstar_self);
}

/* Maximum-entropy Neumann closure at solid walls, eq. (LBM_Neu) with
 * q^p = 0 (an impermeable wall), in place of halfway bounce-back: every
 * interior fluid node (1 <= i, j <= N-2) with a solid upstream node is a
 * boundary point with the wall's unit outward normal (wall_nx, wall_ny).
 * Its unknowns are the set M- of the paper, all populations with
 * e_i.n < 0, whether their upstream node is solid or fluid; populations
 * streamed from a solid node with e_i.n >= 0 (links the wall grazes) are
 * bounced back.  Runs after streaming, which left the bounce-back values
 * in f.  Returns the number of infeasible nodes. */
long orc_apply_wall_closure(const orc_lattice *L, const double *fstar, double *f) {
    int N = L->N;
    size_t NN = (size_t)N * N;
    long infeasible = 0;
    if (!L->wall_nx || !L->wall_ny || !L->solid) return 0;
    for (int j = 1; j < N - 1; ++j) {
        for (int i = 1; i < N - 1; ++i) {
            int n = j * N + i;
            if (is_solid(L, n)) continue;
            unsigned unknown = 0;
            for (int q = 1; q < 9; ++q)
                if (is_solid(L, (j - EY[q]) * N + (i - EX[q]))) unknown |= 1u << q;
            if (!unknown) continue;
            for (int q = 1; q < 9; ++q)
                if (EX[q] * L->wall_nx[n] + EY[q] * L->wall_ny[n] < 0.0) unknown |= 1u << q;
            double fn[9], fs[9];
            for (int q = 0; q < 9; ++q) {
                fn[q] = f[q * NN + n];
                fs[q] = fstar[q * NN + n];
            }
            infeasible += orc_maxent_neumann_normal(fn, unknown, L->wall_nx[n], L->wall_ny[n], 0.0, fs);
            for (int q = 0; q < 9; ++q) f[q * NN + n] = fn[q];
        }
    }
    return infeasible;
}

/* Apply the boundary closures at every perimeter node that has unknowns.
 * bc_value[p] is u^p (Dirichlet) or q^p (Neumann) for perimeter slot p.
 * Returns the number of infeasible nodes. */
long orc_apply_bc(const orc_lattice *L, const double *fstar, double *f,
                  const uint16_t *unknown, const double *bc_value) {
    int N = L->N;
    size_t NN = (size_t)N * N;
    long infeasible = 0;
    for (int p = 0; p < 4 * (N - 1); ++p) {
        int i, j;
        orc_perimeter_node(N, p, &i, &j);
        int n = j * N + i;
        if (is_solid(L, n) || unknown[n] == 0) continue;
        double fn[9], fs[9];
        for (int q = 0; q < 9; ++q) {
            fn[q] = f[q * NN + n];
            fs[q] = fstar[q * NN + n];
        }
        int kind = L->bc_kind ? L->bc_kind[p] : 0;
        if (kind == 0) {
            infeasible += orc_maxent_dirichlet(fn, unknown[n], bc_value[p], L->clamp);
        } else {
            int sx, sy;
            outward_dir(N, i, j, &sx, &sy);
            infeasible += orc_maxent_neumann(fn, unknown[n], sx, sy, bc_value[p], fs);
        }
        for (int q = 0; q < 9; ++q) f[q * NN + n] = fn[q];
    }
    return infeasible;
}

/* ------------------------------------------------------------------------ */
/* Collision, eq. (Collision), with u from eq. (LBM_Macro) and a first-order */
/* reaction source:  f*_i = f_i + (f_i^eq(u) - f_i)/tau - k w_i u.          */
/* ------------------------------------------------------------------------ */
void orc_collide(const orc_lattice *L, const double *f, double *fstar) {
    int N = L->N;
    size_t NN = (size_t)N * N;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < (int)NN; ++n) {
        if (is_solid(L, n)) {
            for (int q = 0; q < 9; ++q) fstar[q * NN + n] = 0.0;
            continue;
        }
        double u = 0.0;
        for (int q = 0; q < 9; ++q) u += f[q * NN + n];
        double feq[9];
        orc_feq(u, L->vx[n], L->vy[n], feq);
        double k = kat(L, n);
        for (int q = 0; q < 9; ++q) {
            double fq = f[q * NN + n];
            fstar[q * NN + n] = fq + (feq[q] - fq) / L->tau - k * WT[q] * u;
        }
    }
}

/* One fine time step: stream, impose the boundary closures, collide.
 * fdst may not alias fsrc.  Returns the infeasible-node count. */
long orc_lbm_substep(const orc_lattice *L, const double *fsrc, double *fdst, const double *bc_value) {
    int N = L->N;
    size_t NN = (size_t)N * N;
    double *f = L->work_f ? L->work_f : (double *)malloc(9 * NN * sizeof(double));
    uint16_t *unknown = L->work_unknown ? L->work_unknown : (uint16_t *)malloc(NN * sizeof(uint16_t));
    orc_stream(L, fsrc, f, unknown);
    long inf = orc_apply_wall_closure(L, fsrc, f);
    inf += orc_apply_bc(L, fsrc, f, unknown, bc_value);
    orc_collide(L, f, fdst);
    if (!L->work_f) free(f);
    if (!L->work_unknown) free(unknown);
    return inf;
}

/* Concentration at every node from the stored post-collision populations.
 * Summing the collision over i gives  sum f*_i = (1 - k) u,  so
 * u = sum_i f*_i / (1 - k); solid nodes return 0. */
void orc_concentration(const orc_lattice *L, const double *fstar, double *u) {
    int N = L->N;
    size_t NN = (size_t)N * N;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < (int)NN; ++n) {
        if (is_solid(L, n)) { u[n] = 0.0; continue; }
        double s = 0.0;
        for (int q = 0; q < 9; ++q) s += fstar[q * NN + n];
        u[n] = s / (1.0 - kat(L, n));
    }
}

/* Boltzmann H function, eq. (BH), summed over fluid nodes. */
double orc_h_function(const orc_lattice *L, const double *f) {
    int N = L->N;
    size_t NN = (size_t)N * N;
    double H = 0.0;
    for (int n = 0; n < (int)NN; ++n) {
        if (is_solid(L, n)) continue;
        for (int q = 0; q < 9; ++q) {
            double v = f[q * NN + n];
            if (v > 0.0) H += v * log(v / WT[q]);
        }
    }
    return H;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of one fine step (reverse mode of orc_lbm_substep), for the      */
/* differentiation form: given lam_in = dJ/df*(t+1), returns                 */
/* lam_out = dJ/df*(t) and accumulates dJ/du^p (per perimeter slot) and     */
/* dJ/dk (per node).  Written as the transpose of each forward pass, in     */
/* reverse order:                                                           */
/*   collision  f*_i = (1 - 1/tau) f_i + f_i^eq(u)/tau - k w_i u, u = sum f: */
/*     dJ/df_j = (1 - 1/tau) l_j + sum_i l_i (f_i^eq(1)/tau - k w_i),       */
/*     dJ/dk  -= u sum_i w_i l_i   (f^eq is linear in u);                   */
/*   Dirichlet closure f_U = w_U (u^p - sum_K f_K) / W (eq. LBM_Dir):        */
/*     G = sum_U w_U dJ/df_U / W;  dJ/df_K -= G;  dJ/du^p += G;  when the   */
/*     closure is clamped at zero (clamp != 0 and R < 0) the unknowns are   */
/*     constant and G = 0;                                                  */
/*   streaming (pull, halfway bounce-back): each dJ/df_i(x) goes back to the */
/*     population it was copied from (times 1 - kappa_s across a reactive   */
/*     link).                                                                */
/* The forward pre-collision field and every closure's R are recomputed    */
/* from fsrc.  Neumann slots are not supported (returns -1).                */
/* ------------------------------------------------------------------------ */
int orc_lbm_adjoint_substep(const orc_lattice *L, const double *fsrc, const double *bc_value,
                            const double *lam_in, double *lam_out, double *grad_bc, double *grad_k) {
    int N = L->N;
    size_t NN = (size_t)N * N;
    if (L->wall_nx) return -1;
    if (L->bc_kind)
        for (int p = 0; p < 4 * (N - 1); ++p)
            if (L->bc_kind[p] != 0) return -1;
    double *f = (double *)malloc(9 * NN * sizeof(double));
    double *lf = (double *)calloc(9 * NN, sizeof(double));
    uint16_t *unknown = (uint16_t *)malloc(NN * sizeof(uint16_t));
    /* forward pre-collision field (streamed, closed) */
    orc_stream(L, fsrc, f, unknown);
    double *fs = (double *)malloc(9 * NN * sizeof(double));
    memcpy(fs, f, 9 * NN * sizeof(double));          /* streamed, before the closure */
    orc_apply_bc(L, fsrc, f, unknown, bc_value);

    /* collision */
    for (int n = 0; n < (int)NN; ++n) {
        if (is_solid(L, n)) continue;
        double u = 0.0, feq1[9], s = 0.0, wl = 0.0;
        for (int q = 0; q < 9; ++q) u += f[q * NN + n];
        orc_feq(1.0, L->vx[n], L->vy[n], feq1);
        double k = kat(L, n);
        for (int i = 0; i < 9; ++i) {
            double li = lam_in[i * NN + n];
            s += li * (feq1[i] / L->tau - k * WT[i]);
            wl += WT[i] * li;
        }
        for (int j = 0; j < 9; ++j) lf[j * NN + n] = (1.0 - 1.0 / L->tau) * lam_in[j * NN + n] + s;
        if (grad_k) grad_k[n] -= u * wl;
    }
    /* Dirichlet closure */
    for (int p = 0; p < 4 * (N - 1); ++p) {
        int i, j;
        orc_perimeter_node(N, p, &i, &j);
        int n = j * N + i;
        if (is_solid(L, n) || unknown[n] == 0) continue;
        double known = 0.0, wsum = 0.0, g = 0.0;
        for (int q = 0; q < 9; ++q) {
            if (unknown[n] & (1u << q)) wsum += WT[q];
            else known += fs[q * NN + n];
        }
        int clamped = L->clamp && (bc_value[p] - known < 0.0);
        if (!clamped) {
            for (int q = 0; q < 9; ++q)
                if (unknown[n] & (1u << q)) g += WT[q] * lf[q * NN + n];
            g /= wsum;
            for (int q = 0; q < 9; ++q)
                if (!(unknown[n] & (1u << q))) lf[q * NN + n] -= g;
            if (grad_bc) grad_bc[p] += g;
        }
        for (int q = 0; q < 9; ++q)
            if (unknown[n] & (1u << q)) lf[q * NN + n] = 0.0;
    }
    /* streaming */
    memset(lam_out, 0, 9 * NN * sizeof(double));
    for (int j = 0; j < N; ++j) {
        for (int i = 0; i < N; ++i) {
            int n = j * N + i;
            if (is_solid(L, n)) continue;
            for (int q = 0; q < 9; ++q) {
                if (unknown[n] & (1u << q)) continue;
                int si = i - EX[q], sj = j - EY[q];
                if (si < 0 || si >= N) si = (si + N) % N;    /* only reached when periodic */
                if (sj < 0 || sj >= N) sj = (sj + N) % N;
                int s = sj * N + si;
                if (is_solid(L, s)) lam_out[OPP[q] * NN + n] += (1.0 - L->kappa_s) * lf[q * NN + n];
                else lam_out[q * NN + s] += lf[q * NN + n];
            }
        }
    }
    free(fs);
    free(f);
    free(lf);
    free(unknown);
    return 0;
}
