"""Algorithm 1 (hybrid multi-time-step coupling, Sec. 6.2) written out on
top of the oracle's C pieces.  TEST INFRASTRUCTURE ONLY.

Readings of the algorithm taken here (where the paper leaves room):

* Each coarse step runs exactly ``max_iter`` Schwarz iterations and each
  iteration exactly ``eta`` fine steps; fine step j of the coarse step
  [t_n, t_n + eta] reaches time t_n + j and receives the interface value of
  eq. (MTS), (1 - j/eta) a + (j/eta) b, where a and b are the coarse
  solution at t_n and t_n + eta interpolated at the interface node.
* Every Schwarz iteration restarts both subdomains from their state at t_n;
  only the last iteration is kept.
* The fine-to-coarse data of the first iteration come from the fine state
  at t_n; later iterations use the fine result of the previous iteration.
* The coarse subdomain is the whole square [0, L]^2 with Dirichlet data on
  its outer edges; its interface Gamma_{f->c} is the set of coarse nodes
  inside the fine patch at least ``overlap_elems`` elements away from the
  patch boundary.  The fine interface Gamma_{c->f} is the whole perimeter
  of the lattice patch.
"""
from __future__ import annotations

import numpy as np

from . import FemStepper, Lattice, fem_interpolate, fine_to_coarse, perimeter_nodes, relaxation_time


def coarse_dirichlet_sets(M, L, N, x0, y0, overlap_elems=1, outer_natural=0):
    """(outer_nodes, interface_nodes): the Dirichlet nodes of the outer edges
    (edge e = 0: x = 0, 1: x = L, 2: y = 0, 3: y = L; edges whose bit is set
    in outer_natural keep the natural condition of the weak form), and the
    coarse nodes that take Dirichlet data from the lattice (Gamma_{f->c})."""
    h = L / M
    s = M + 1
    kk, ll = np.meshgrid(np.arange(s), np.arange(s), indexing="xy")
    idx = ll * s + kk
    edge = (kk == 0) | (kk == M) | (ll == 0) | (ll == M)
    outer = (((kk == 0) & (outer_natural & 1 == 0)) | ((kk == M) & (outer_natural & 2 == 0)) |
             ((ll == 0) & (outer_natural & 4 == 0)) | ((ll == M) & (outer_natural & 8 == 0)))
    X, Y = kk * h, ll * h
    ov = overlap_elems * h
    tol = 1e-9 * h
    x1, y1 = x0 + (N - 1), y0 + (N - 1)
    inner = ((X - x0 >= ov - tol) & (x1 - X >= ov - tol) &
             (Y - y0 >= ov - tol) & (y1 - Y >= ov - tol))
    inner &= ~edge
    return np.sort(idx[outer]), np.sort(idx[inner])


def algorithm1_step(h):
    """One coarse step of Algorithm 1 on a two-subdomain hybrid ``h`` (any
    dimension): h.fstar and h.d hold the fine and coarse states at t_n;
    h.fine_to_coarse, h.coarse_to_fine, h.coarse_step and h.lbm_substeps are
    the transfers and the two solvers; h.max_iter Schwarz iterations, each
    restarting both subdomains from t_n, the last one committed."""
    ufc = h.fine_to_coarse(h.fstar)
    a = h.coarse_to_fine(h.d)
    for _ in range(h.max_iter):
        d1 = h.coarse_step(h.d, ufc)
        b = h.coarse_to_fine(d1)
        F = h.lbm_substeps(h.fstar, a, b)
        ufc = h.fine_to_coarse(F)
    h.fstar = F
    h.d = d1


class HybridOracle:
    """State and steps of the two-subdomain hybrid method on the host."""

    def __init__(self, problem, tau=None, eta=None, max_iter=None, outer_value=None, outer_natural=None,
                 wall_normals=None):
        cfg = problem.cfg
        self.p = problem
        self.N, self.M, self.L = cfg.N, cfg.M, problem.L
        self.eta = cfg.eta if eta is None else eta
        self.max_iter = cfg.max_iter if max_iter is None else max_iter
        self.k = cfg.k
        tau = relaxation_time(cfg.D, cfg.tau if tau is None else tau)
        # outer edges and values as the workload states them unless given
        outer_value = cfg.outer_value if outer_value is None else outer_value
        outer_natural = cfg.outer_natural if outer_natural is None else outer_natural
        kfine = cfg.k if getattr(problem, "k_field", None) is None else problem.k_field
        # wall_normals: maximum-entropy zero-flux closure at the grains' walls
        # with these unit outward normals ([2, N, N]) instead of bounce-back
        self.lat = Lattice(self.N, tau, problem.vx.astype(np.float64), problem.vy.astype(np.float64),
                           solid=problem.solid, k=kfine, clamp=cfg.bc_clamp, wall_normals=wall_normals)
        self.outer, self.fc = coarse_dirichlet_sets(self.M, self.L, self.N, problem.x0, problem.y0,
                                                    cfg.overlap_elems, outer_natural)
        rows = np.sort(np.concatenate([self.outer, self.fc]))
        self.rows_sorted = rows
        pos = np.searchsorted(self.fc, rows)
        pos_c = np.minimum(pos, max(len(self.fc) - 1, 0))
        self._is_fc = (pos < len(self.fc)) & (self.fc[pos_c] == rows) if len(self.fc) else np.zeros(len(rows), bool)
        self._fc_pos = pos_c
        self.outer_value = outer_value
        self.fem = FemStepper(self.M, self.L, cfg.D, cfg.k, float(self.eta), cfg.supg, problem.vc, rows)
        ii, jj = perimeter_nodes(self.N)
        self.perim_X = problem.x0 + ii
        self.perim_Y = problem.y0 + jj
        h = self.L / self.M
        s = self.M + 1
        self.fc_px = (self.fc % s) * h - problem.x0
        self.fc_py = (self.fc // s) * h - problem.y0
        self.fstar = self.lat.init(problem.u0_fine)
        self.d = np.array(problem.u0_coarse, dtype=np.float64)
        self.infeasible = 0

    # -- transfers ---------------------------------------------------------
    def fine_to_coarse(self, fstar):
        u = self.lat.concentration(fstar)
        return fine_to_coarse(self.N, self.p.solid, u, self.fc_px, self.fc_py)

    def coarse_to_fine(self, d):
        return fem_interpolate(self.M, self.L, d, self.perim_X, self.perim_Y)

    # -- coarse step -------------------------------------------------------
    def coarse_step(self, d0, ufc):
        vals = np.full(len(self.rows_sorted), self.outer_value, dtype=np.float64)
        vals[self._is_fc] = np.asarray(ufc)[self._fc_pos[self._is_fc]]
        return self.fem.step(d0, vals)

    # -- fine sub-steps ----------------------------------------------------
    def lbm_substeps(self, fstar0, a, b, n_sub=None):
        F = fstar0
        n_sub = self.eta if n_sub is None else n_sub
        if not hasattr(self, "_ping"):
            self._ping = (np.empty_like(fstar0), np.empty_like(fstar0))
        for j in range(1, n_sub + 1):
            lam = j / self.eta
            up = (1.0 - lam) * a + lam * b
            F, inf = self.lat.substep(F, up, out=self._ping[j % 2])
            self.infeasible += inf
        # the result leaves the step buffers (the caller keeps it as state)
        return F.copy() if n_sub > 0 else F

    # -- Algorithm 1 -------------------------------------------------------
    def step(self):
        algorithm1_step(self)

    def run(self, steps):
        for _ in range(steps):
            self.step()
        return self

    def fine_concentration(self):
        return self.lat.concentration(self.fstar)


def run_hybrid(problem, steps=None, **kw):
    o = HybridOracle(problem, **kw)
    o.run(problem.cfg.steps if steps is None else steps)
    return o
