"""Algorithm 2 (hybrid coupling with several subdomains, Sec. 6.3) for one
coarse subdomain and several fine lattice patches -- TEST INFRASTRUCTURE
ONLY (tests, smoke and the benchmark's CPU leg use it; the product path
never does).

Reading: the coarse subdomain is the whole square (as for one patch); its
Dirichlet rows are the outer edges and, for every patch, the coarse nodes
inside that patch at least ``overlap_elems`` elements from its boundary
(the patches are disjoint and far enough apart that no coarse node belongs
to two of them); each Schwarz iteration first advances the coarse
subdomain with the values every patch produced in the previous iteration
(the first from the patches' states at t_n), then advances every patch by
eta fine steps from t_n with eq. (MTS) at its own perimeter -- Algorithm 1
for each patch, with the coarse solve shared.
"""
from __future__ import annotations

import numpy as np

from . import FemStepper, Lattice, fem_interpolate, fine_to_coarse, perimeter_nodes, relaxation_time
from .hybrid import coarse_dirichlet_sets


class ManyPatchOracle:
    def __init__(self, mp, outer_value=0.0):
        self.mp = mp
        M, L = mp.M, mp.L
        self.M, self.L, self.eta, self.max_iter = M, L, mp.eta, mp.max_iter
        self.outer_value = outer_value
        h = L / M
        s = M + 1
        outer = None
        self.fc = []
        self.lat, self.perim, self.fc_p = [], [], []
        for p in mp.patches:
            o, fc = coarse_dirichlet_sets(M, L, p.N, p.x0, p.y0, mp.overlap_elems)
            outer = o
            self.fc.append(fc)
            self.lat.append(Lattice(p.N, relaxation_time(mp.D), p.vx.astype(np.float64), p.vy.astype(np.float64),
                                    solid=p.solid, k=mp.k, clamp=mp.bc_clamp))
            ii, jj = perimeter_nodes(p.N)
            self.perim.append((p.x0 + ii, p.y0 + jj))
            self.fc_p.append(((fc % s) * h - p.x0, (fc // s) * h - p.y0))
        allfc = np.concatenate(self.fc) if self.fc else np.zeros(0, np.int64)
        if len(np.unique(allfc)) != len(allfc):
            raise ValueError("a coarse node lies in the interface set of two patches")
        self.rows = np.sort(np.concatenate([outer, allfc]))
        self.fem = FemStepper(M, L, mp.D, mp.k, float(mp.eta), mp.supg, mp.vc, self.rows)
        self.fstar = [lat.init(p.u0_fine) for lat, p in zip(self.lat, mp.patches)]
        self.d = np.array(mp.u0_coarse, dtype=np.float64)

    def fine_to_coarse(self, j, fstar):
        p = self.mp.patches[j]
        u = self.lat[j].concentration(fstar)
        return fine_to_coarse(p.N, p.solid, u, *self.fc_p[j])

    def coarse_to_fine(self, j, d):
        return fem_interpolate(self.M, self.L, d, *self.perim[j])

    def coarse_step(self, d0, ufc):
        """One coarse step with the outer rows at outer_value and each
        patch's interface rows at its transferred values."""
        vals = np.full(len(self.rows), self.outer_value, dtype=np.float64)
        for fc, u in zip(self.fc, ufc):
            vals[np.searchsorted(self.rows, fc)] = u
        return self.fem.step(d0, vals)

    def substeps(self, j, fstar0, a, b):
        F = fstar0
        for t in range(1, self.eta + 1):
            lam = t / self.eta
            F, _ = self.lat[j].substep(F, (1.0 - lam) * a + lam * b)
        return F

    def step(self):
        n = len(self.mp.patches)
        ufc = [self.fine_to_coarse(j, self.fstar[j]) for j in range(n)]
        a = [self.coarse_to_fine(j, self.d) for j in range(n)]
        for _ in range(self.max_iter):
            d1 = self.coarse_step(self.d, ufc)
            F = [self.substeps(j, self.fstar[j], a[j], self.coarse_to_fine(j, d1)) for j in range(n)]
            ufc = [self.fine_to_coarse(j, F[j]) for j in range(n)]
        self.fstar = F
        self.d = d1

    def run(self, steps):
        for _ in range(steps):
            self.step()
        return self
