"""Dissolving solids in the hybrid method -- TEST INFRASTRUCTURE ONLY (tests,
smoke and the benchmark's CPU leg use it; the product path never does).

The pore geometry carries a scalar mass per solid node and a first-order
surface reaction at every fluid-solid link; solids whose mass is used up
turn into fluid.  The paper's calcite example (Sec. 7.4) keeps its solids
fixed, so the model below is a reading, written out step by step:

* surface reaction (per fine step, in the halfway bounce-back of Sec. 4.1):
  the population that a fluid node x sent towards a solid neighbour returns
  relaxed towards w_q c_sat, f_q(x) = (1 - kappa_s) f*_opp(q)(x) +
  kappa_s w_q c_sat; that link adds J = kappa_s (w_q c_sat - f*_opp(q)(x))
  to the fluid and takes it from the solid node (kappa_s = 0: plain
  bounce-back);
* geometry is frozen within a coarse step (every Schwarz pass restarts from
  the committed geometry as from the committed state); each pass sums the
  link fluxes of its fine steps per solid node, and the commit subtracts the
  last pass's sums from the solid masses;
* at the commit a solid node whose mass is <= 0 becomes fluid; it takes the
  post-collision equilibrium of the mean concentration of its fluid
  neighbours (8-neighbourhood in the patch, the fluid set before the
  commit) at zero velocity, f*_q = w_q u_mean (1 - k); the advection field
  is not recomputed (it is zero there);
* the fine-to-coarse transfer (Sec. 6.2 item ii) uses the bilinear weights
  of the current fluid corners, renormalised; a coarse node whose fluid
  corners carry no weight keeps the nearest fluid node chosen for the
  initial geometry (fluid never turns solid, so it stays fluid) until a
  corner with weight turns fluid.
"""
from __future__ import annotations

import numpy as np

from . import Lattice, d2q9, relaxation_time
from .hybrid import HybridOracle, algorithm1_step
from .hybrid_adjoint import f2c_weights


def link_flux(lat, fstar, solid):
    """Mass moved into the fluid by the surface reaction during one fine
    step from fstar, summed per solid node ([N, N]; zero at fluid nodes)."""
    N = lat.N
    ex, ey, w, opp = d2q9()
    f = np.asarray(fstar, np.float64).reshape(9, N, N)
    sol = np.asarray(solid, bool)
    out = np.zeros((N, N))
    if lat.kappa_s == 0.0:
        return out
    for q in range(1, 9):
        # fluid node x = s + e_q pulls direction q from the solid node s
        dx, dy = int(ex[q]), int(ey[q])
        i0, i1 = max(0, -dx), N - max(0, dx)
        j0, j1 = max(0, -dy), N - max(0, dy)
        s_sol = sol[j0:j1, i0:i1]
        x_fluid = ~sol[j0 + dy:j1 + dy, i0 + dx:i1 + dx]
        fx = f[opp[q], j0 + dy:j1 + dy, i0 + dx:i1 + dx]
        out[j0:j1, i0:i1] += np.where(s_sol & x_fluid, lat.kappa_s * (w[q] * lat.c_sat - fx), 0.0)
    return out


def convert(fstar, solid, mass, flux, kfield):
    """Commit of the geometry: masses lose the pass's flux, exhausted solids
    become fluid with the equilibrium of their fluid neighbours' mean
    concentration.  Returns (fstar, solid, mass, converted count)."""
    N = solid.shape[0]
    ex, ey, w, _ = d2q9()
    sol = np.asarray(solid, bool)
    f = np.array(fstar, np.float64).reshape(9, N, N)
    m = np.where(sol, np.asarray(mass, np.float64) - np.asarray(flux, np.float64), 0.0)
    conv = sol & (m <= 0.0)
    u = np.where(sol, 0.0, f.sum(axis=0) / (1.0 - kfield))
    for j, i in zip(*np.nonzero(conv)):
        vals = []
        for q in range(1, 9):
            xi, xj = i + ex[q], j + ey[q]
            if 0 <= xi < N and 0 <= xj < N and not sol[xj, xi]:
                vals.append(u[xj, xi])
        ubar = sum(vals) / len(vals) if vals else 0.0
        f[:, j, i] = np.asarray(w) * ubar * (1.0 - kfield[j, i])
    new_solid = sol & ~conv
    m[conv] = 0.0
    return f, new_solid.astype(np.uint8), m, int(conv.sum())


class DissolvingHybrid(HybridOracle):
    """HybridOracle whose solids dissolve (readings in the module text)."""

    def __init__(self, problem, mass, kappa_s, c_sat, **kw):
        super().__init__(problem, **kw)
        self.kappa_s, self.c_sat = float(kappa_s), float(c_sat)
        self.solid = np.asarray(problem.solid, np.uint8).copy()
        self.mass = np.where(self.solid != 0, np.asarray(mass, np.float64), 0.0)
        cfg = problem.cfg
        N = self.N
        self.kf = np.full((N, N), cfg.k)
        self.converted = 0
        # corners and raw bilinear weights of every Gamma_{f->c} node, and
        # the initial geometry's nearest fluid node for all-solid corners
        self.corners = []
        for x, y in zip(self.fc_px, self.fc_py):
            i0 = min(max(int(np.floor(x)), 0), N - 2)
            j0 = min(max(int(np.floor(y)), 0), N - 2)
            gx, gy = x - i0, y - j0
            nd = [j0 * N + i0, j0 * N + i0 + 1, (j0 + 1) * N + i0 + 1, (j0 + 1) * N + i0]
            wr = [(1 - gx) * (1 - gy), gx * (1 - gy), gx * gy, (1 - gx) * gy]
            self.corners.append((nd, wr))
        rows = f2c_weights(N, self.solid, self.fc_px, self.fc_py)
        sol0 = self.solid.reshape(-1) != 0
        self.fallback = [rows[c][0][0] if sum(wr[m] for m in range(4) if not sol0[nd[m]]) == 0.0 else None
                         for c, (nd, wr) in enumerate(self.corners)]
        self._rebuild()
        self.fstar = self.lat.init(problem.u0_fine)

    def _rebuild(self):
        cfg = self.p.cfg
        # advection is zero wherever a solid stood initially (and stays so)
        sol0 = np.asarray(self.p.solid) != 0
        vx = np.where(sol0, 0.0, self.p.vx.astype(np.float64))
        vy = np.where(sol0, 0.0, self.p.vy.astype(np.float64))
        self.lat = Lattice(self.N, relaxation_time(cfg.D, cfg.tau), vx, vy, solid=self.solid, k=cfg.k, clamp=cfg.bc_clamp,
                           kappa_s=self.kappa_s, c_sat=self.c_sat)

    def transfer(self, u, solid):
        """Fine-to-coarse values of the concentration field u [N, N] with the
        fluid corners of the geometry ``solid``."""
        u = np.asarray(u).reshape(-1)
        sol = np.asarray(solid).reshape(-1) != 0
        out = np.empty(len(self.corners))
        for c, ((nd, wr), fb) in enumerate(zip(self.corners, self.fallback)):
            wsum = sum(wr[m] for m in range(4) if not sol[nd[m]])
            if wsum > 0.0:
                out[c] = sum(wr[m] * u[nd[m]] for m in range(4) if not sol[nd[m]]) / wsum
            else:
                out[c] = u[fb]
        return out

    def fine_to_coarse(self, fstar):
        return self.transfer(self.lat.concentration(fstar), self.solid)

    def lbm_substeps(self, fstar0, a, b, n_sub=None):
        n_sub = self.eta if n_sub is None else n_sub
        self.flux = np.zeros((self.N, self.N))
        F = fstar0
        for j in range(1, n_sub + 1):
            lam = j / self.eta
            self.flux += link_flux(self.lat, F, self.solid)
            F, inf = self.lat.substep(F, (1.0 - lam) * a + lam * b)
            self.infeasible += inf
        return F

    def step(self):
        algorithm1_step(self)
        self.fstar, self.solid, self.mass, n = convert(self.fstar, self.solid, self.mass, self.flux, self.kf)
        self.converted += n
        if n:
            self._rebuild()
