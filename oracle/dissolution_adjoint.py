"""Reverse mode of one coarse step with dissolving solids -- TEST
INFRASTRUCTURE ONLY (tests, smoke and the benchmark's CPU leg use it; the
product path never does).

A coarse step of the dissolving-solid model (oracle/dissolution.py) is the
step of Algorithm 1 (Sec. 6.2) on the geometry frozen for that step -- its
reactive bounce-back f_q = (1 - kappa_s) f*_opp(q) + kappa_s w_q c_sat is
affine in the state -- followed by the commit.  Once the set of nodes that
convert is fixed, the commit is linear in the committed state: a converted
node n takes

    f*_q(n) = w_q (1 - k_n) (1 / |F(n)|) sum_{x in F(n)} sum_p f*_p(x) / (1 - k_x),

F(n) its fluid 8-neighbours before the commit.  The set itself comes from
comparing masses with link fluxes, a piecewise-constant decision whose
derivative vanishes almost everywhere, so the masses are not
differentiated.  The adjoint therefore transposes the conversion first
(gathering each converted node's cotangent onto its fluid neighbours, and
its k terms into dJ/dk), then runs the passes backwards exactly as for
fixed solids, with the step's own lattice (geometry and reaction), its
transfer rows (weights of the fluid corners of that step) and fluid set.

``replay`` re-applies a recorded step -- same geometry, same converting
nodes -- to any state and per-node rate; it is the map the adjoint
transposes, and the pins use it for the dot-product identity and central
differences.
"""
from __future__ import annotations

import numpy as np

from . import Lattice, d2q9
from .dissolution import convert, link_flux
from .hybrid_adjoint import HybridStepAdjoint


def dynamic_rows(o):
    """Fine-to-coarse rows of a DissolvingHybrid for its current geometry:
    (nodes, weights) per Gamma_{f->c} node, the fluid corners with their
    renormalised bilinear weights, or the fallback node with weight 1."""
    sol = np.asarray(o.solid).reshape(-1) != 0
    rows = []
    for (nd, wr), fb in zip(o.corners, o.fallback):
        fl = [m for m in range(4) if not sol[nd[m]]]
        wsum = sum(wr[m] for m in fl)
        if wsum > 0.0:
            rows.append(([nd[m] for m in fl], [wr[m] / wsum for m in fl]))
        else:
            rows.append(([fb], [1.0]))
    return rows


def _fluid_neighbours(N, sol_flat, n):
    ex, ey, _, _ = d2q9()
    j, i = divmod(int(n), N)
    out = []
    for q in range(1, 9):
        xi, xj = i + int(ex[q]), j + int(ey[q])
        if 0 <= xi < N and 0 <= xj < N and not sol_flat[xj * N + xi]:
            out.append(xj * N + xi)
    return out


def apply_conversion(F, solid_before, conv, kfield):
    """The commit's conversion with a fixed converting set: every node in
    conv takes w_q (1 - k_n) times the mean concentration of its fluid
    neighbours (fluid set before the commit); the rest is unchanged."""
    N = solid_before.shape[0]
    _, _, w, _ = d2q9()
    sol = np.asarray(solid_before).reshape(-1) != 0
    k = np.asarray(kfield, np.float64).reshape(-1)
    f = np.array(F, np.float64).reshape(9, N * N)
    u = np.where(sol, 0.0, f.sum(axis=0) / (1.0 - k))
    for n in np.flatnonzero(np.asarray(conv).reshape(-1)):
        vals = [u[x] for x in _fluid_neighbours(N, sol, n)]
        ubar = sum(vals) / len(vals) if vals else 0.0
        f[:, n] = np.asarray(w) * ubar * (1.0 - k[n])
    return f.reshape(9, N, N)


class DissolvingStepAdjoint(HybridStepAdjoint):
    """Recorded forward, replay and adjoint of coarse steps of a
    DissolvingHybrid (outer Dirichlet value 0, no clamp)."""

    def __init__(self, o):
        super().__init__(o)

    def forward(self, F, d):
        """One coarse step from (F, d) on the hybrid's current geometry, as
        DissolvingHybrid.step; the hybrid's solids and masses advance with
        it.  Returns (F_new, d_new, tape)."""
        o = self.o
        solid_before = o.solid.copy()
        tape = {"F": F, "passes": [], "lat": o.lat, "rows": dynamic_rows(o), "solid": solid_before,
                "fluid": solid_before.reshape(-1) == 0}
        ufc_src = F
        a = o.coarse_to_fine(d)
        for _ in range(o.max_iter):
            ufc = o.fine_to_coarse(ufc_src)
            d1 = o.coarse_step(d, ufc)
            b = o.coarse_to_fine(d1)
            states = [F]
            flux = np.zeros((o.N, o.N))
            for j in range(1, o.eta + 1):
                lam = j / o.eta
                flux += link_flux(o.lat, states[-1], o.solid)
                nxt, _ = o.lat.substep(states[-1], (1 - lam) * a + lam * b)
                states.append(nxt)
            tape["passes"].append({"src": ufc_src, "a": a, "b": b, "states": states})
            ufc_src = states[-1]
        F_new, o.solid, o.mass, n = convert(ufc_src, solid_before, o.mass, flux, o.kf)
        o.converted += n
        if n:
            o._rebuild()
        tape["pre"] = ufc_src
        tape["conv"] = (solid_before != 0) & (o.solid == 0)
        return F_new, d1, tape

    def replay(self, tape, F, d, kfield=None):
        """The recorded step (its geometry, its converting nodes) applied to
        (F, d), with the per-node rate kfield [N, N] in the fine steps, the
        transfer's concentrations and the conversion (default: the
        hybrid's)."""
        o = self.o
        lat0 = tape["lat"]
        k = o.kf if kfield is None else np.asarray(kfield, np.float64)
        lat = lat0 if kfield is None else Lattice(o.N, lat0.tau, lat0.vx, lat0.vy, solid=tape["solid"], k=k,
                                                  clamp=o.p.cfg.bc_clamp, kappa_s=lat0.kappa_s,
                                                  c_sat=lat0.c_sat)
        ufc_src = F
        a = o.coarse_to_fine(d)
        for _ in range(len(tape["passes"])):
            ufc = o.transfer(lat.concentration(ufc_src), tape["solid"])
            d1 = o.coarse_step(d, ufc)
            b = o.coarse_to_fine(d1)
            G = F
            for j in range(1, o.eta + 1):
                lam = j / o.eta
                G, _ = lat.substep(G, (1 - lam) * a + lam * b)
            ufc_src = G
        return apply_conversion(ufc_src, tape["solid"], tape["conv"], k), d1

    def conversion_T(self, tape, lam):
        """Transpose of the recorded conversion: (dJ/d(state before the
        commit) [9,N,N], dJ/dk [N,N]) for lam = dJ/d(committed state)."""
        N = self.o.N
        _, _, w, _ = d2q9()
        sol = tape["solid"].reshape(-1) != 0
        k = np.asarray(self.o.kf, np.float64).reshape(-1)
        pre = np.asarray(tape["pre"], np.float64).reshape(9, N * N)
        u = np.where(sol, 0.0, pre.sum(axis=0) / (1.0 - k))
        lam = np.asarray(lam, np.float64).reshape(9, N * N)
        out = lam.copy()
        gk = np.zeros(N * N)
        for n in np.flatnonzero(tape["conv"].reshape(-1)):
            nbrs = _fluid_neighbours(N, sol, n)
            lw = sum(w[q] * lam[q, n] for q in range(9))
            ubar = sum(u[x] for x in nbrs) / len(nbrs) if nbrs else 0.0
            gk[n] -= ubar * lw
            if nbrs:
                g = (1.0 - k[n]) * lw / len(nbrs)
                for x in nbrs:
                    out[:, x] += g / (1.0 - k[x])
                    gk[x] += g * u[x] / (1.0 - k[x])
            out[:, n] = 0.0
        return out.reshape(9, N, N), gk.reshape(N, N)

    def adjoint(self, tape, lam_f, lam_d, outer=False):
        """(dJ/dF, dJ/dd^n, dJ/dk[, dJ/dg_outer]) of the recorded step for
        lam_f = dJ/df*(t_{n+1}), lam_d = dJ/dd^{n+1}."""
        lam_pre, gk_conv = self.conversion_T(tape, lam_f)
        res = super().adjoint(tape, lam_pre, lam_d, outer=outer)
        return (res[0], res[1], res[2] + gk_conv) + tuple(res[3:])
