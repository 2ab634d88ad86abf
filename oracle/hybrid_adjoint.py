"""Reverse mode (adjoint) of one coarse step of Algorithm 1 -- TEST
INFRASTRUCTURE ONLY (tests, smoke and the benchmark's CPU leg use it; the
product path never does).

With zero outer Dirichlet data and the interface closure applied as printed
(no clamp), one coarse step of Algorithm 1 (Sec. 6.2) maps the committed
state (f*(t_n), d^n) linearly to (f*(t_{n+1}), d^{n+1}): every piece is
linear -- the fine steps (Sec. 4.1, eq. LBM_Dir, eq. MTS), the
coarse-to-fine interpolation (Sec. 6.2 item i), the trapezoidal coarse step
with strong Dirichlet rows (eq. FEM_discrete) and the fine-to-coarse
transfer (Sec. 6.2 item ii).  The adjoint runs the Schwarz passes backwards
through the transposes of the pieces:

  pass p (p = P-1 .. 0), given lam_p = dJ/d(fine result of pass p):
    fine steps      lam_F += S^T lam_p, giving dJ/da, dJ/db of the pass
    c->f            lam_dn += C^T dJ/da;  lam_d1 = C^T dJ/db (+ dJ/dd^{n+1} on the last pass)
    coarse solve    mu = A_D^{-T} lam_d1;  lam_dn += B^T (mu on free rows);
                    dJ/d(Dirichlet value) = mu on the Dirichlet rows
    f->c            the fine state the pass's transfer read (f*(t_n) for
                    p = 0, the previous pass's result otherwise) receives
                    T^T dJ/du_fc

Each transpose is written from the definition of its forward map (the
oracle's C functions): Q1 shape functions on the containing element
(element index clamped to M - 1), bilinear weights on the lattice square
with solid corners dropped and the remaining weights renormalised or, with
four solid corners, the nearest fluid node; the coarse matrices come from
the oracle's assembly, A_D with its Dirichlet rows replaced by identity rows
(as the oracle's banded solve uses it); the transposed solve is SciPy's
sparse direct solve of A_D^T.  Each transpose is pinned against its forward
C function by the dot-product identity in the tests.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem_matrices


def band_to_csr(M, band):
    """Sparse copy of an oracle band matrix (kl = ku = M + 2, LAPACK band
    storage with the LU fill rows, column-major)."""
    n = (M + 1) ** 2
    kl = ku = M + 2
    ldab = 2 * kl + ku + 1
    kv = kl + ku
    band = np.asarray(band, np.float64)
    rows, cols, vals = [], [], []
    for off in range(-kl, ku + 1):          # entry (i, j) with j - i = off
        i = np.arange(max(0, -off), min(n, n - off))
        j = i + off
        v = band[j * ldab + kv + i - j]
        nz = v != 0.0
        rows.append(i[nz])
        cols.append(j[nz])
        vals.append(v[nz])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def c2f_weights(M, L, X, Y):
    """Rows of the coarse-to-fine interpolation: for each point (X, Y) the
    four corner nodes of its containing element and their Q1 weights."""
    h = L / M
    s = M + 1
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    sx, sy = X / h, Y / h
    ex = np.clip(np.floor(sx).astype(int), 0, M - 1)
    ey = np.clip(np.floor(sy).astype(int), 0, M - 1)
    xi, et = sx - ex, sy - ey
    idx = np.stack([ey * s + ex, ey * s + ex + 1, (ey + 1) * s + ex + 1, (ey + 1) * s + ex], axis=1)
    w = np.stack([(1 - xi) * (1 - et), xi * (1 - et), xi * et, (1 - xi) * et], axis=1)
    return idx, w


def _nearest_fluid(N, solid, px, py):
    """Nearest fluid node (squared distance, lowest j*N + i on ties) found
    by growing squares around the rounded point, as the forward does."""
    ci, cj = int(math.floor(px + 0.5)), int(math.floor(py + 0.5))
    for r in range(1, 2 * N + 1):
        best, bd = -1, 0.0
        for j in range(max(cj - r, 0), min(cj + r, N - 1) + 1):
            for i in range(max(ci - r, 0), min(ci + r, N - 1) + 1):
                if solid[j, i]:
                    continue
                d2 = (i - px) ** 2 + (j - py) ** 2
                if best < 0 or d2 < bd:
                    best, bd = j * N + i, d2
        if best >= 0 and math.sqrt(bd) <= r - 0.5:
            return best
    return -1


def f2c_weights(N, solid, px, py):
    """Rows of the fine-to-coarse transfer: for each coarse node at lattice
    coordinates (px, py), the lattice nodes (flat j*N + i) and weights that
    combine their concentrations."""
    rows = []
    for x, y in zip(np.atleast_1d(px), np.atleast_1d(py)):
        i0 = min(max(int(math.floor(x)), 0), N - 2)
        j0 = min(max(int(math.floor(y)), 0), N - 2)
        gx, gy = x - i0, y - j0
        nd = [j0 * N + i0, j0 * N + i0 + 1, (j0 + 1) * N + i0 + 1, (j0 + 1) * N + i0]
        w = [(1 - gx) * (1 - gy), gx * (1 - gy), gx * gy, (1 - gx) * gy]
        if solid is None:
            rows.append((nd, w))
            continue
        fl = [c for c in range(4) if not solid.flat[nd[c]]]
        wsum = sum(w[c] for c in fl)
        if wsum > 0.0:
            rows.append(([nd[c] for c in fl], [w[c] / wsum for c in fl]))
        else:
            nf = _nearest_fluid(N, solid, x, y)
            rows.append(([nf], [1.0]) if nf >= 0 else ([], []))
    return rows


class HybridStepAdjoint:
    """Recorded forward and adjoint of one coarse step of a HybridOracle
    (no clamp: the step is then affine in the state)."""

    def __init__(self, o):
        # with outer Dirichlet data g != 0 the step is affine; its adjoint is
        # that of the linear part (g enters only through dJ/dg)
        self.o = o
        cfg = o.p.cfg
        a, b = fem_matrices(o.M, o.L, cfg.D, cfg.k, float(o.eta), cfg.supg, o.p.vc)
        self.A = band_to_csr(o.M, a).tolil()
        for r in o.rows_sorted:                  # strong Dirichlet rows: identity
            self.A.rows[r] = [int(r)]
            self.A.data[r] = [1.0]
        self.A = self.A.tocsr()
        self.B = band_to_csr(o.M, b)
        self.free = np.ones(self.A.shape[0], bool)
        self.free[o.rows_sorted] = False
        self.AT_lu = spla.splu(self.A.T.tocsc())
        self.c2f_idx, self.c2f_w = c2f_weights(o.M, o.L, o.perim_X, o.perim_Y)
        self.f2c_rows = f2c_weights(o.N, o.p.solid, o.fc_px, o.fc_py)
        N = o.N
        self.kfield = (o.lat.kfield if o.lat.kfield is not None else np.full((N, N), o.lat.kval)).reshape(-1)
        sol = o.p.solid
        self.fluid = np.ones(N * N, bool) if sol is None else (np.asarray(sol).reshape(-1) == 0)

    # -- transposes of the pieces -------------------------------------------
    def c2f_T(self, g):
        """C^T g: per-slot cotangents g to the coarse nodes."""
        out = np.zeros(self.A.shape[0])
        np.add.at(out, self.c2f_idx.reshape(-1), (self.c2f_w * np.asarray(g)[:, None]).reshape(-1))
        return out

    def f2c_T(self, lam_ufc, g_state, rows=None, fluid=None):
        """T^T lam_ufc for the transfer read of state g_state: (dJ/df* [9,N,N],
        dJ/dk [N,N]); u = sum_q f*_q / (1 - k) at fluid nodes.  rows and
        fluid: the transfer's rows and fluid set (default: the problem's
        fixed geometry)."""
        N = self.o.N
        rows = self.f2c_rows if rows is None else rows
        fluid = self.fluid if fluid is None else fluid
        lam_u = np.zeros(N * N)
        for (nd, w), l in zip(rows, lam_ufc):
            for n, wn in zip(nd, w):
                lam_u[n] += wn * l
        lam_u[~fluid] = 0.0
        one_k = 1.0 - self.kfield
        lam_f = np.broadcast_to(lam_u / one_k, (9, N * N)).copy()
        s = np.asarray(g_state).reshape(9, N * N).sum(axis=0)
        gk = lam_u * s / one_k ** 2
        return lam_f.reshape(9, N, N), gk.reshape(N, N)

    def coarse_T(self, lam_d1):
        """Transpose of d1 = A_D^{-1} (B d on free rows, values on Dirichlet
        rows): (dJ/dd, dJ/d(values) aligned with rows_sorted)."""
        mu = self.AT_lu.solve(np.asarray(lam_d1, np.float64))
        lam_d = self.B.T @ np.where(self.free, mu, 0.0)
        return lam_d, mu[self.o.rows_sorted]

    def ufc_of_values(self, lam_vals):
        """dJ/du_fc from dJ/d(Dirichlet values): the values of the
        Gamma_{f->c} rows are the transfer's outputs."""
        o = self.o
        lam_ufc = np.zeros(len(o.fc))
        lam_ufc[o._fc_pos[o._is_fc]] = np.asarray(lam_vals)[o._is_fc]
        return lam_ufc

    # -- forward with tape, then reverse -------------------------------------
    def forward(self, F, d):
        """One coarse step from (F, d) (Algorithm 1, as HybridOracle.step);
        returns (F_new, d_new, tape)."""
        o = self.o
        tape = {"F": F, "passes": []}
        ufc_src = F
        a = o.coarse_to_fine(d)
        for _ in range(o.max_iter):
            ufc = o.fine_to_coarse(ufc_src)
            d1 = o.coarse_step(d, ufc)
            b = o.coarse_to_fine(d1)
            states = [F]
            for j in range(1, o.eta + 1):
                lam = j / o.eta
                nxt, _ = o.lat.substep(states[-1], (1 - lam) * a + lam * b)
                states.append(nxt)
            tape["passes"].append({"src": ufc_src, "a": a, "b": b, "states": states})
            ufc_src = states[-1]
        return ufc_src, d1, tape

    def adjoint(self, tape, lam_f, lam_d, outer=False, lam_sub=None):
        """(dJ/dF, dJ/dd^n, dJ/dk) for cotangents lam_f = dJ/df*(t_{n+1})
        [9,N,N] and lam_d = dJ/dd^{n+1} [(M+1)^2]; with outer, also dJ/dg
        for the prescribed values g of the outer-edge Dirichlet rows (per
        mesh node, zero elsewhere).  lam_sub [9,N,N]: J also holds
        <lam_sub, f*(t_n + j)> for every intermediate fine state j = 1 ..
        eta-1 of the committed (last) pass, so an objective can integrate
        over every fine step."""
        o = self.o
        N = o.N
        # a tape may carry the lattice, transfer rows and fluid set of its
        # own step (dissolving solids); else those of the fixed geometry
        lat = tape.get("lat", o.lat)
        lam_F = np.zeros((9, N, N))
        lam_dn = np.zeros(self.A.shape[0])
        g_outer = np.zeros(self.A.shape[0])
        gk = np.zeros((N, N))
        lam_p = np.asarray(lam_f, np.float64)
        passes = tape["passes"]
        for p in range(len(passes) - 1, -1, -1):
            rec = passes[p]
            lam = lam_p
            ga = np.zeros(4 * (N - 1))
            gb = np.zeros(4 * (N - 1))
            for j in range(o.eta, 0, -1):
                lt = j / o.eta
                up = (1 - lt) * rec["a"] + lt * rec["b"]
                lam, gbc, kk = lat.adjoint_substep(rec["states"][j - 1], up, lam)
                if lam_sub is not None and p == len(passes) - 1 and j - 1 >= 1:
                    lam = lam + lam_sub
                ga += (1 - lt) * gbc
                gb += lt * gbc
                gk += kk
            lam_F += lam
            lam_dn += self.c2f_T(ga)
            lam_d1 = self.c2f_T(gb)
            if p == len(passes) - 1:
                lam_d1 = lam_d1 + np.asarray(lam_d, np.float64)
            ld, lvals = self.coarse_T(lam_d1)
            lam_dn += ld
            rows = o.rows_sorted
            g_outer[rows[~o._is_fc]] += np.asarray(lvals)[~o._is_fc]
            lf, kf = self.f2c_T(self.ufc_of_values(lvals), rec["src"], tape.get("rows"), tape.get("fluid"))
            gk += kf
            if p == 0:
                lam_F += lf
            else:
                lam_p = lf
        if outer:
            return lam_F, lam_dn, gk, g_outer
        return lam_F, lam_dn, gk
