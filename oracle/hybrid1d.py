"""One-dimensional hybrid (Sec. 7.1: D1Q2 lattice Boltzmann on the fine
subdomain, two-node linear Galerkin finite elements on the coarse one)
driven by the same Algorithm 1 loop as the two-dimensional oracle
(``hybrid.algorithm1_step``).  TEST INFRASTRUCTURE ONLY: it pins the
coupling logic against the errors the paper prints for the advected
Gaussian hill (Tables 1DGauss_1 - 1DGauss_6).

Set-up (Sec. 7.1): Omega = (0, 1), zero flux at both ends; coarse
subdomain (0, 1/2 + L_ov/2), fine subdomain (1/2 - L_ov/2, 1); advection
velocity v, diffusion D, no source.  Time steps dt = h^2 / (2 D) on both
grids, so eta = (h_c / h_f)^2 and the D1Q2 relaxation time is 1.

* D1Q2 (Sec. 4.1 in one dimension): velocities +-c, c = h_f / dt_f,
  weights 1/2, c_s^2 = c^2; f_i^eq = (u / 2) (1 + e_i v / c_s^2); BGK
  collision with tau = 1/2 + D dt_f / h_f^2.  The stored state is f*.
* Fine boundaries: at x = 1/2 - L_ov/2 the incoming population is the
  single unknown of the maximum-entropy Dirichlet closure, eq. (LBM_Dir):
  f_+ = u^p - f_-, with u^p from eq. (MTS); at x = 1 zero flux (the
  Neumann closure with q = 0 and one unknown): f_- = f_+.
* Coarse: linear elements of size h_c, consistent mass, Galerkin
  advection-diffusion, trapezoidal rule (the d-form A d1 = B d0 of the 2-D
  oracle); zero flux at x = 0 is the natural condition; the right end node
  x = 1/2 + L_ov/2 takes its Dirichlet value from the lattice.
* Transfers: both interface points coincide with nodes of the other grid
  (the printed discretisations make (1/2 -+ L_ov/2) multiples of h_c and
  of h_f), so the transfers are nodal values.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded
from scipy.sparse import diags

from .hybrid import algorithm1_step


def gaussian_exact(x, t, phi, sigma0, x0, v, D):
    """Advected, spreading Gaussian of mass phi on the real line."""
    s2 = sigma0 ** 2 + 2.0 * D * t
    return phi / np.sqrt(2.0 * np.pi * s2) * np.exp(-(x - x0 - v * t) ** 2 / (2.0 * s2))


class Hybrid1D:
    def __init__(self, h_c, h_f, L_ov, max_iter, v=1.0, D=1e-2, phi=0.1, sigma0=1e-2, x0=0.3):
        self.v, self.D = v, D
        self.max_iter = max_iter
        self.dt_c = h_c ** 2 / (2.0 * D)
        self.dt_f = h_f ** 2 / (2.0 * D)
        self.eta = int(round(self.dt_c / self.dt_f))
        assert abs(self.eta * self.dt_f - self.dt_c) < 1e-12 * self.dt_c
        xc_end = 0.5 + 0.5 * L_ov
        xf_start = 0.5 - 0.5 * L_ov
        nc = int(round(xc_end / h_c))
        nf = int(round((1.0 - xf_start) / h_f))
        assert abs(nc * h_c - xc_end) < 1e-9 and abs(nf * h_f - (1.0 - xf_start)) < 1e-9
        self.xc = np.arange(nc + 1) * h_c
        self.xf = xf_start + np.arange(nf + 1) * h_f
        self.ic_interface = int(round(xf_start / h_c))          # coarse node at the fine boundary
        assert abs(self.xc[self.ic_interface] - xf_start) < 1e-9
        self.if_interface = int(round((xc_end - xf_start) / h_f))  # fine node at the coarse boundary
        assert abs(self.xf[self.if_interface] - xc_end) < 1e-9
        self.exact = lambda x, t: gaussian_exact(x, t, phi, sigma0, x0, v, D)
        # D1Q2 in lattice units of the fine grid
        self.vl = v * self.dt_f / h_f
        self.tau = 0.5 + D * self.dt_f / h_f ** 2
        # coarse matrices
        n = nc + 1
        M = np.zeros((n, n))
        K = np.zeros((n, n))
        me = h_c / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
        ke = (v / 2.0 * np.array([[-1.0, 1.0], [-1.0, 1.0]])            # int N_a v dN_b/dx
              + D / h_c * np.array([[1.0, -1.0], [-1.0, 1.0]]))           # int D dN_a/dx dN_b/dx
        for e in range(nc):
            M[e:e + 2, e:e + 2] += me
            K[e:e + 2, e:e + 2] += ke
        A = M + 0.5 * self.dt_c * K
        self.B = diags([np.diag(M - 0.5 * self.dt_c * K, k) for k in (-1, 0, 1)], [-1, 0, 1], format="csr")
        A[-1, :] = 0.0
        A[-1, -1] = 1.0
        # tridiagonal A in LAPACK band storage for scipy.linalg.solve_banded
        self.Ab = np.zeros((3, n))
        self.Ab[0, 1:] = np.diag(A, 1)
        self.Ab[1, :] = np.diag(A)
        self.Ab[2, :-1] = np.diag(A, -1)
        self.t = 0.0
        self.d = self.exact(self.xc, 0.0)
        self.fstar = self._collide(self._feq(self.exact(self.xf, 0.0)))

    # -- D1Q2 ----------------------------------------------------------------
    def _feq(self, u):
        return np.stack([0.5 * u * (1.0 + self.vl), 0.5 * u * (1.0 - self.vl)])

    def _collide(self, f):
        u = f[0] + f[1]
        return f + (self._feq(u) - f) / self.tau

    def _substep(self, fstar, up):
        f = np.empty_like(fstar)
        f[0, 1:] = fstar[0, :-1]                 # + population moves right
        f[1, :-1] = fstar[1, 1:]                 # - population moves left
        f[0, 0] = up - f[1, 0]                   # Dirichlet closure at the left end
        f[1, -1] = f[0, -1]                      # zero flux at x = 1
        return self._collide(f)

    # -- Algorithm 1 interface ----------------------------------------------
    def fine_to_coarse(self, fstar):
        return float(fstar[0, self.if_interface] + fstar[1, self.if_interface])

    def coarse_to_fine(self, d):
        return float(d[self.ic_interface])

    def coarse_step(self, d0, ufc):
        rhs = self.B @ d0
        rhs[-1] = ufc
        return solve_banded((1, 1), self.Ab, rhs)

    def lbm_substeps(self, fstar0, a, b):
        F = fstar0
        for j in range(1, self.eta + 1):
            lam = j / self.eta
            F = self._substep(F, (1.0 - lam) * a + lam * b)
        return F

    def step(self):
        algorithm1_step(self)
        self.t += self.dt_c

    def run(self, T):
        n = int(round(T / self.dt_c))
        for _ in range(n):
            self.step()
        return self

    def errors(self):
        """(E_c, E_f): max-norm errors on the coarse and fine nodes, eq. (Error1D)."""
        uf = self.fstar[0] + self.fstar[1]
        return (float(np.abs(self.d - self.exact(self.xc, self.t)).max()),
                float(np.abs(uf - self.exact(self.xf, self.t)).max()))
