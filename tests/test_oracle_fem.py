"""Pins of the oracle's coarse FEM and grid transfers (no GPU): closed-form
element matrices, exactness and convergence properties fixed by the
mathematics, and a direct solver checked against numpy."""
import math

import numpy as np
import pytest

# local node a -> (ax, ay) in the element's tensor-product index
AXY = [(0, 0), (1, 0), (1, 1), (0, 1)]


def _tensor(Ax, Ay):
    return np.array([[Ax[a[0], b[0]] * Ay[a[1], b[1]] for b in AXY] for a in AXY])


def _closed_forms(h):
    """Exact integrals of products of 1-D linear shape functions on [0, h]."""
    m = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])        # int N_a N_b
    c = np.array([[-0.5, 0.5], [-0.5, 0.5]])                 # int N_a N_b'
    s = 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])        # int N_a' N_b'
    Mass = _tensor(m, m)
    Ax = _tensor(c, m)            # int N_a dN_b/dx
    Ay = _tensor(m, c)
    Sxx = _tensor(s, m)
    Syy = _tensor(m, s)
    Sxy = _tensor(c.T, c)         # int dN_a/dx dN_b/dy
    return Mass, Ax, Ay, Sxx, Syy, Sxy


def test_supg_chi(orc):
    """chi(a) = coth a - 1/a (eq. SUPG_tau) against a 50-digit evaluation."""
    import mpmath
    mpmath.mp.dps = 50
    for a in [1e-9, 1e-6, 1e-4, 1e-3, 0.05, 0.0999, 0.1, 0.3, 0.7, 2.0, 10.0, 50.0, 500.0]:
        ref = float(mpmath.coth(mpmath.mpf(a)) - 1 / mpmath.mpf(a))
        assert abs(orc.supg_chi(a) - ref) <= 1e-13 * ref, a


@pytest.mark.parametrize("supg", [0, 1])
def test_element_matrices_closed_form(orc, supg):
    h, D, k = 2.5, 0.03, 0.02
    v = np.array([0.4, -0.15])
    Mass, Ax, Ay, Sxx, Syy, Sxy = _closed_forms(h)
    Me, Ke, Mse, Kse = orc.fem_element(h, D, k, supg, np.tile(v, (4, 1)))
    assert np.allclose(Me, Mass, rtol=1e-14, atol=1e-15)
    Cv = v[0] * Ax + v[1] * Ay
    assert np.allclose(Ke, Cv + D * (Sxx + Syy) + k * Mass, rtol=1e-13, atol=1e-15)
    if supg:
        speed = np.hypot(*v)
        tau = h / (2 * speed) * orc.supg_chi(speed * h / (2 * D))
        assert np.allclose(Mse, tau * Cv.T, rtol=1e-13, atol=1e-16)
        streamline = v[0] ** 2 * Sxx + v[1] ** 2 * Syy + v[0] * v[1] * (Sxy + Sxy.T)
        assert np.allclose(Kse, tau * (streamline + k * Cv.T), rtol=1e-13, atol=1e-16)
    else:
        assert not Mse.any() and not Kse.any()
    # textbook numbers: Q1 mass h^2/36 [4 2 1 2], Laplacian [2/3 -1/6 -1/3 -1/6]
    assert np.allclose(Mass[0], h * h / 36 * np.array([4, 2, 1, 2]))
    assert np.allclose((Sxx + Syy)[0], [2 / 3, -1 / 6, -1 / 3, -1 / 6])


def test_band_lu_matches_numpy(orc):
    M = 5
    n = (M + 1) ** 2
    rng = np.random.default_rng(4)
    A = np.zeros((n, n))
    for i in range(n):
        for j in range(max(0, i - M - 2), min(n, i + M + 3)):
            A[i, j] = rng.standard_normal()
    # rows that force pivoting: tiny diagonal
    A[3, 3] = 1e-12
    A[10, :] = 0.0
    A[10, 10] = 1.0
    b = rng.standard_normal(n)
    x = orc.band_solve(M, A, b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)


def _boundary_nodes(M):
    s = M + 1
    kk, ll = np.meshgrid(np.arange(s), np.arange(s), indexing="xy")
    idx = (ll * s + kk).ravel()
    on = ((kk == 0) | (kk == M) | (ll == 0) | (ll == M)).ravel()
    return np.sort(idx[on]), kk.ravel(), ll.ravel()


@pytest.mark.parametrize("supg", [0, 1])
def test_patch_test(orc, supg):
    """P8: u = a + b (x - vx t) + c (y - vy t) with uniform v solves the ADE
    exactly; Q1 reproduces it in space, the trapezoid in time, and the SUPG
    residual vanishes, so one step is exact."""
    M, L, D, dt = 6, 12.0, 0.05, 0.7
    v = (0.3, -0.2)
    h = L / M
    rows, kk, ll = _boundary_nodes(M)
    X, Y = kk * h, ll * h
    exact = lambda t: 1.0 + 0.3 * (X - v[0] * t) - 0.2 * (Y - v[1] * t)
    vn = np.tile(np.asarray(v), ((M + 1) ** 2, 1))
    st = orc.FemStepper(M, L, D, 0.0, dt, supg, vn, rows)
    d1 = st.step(exact(0.3), exact(0.3 + dt)[rows])
    assert np.allclose(d1, exact(0.3 + dt), rtol=1e-12, atol=1e-13)


def test_uniform_reaction_decay(orc):
    """A uniform field decays by (1 - k dt/2)/(1 + k dt/2) per trapezoidal
    step (P2, coarse side), with SUPG active."""
    M, L, D, dt, k = 5, 10.0, 0.01, 2.0, 0.03
    rows, _, _ = _boundary_nodes(M)
    vn = np.tile([0.05, 0.02], ((M + 1) ** 2, 1))
    st = orc.FemStepper(M, L, D, k, dt, 1, vn, rows)
    r = (1 - k * dt / 2) / (1 + k * dt / 2)
    d = np.full((M + 1) ** 2, 2.0)
    for n in range(1, 6):
        d = st.step(d, np.full(len(rows), 2.0 * r ** n))
    assert np.allclose(d, 2.0 * r ** 5, rtol=1e-13)


def test_heat_mode_second_order(orc):
    """Pure diffusion of sin(pi x/L) sin(pi y/L) with u = 0 walls: the Q1 +
    trapezoid error at fixed T falls as h^2."""
    L, D, T, nt = 1.0, 0.1, 0.3, 120
    errs = []
    for M in (8, 16, 32):
        h = L / M
        rows, kk, ll = _boundary_nodes(M)
        X, Y = kk * h, ll * h
        u0 = np.sin(np.pi * X / L) * np.sin(np.pi * Y / L)
        st = orc.FemStepper(M, L, D, 0.0, T / nt, 0, np.zeros(((M + 1) ** 2, 2)), rows)
        d = u0.copy()
        for _ in range(nt):
            d = st.step(d, np.zeros(len(rows)))
        errs.append(np.abs(d - u0 * math.exp(-2 * D * math.pi ** 2 * T / L ** 2)).max())
    orders = np.log2(np.asarray(errs[:-1]) / np.asarray(errs[1:]))
    assert np.all((orders > 1.8) & (orders < 2.3)), orders


# ----------------------------------------------------------------------------
# grid transfers (P9)
# ----------------------------------------------------------------------------

def test_fem_interpolant_exact_on_bilinear(orc):
    M, L = 7, 21.0
    s = M + 1
    kk, ll = np.meshgrid(np.arange(s), np.arange(s), indexing="xy")
    g = lambda x, y: 0.3 + 0.2 * x - 0.1 * y + 0.05 * x * y
    d = g(kk * L / M, ll * L / M).ravel()
    rng = np.random.default_rng(8)
    X, Y = rng.uniform(0, L, 200), rng.uniform(0, L, 200)
    # bilinear in each element -> exact for any bilinear g
    assert np.allclose(orc.fem_interpolate(M, L, d, X, Y), g(X, Y), rtol=1e-13, atol=1e-13)


def test_fine_to_coarse_exact_and_solids(orc):
    N = 12
    jj, ii = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    g = lambda x, y: 1.0 + 0.5 * x - 0.25 * y + 0.125 * x * y
    u = g(ii, jj).astype(float)
    rng = np.random.default_rng(9)
    px, py = rng.uniform(0, N - 1, 100), rng.uniform(0, N - 1, 100)
    assert np.allclose(orc.fine_to_coarse(N, None, u, px, py), g(px, py), rtol=1e-14)
    # solid corners: a constant field stays exact under the renormalised weights
    solid = np.zeros((N, N), np.uint8)
    solid[4:8, 4:8] = 1
    uc = np.where(solid, 0.0, 3.0)
    assert np.allclose(orc.fine_to_coarse(N, solid, uc, [3.5, 7.5, 5.2], [4.5, 3.4, 7.9]), 3.0)
    # one fluid corner left: its value alone
    uf = np.arange(N * N, dtype=float).reshape(N, N)
    assert np.isclose(orc.fine_to_coarse(N, solid, uf, [3.8], [5.0])[0], uf[5, 3], rtol=1e-15)
    # all four corners solid: nearest fluid node; (i, j) = (3, 5) and (3, 6)
    # tie at distance 2.4515..., the lower index j*N + i wins
    got = orc.fine_to_coarse(N, solid, uf, [5.4], [5.5])
    assert got[0] == uf[5, 3]


def test_transfer_orders(orc):
    """c->f transfer error O(h^2) in the mesh size (as in Table FEM2LBM), and
    f->c transfer error O(h'^2) in the lattice spacing (bilinear
    interpolation of nodal samples)."""
    L = 1.0
    g = lambda x, y: np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
    rng = np.random.default_rng(10)
    X, Y = rng.uniform(0, L, 400), rng.uniform(0, L, 400)
    e = []
    for M in (10, 20, 40):
        s = M + 1
        kk, ll = np.meshgrid(np.arange(s), np.arange(s), indexing="xy")
        d = g(kk * L / M, ll * L / M).ravel()
        e.append(np.abs(orc.fem_interpolate(M, L, d, X, Y) - g(X, Y)).max())
    o = np.log2(np.asarray(e[:-1]) / np.asarray(e[1:]))
    assert np.all(o > 1.7), o
    e = []
    for N in (21, 41, 81):
        hp = L / (N - 1)
        jj, ii = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        u = g(ii * hp, jj * hp)
        e.append(np.abs(orc.fine_to_coarse(N, None, u, X / hp, Y / hp) - g(X, Y)).max())
    o = np.log2(np.asarray(e[:-1]) / np.asarray(e[1:]))
    assert np.all(o > 1.7), o
