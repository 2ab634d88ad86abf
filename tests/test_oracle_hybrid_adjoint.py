"""Pins of the oracle's reverse mode of one coarse step of Algorithm 1.

Every transpose is checked against its forward map (the oracle's C
functions and banded solve) by the dot-product identity <c, G x> =
<G^T c, x>; the whole step (linear with zero outer data and no clamp) by
the same identity against HybridOracle.step; the reaction-rate gradient by
central differences (the step is a polynomial in each node's rate)."""
import numpy as np
import pytest

from paper_1601_02708_amd import configs


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


@pytest.fixture(scope="module")
def small(orc):
    from oracle.hybrid_adjoint import HybridStepAdjoint
    p = configs.build_problem(configs.SMALL.replace(k=2e-3))
    o = orc.HybridOracle(p)
    return p, o, HybridStepAdjoint(o)


@pytest.fixture(scope="module")
def pore(orc):
    from oracle.hybrid_adjoint import HybridStepAdjoint
    p = configs.build_problem(configs.PORE2048.replace(N=97, M=16, eta=3))
    o = orc.HybridOracle(p)
    return p, o, HybridStepAdjoint(o)


def test_c2f_transpose(small):
    p, o, adj = small
    rng = np.random.default_rng(1)
    d = rng.standard_normal((o.M + 1) ** 2)
    g = rng.standard_normal(4 * (o.N - 1))
    assert _rel(float(g @ o.coarse_to_fine(d)), float(adj.c2f_T(g) @ d)) <= 1e-13


@pytest.mark.parametrize("case", ["small", "pore"])
def test_f2c_transpose_and_rate(request, case):
    p, o, adj = request.getfixturevalue(case)
    rng = np.random.default_rng(2)
    f = rng.uniform(0.0, 1.0, (9, o.N, o.N))
    lam = rng.standard_normal(len(o.fc))
    lf, gk = adj.f2c_T(lam, f)
    assert _rel(float(lam @ o.fine_to_coarse(f)), float(np.sum(lf * f))) <= 1e-13
    # dJ/dk by central differences of the forward transfer in one node's rate
    fluid = np.flatnonzero(adj.fluid)
    used = [n for n in fluid if gk.flat[n] != 0.0][:3]
    assert used
    for n in used:
        eps = 1e-6
        vals = []
        for s in (1, -1):
            kf = adj.kfield.copy()
            kf[n] += s * eps
            u = np.where(adj.fluid, f.reshape(9, -1).sum(0) / (1.0 - kf), 0.0).reshape(o.N, o.N)
            vals.append(float(lam @ orc_f2c(o, u)))
        assert _rel((vals[0] - vals[1]) / (2 * eps), float(gk.flat[n])) <= 1e-7


def orc_f2c(o, u):
    from oracle import fine_to_coarse
    return fine_to_coarse(o.N, o.p.solid, u, o.fc_px, o.fc_py)


def test_f2c_transpose_with_all_solid_corners(orc):
    """Points whose four lattice corners are solid take the nearest fluid
    node; dropped corners renormalise the others."""
    from oracle import fine_to_coarse
    from oracle.hybrid_adjoint import f2c_weights
    N = 24
    solid = np.zeros((N, N), np.uint8)
    solid[5:12, 6:13] = 1          # a block around (9.3, 8.6) and its neighbourhood
    solid[15, 15] = 1              # one solid corner
    px = np.array([9.3, 15.4, 3.5, 12.9])
    py = np.array([8.6, 14.7, 3.2, 6.1])
    rows = f2c_weights(N, solid, px, py)
    assert len(rows[0][0]) == 1 and len(rows[1][0]) == 3
    rng = np.random.default_rng(3)
    u = rng.standard_normal((N, N))
    lam = rng.standard_normal(len(px))
    back = np.zeros(N * N)
    for (nd, w), l in zip(rows, lam):
        for n, wn in zip(nd, w):
            back[n] += wn * l
    assert _rel(float(lam @ fine_to_coarse(N, solid, u, px, py)), float(back @ u.reshape(-1))) <= 1e-13


@pytest.mark.parametrize("case", ["small", "pore"])
def test_coarse_solve_transpose(request, case):
    p, o, adj = request.getfixturevalue(case)
    rng = np.random.default_rng(4)
    d = rng.standard_normal((o.M + 1) ** 2)
    vals = rng.standard_normal(len(o.rows_sorted))
    lam = rng.standard_normal((o.M + 1) ** 2)
    ld, lv = adj.coarse_T(lam)
    lhs = float(lam @ o.fem.step(d, vals))
    assert _rel(lhs, float(ld @ d) + float(lv @ vals)) <= 1e-11


@pytest.mark.parametrize("case", ["small", "pore"])
def test_recorded_forward_is_the_step(request, case):
    p, o, adj = request.getfixturevalue(case)
    F, d = o.fstar.copy(), o.d.copy()
    F1, d1, _ = adj.forward(F, d)
    o2 = type(o)(p)
    o2.fstar, o2.d = F.copy(), d.copy()
    o2.step()
    assert np.array_equal(F1, o2.fstar) and np.array_equal(d1, o2.d)


@pytest.mark.parametrize("case", ["small", "pore"])
def test_step_dot_product_identity(request, case):
    """<(lam_f, lam_d), Step(F, d)> = <lam_F, F> + <lam_dn, d>: the step is
    linear (zero outer data, no clamp)."""
    p, o, adj = request.getfixturevalue(case)
    rng = np.random.default_rng(5)
    F = rng.uniform(0.0, 0.2, (9, o.N, o.N))
    if p.solid is not None:
        F[:, p.solid != 0] = 0.0
    d = rng.standard_normal((o.M + 1) ** 2)
    lam_f = rng.standard_normal((9, o.N, o.N))
    if p.solid is not None:
        lam_f[:, p.solid != 0] = 0.0
    lam_d = rng.standard_normal((o.M + 1) ** 2)
    F1, d1, tape = adj.forward(F, d)
    lF, ld, _ = adj.adjoint(tape, lam_f, lam_d)
    lhs = float(np.sum(lam_f * F1)) + float(lam_d @ d1)
    rhs = float(np.sum(lF * F)) + float(ld @ d)
    assert _rel(lhs, rhs) <= 1e-11, (lhs, rhs)


@pytest.mark.parametrize("case", ["small", "pore"])
def test_step_dot_product_identity_with_substep_cotangent(request, case):
    """An objective that also reads every intermediate fine state of the
    committed pass, J = <lam_f, F1> + <lam_d, d1> + sum_{j=1}^{eta-1}
    <w, f*(t_n + j)>, against the adjoint with lam_sub = w (linear step)."""
    p, o, adj = request.getfixturevalue(case)
    rng = np.random.default_rng(15)
    F = rng.uniform(0.0, 0.2, (9, o.N, o.N))
    if p.solid is not None:
        F[:, p.solid != 0] = 0.0
    d = rng.standard_normal((o.M + 1) ** 2)
    lam_f = rng.standard_normal((9, o.N, o.N))
    w = rng.standard_normal((9, o.N, o.N))
    if p.solid is not None:
        lam_f[:, p.solid != 0] = 0.0
        w[:, p.solid != 0] = 0.0
    lam_d = rng.standard_normal((o.M + 1) ** 2)
    F1, d1, tape = adj.forward(F, d)
    states = tape["passes"][-1]["states"]
    lF, ld, _ = adj.adjoint(tape, lam_f, lam_d, lam_sub=w)
    lhs = float(np.sum(lam_f * F1)) + float(lam_d @ d1) + sum(float(np.sum(w * s)) for s in states[1:-1])
    rhs = float(np.sum(lF * F)) + float(ld @ d)
    assert _rel(lhs, rhs) <= 1e-11, (lhs, rhs)
    lF0, _, _ = adj.adjoint(tape, lam_f, lam_d)
    assert not np.allclose(lF, lF0)


def test_step_rate_gradient_by_central_differences(small, orc):
    from oracle.hybrid_adjoint import HybridStepAdjoint
    p, o, adj = small
    rng = np.random.default_rng(6)
    F = rng.uniform(0.0, 0.2, (9, o.N, o.N))
    d = rng.standard_normal((o.M + 1) ** 2)
    lam_f = rng.standard_normal((9, o.N, o.N))
    lam_d = rng.standard_normal((o.M + 1) ** 2)
    _, _, tape = adj.forward(F, d)
    _, _, gk = adj.adjoint(tape, lam_f, lam_d)
    dk = rng.standard_normal((o.N, o.N))
    k0 = adj.kfield.reshape(o.N, o.N)
    eps = 1e-5

    def J(kf):
        o2 = orc.HybridOracle(p)
        o2.lat = orc.Lattice(o.N, o.lat.tau, o.lat.vx, o.lat.vy, solid=p.solid, k=kf)
        a2 = HybridStepAdjoint(o2)
        F1, d1, _ = a2.forward(F, d)
        return float(np.sum(lam_f * F1)) + float(lam_d @ d1)

    fd = (J(k0 + eps * dk) - J(k0 - eps * dk)) / (2 * eps)
    assert _rel(fd, float(np.sum(gk * dk))) <= 1e-7


def test_outer_value_gradient_by_central_differences(small, orc):
    """dJ/d(outer Dirichlet value): the step is affine in the prescribed
    outer value g, so sum_nodes dJ/dg equals the central difference of J in
    a uniform g (exact up to rounding)."""
    from oracle.hybrid_adjoint import HybridStepAdjoint
    p, o, adj = small
    rng = np.random.default_rng(7)
    F = rng.uniform(0.0, 0.2, (9, o.N, o.N))
    d = rng.standard_normal((o.M + 1) ** 2)
    lam_f = rng.standard_normal((9, o.N, o.N))
    lam_d = rng.standard_normal((o.M + 1) ** 2)
    _, _, tape = adj.forward(F, d)
    _, _, _, g_outer = adj.adjoint(tape, lam_f, lam_d, outer=True)
    assert np.all(g_outer[o.fc] == 0.0)

    def J(g):
        o2 = orc.HybridOracle(p, outer_value=g)
        o2.fstar, o2.d = F.copy(), d.copy()
        o2.step()
        return float(np.sum(lam_f * o2.fstar)) + float(lam_d @ o2.d)

    fd = (J(0.1) - J(-0.1)) / 0.2
    assert _rel(fd, float(g_outer.sum())) <= 1e-9
