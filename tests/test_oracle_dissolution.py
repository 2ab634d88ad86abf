"""Pins of the oracle's dissolving-solid model (surface reaction at
fluid-solid links, per-solid mass, solid-to-fluid conversion at the commit):
closed forms, the mass balance the reaction must satisfy, the reduction to
plain bounce-back, the adjoint's dot-product identity with the reaction."""
import numpy as np
import pytest

from paper_1601_02708_amd import configs


def _box(orc, N=16, kappa=0.3, c_sat=0.8, k=0.0, seed=1, periodic=True):
    rng = np.random.default_rng(seed)
    solid = np.zeros((N, N), np.uint8)
    solid[5:8, 6:10] = 1
    solid[11, 3] = 1
    vx = rng.uniform(-0.05, 0.05, (N, N))
    vy = rng.uniform(-0.05, 0.05, (N, N))
    vx[solid != 0] = 0
    vy[solid != 0] = 0
    lat = orc.Lattice(N, 0.8, vx, vy, solid=solid, k=k, periodic_x=periodic, periodic_y=periodic,
                      kappa_s=kappa, c_sat=c_sat)
    f = rng.uniform(0.01, 0.2, (9, N, N))
    f[:, solid != 0] = 0.0
    return lat, solid, f, rng


def test_no_reaction_is_plain_bounce_back(orc):
    lat, solid, f, _ = _box(orc, kappa=0.0)
    plain = orc.Lattice(lat.N, lat.tau, lat.vx, lat.vy, solid=solid, periodic_x=True, periodic_y=True)
    assert np.array_equal(lat.substep(f)[0], plain.substep(f)[0])
    from oracle.dissolution import link_flux
    assert not link_flux(lat, f, solid).any()


def test_reflected_population_closed_form(orc):
    """Next to a solid node the pulled population is the node's own opposite
    one relaxed towards w_q c_sat."""
    lat, solid, f, _ = _box(orc)
    ex, ey, w, opp = orc.d2q9()
    g, _ = lat.stream(f)
    # node (row 6, column 10) sits right of the block (columns 6..9)
    j, i = 6, 10
    assert solid[j, i] == 0 and solid[j, i - 1] != 0
    q = [n for n in range(9) if ex[n] == 1 and ey[n] == 0][0]     # pulls from (6, 9), solid
    expect = (1 - lat.kappa_s) * f[opp[q], j, i] + lat.kappa_s * w[q] * lat.c_sat
    assert abs(g[q, j, i] - expect) <= 1e-15


def test_fluid_mass_gains_exactly_the_link_flux(orc):
    """Periodic box, k = 0: BGK conserves mass and bounce-back returns what
    it receives, so the fluid's total changes by the summed link flux."""
    from oracle.dissolution import link_flux
    lat, solid, f, _ = _box(orc, k=0.0)
    f1, _ = lat.substep(f)
    gain = f1[:, solid == 0].sum() - f[:, solid == 0].sum()
    assert abs(gain - link_flux(lat, f, solid).sum()) <= 1e-13 * f.sum()


def test_adjoint_dot_product_with_reaction(orc):
    """With c_sat = 0 (and a periodic box) the reactive step is linear:
    <c, F(x)> = <F^T c, x> holds with the reaction's 1 - kappa_s factor."""
    lat, solid, f, rng = _box(orc, c_sat=0.0)
    N = lat.N
    x = rng.standard_normal((9, N, N))
    x[:, solid != 0] = 0.0
    c = rng.standard_normal((9, N, N))
    lhs = float(np.sum(c * lat.substep(x)[0]))
    lam, _, _ = lat.adjoint_substep(np.zeros_like(x), None, c)
    assert abs(lhs - float(np.sum(lam * x))) <= 1e-12 * max(1.0, abs(lhs))


def test_convert_closed_form(orc):
    from oracle.dissolution import convert
    N = 8
    solid = np.zeros((N, N), np.uint8)
    solid[3, 3] = solid[3, 4] = 1
    mass = np.zeros((N, N))
    mass[3, 3], mass[3, 4] = 0.5, 0.5
    flux = np.zeros((N, N))
    flux[3, 3], flux[3, 4] = 0.6, 0.2
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, (9, N, N))
    f[:, solid != 0] = 0
    kf = np.full((N, N), 0.01)
    f2, s2, m2, n = convert(f, solid, mass, flux, kf)
    assert n == 1 and s2[3, 3] == 0 and s2[3, 4] == 1
    assert m2[3, 3] == 0.0 and abs(m2[3, 4] - 0.3) <= 1e-15
    u = f.sum(axis=0) / (1 - kf)
    nb = [u[j, i] for j in (2, 3, 4) for i in (2, 3, 4) if (j, i) != (3, 3) and solid[j, i] == 0]
    _, _, w, _ = orc.d2q9()
    assert np.allclose(f2[:, 3, 3], w * np.mean(nb) * 0.99, rtol=0, atol=1e-15)
    assert np.array_equal(f2[:, solid == 0], f[:, solid == 0])


def test_dissolving_hybrid_invariants(orc):
    """A run in which solids dissolve: the solid set only shrinks, the
    converted count matches and the remaining masses stay positive."""
    from oracle.dissolution import DissolvingHybrid
    p = configs.build_problem(configs.PORE2048.replace(N=65, M=16, eta=3))
    rng = np.random.default_rng(7)
    mass = rng.uniform(0.002, 0.01, p.solid.shape)
    o = DissolvingHybrid(p, mass, kappa_s=0.2, c_sat=1.0)
    n0 = int(o.solid.sum())
    prev = o.solid.copy()
    for _ in range(4):
        o.step()
        assert np.all(o.solid <= prev)
        prev = o.solid.copy()
        assert np.all(o.mass[o.solid != 0] > 0.0)
    assert o.converted == n0 - int(o.solid.sum()) and o.converted > 0
