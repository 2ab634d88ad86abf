"""Properties of the seeded input generators (no GPU)."""
import numpy as np

from paper_1601_02708_amd import configs, inputs


def test_disks_properties():
    N = 256
    pack = inputs.random_disks(N, 0.6, seed=3)
    assert 0.59 <= pack.porosity <= 0.6
    assert np.isclose(1 - pack.solid.mean(), pack.porosity)
    c, r = pack.centers, pack.radii
    assert np.all((r >= 6) & (r <= 20))
    # margin of 2 lattice units inside the patch
    assert np.all(c - r[:, None] >= 2 - 1e-12) and np.all(c + r[:, None] <= N - 1 - 2 + 1e-12)
    # surface gap >= 1
    d = np.hypot(c[:, None, 0] - c[None, :, 0], c[:, None, 1] - c[None, :, 1])
    gap = d - r[:, None] - r[None, :]
    np.fill_diagonal(gap, np.inf)
    assert gap.min() >= 1 - 1e-12
    # a frame two nodes wide along the patch boundary stays fluid
    s = pack.solid
    assert not s[:2].any() and not s[-2:].any() and not s[:, :2].any() and not s[:, -2:].any()


def test_generators_deterministic():
    a = inputs.random_disks(128, 0.7, seed=11)
    b = inputs.random_disks(128, 0.7, seed=11)
    assert np.array_equal(a.solid, b.solid)
    c = inputs.random_disks(128, 0.7, seed=12)
    assert not np.array_equal(a.solid, c.solid)


def test_stream_velocity_divergence_free_and_scaled():
    cfg = configs.SMALL.replace(N=200, M=10, porosity=0.7, velocity="stream")
    p = configs.build_problem(cfg)
    speed = np.hypot(p.vx.astype(float), p.vy.astype(float))
    fluid = p.solid == 0
    assert abs(speed[fluid].max() - 0.05) < 1e-7
    assert np.all(p.vx[~fluid] == 0) and np.all(p.vy[~fluid] == 0)
    # divergence of the analytic field (central differences, no solids)
    sf = inputs.stream_function(cfg.seed + 2000, p.L)
    X, Y = inputs.fine_coords(cfg.N)
    e = 1e-3
    div = (sf.velocity(X + e, Y)[0] - sf.velocity(X - e, Y)[0]) / (2 * e) + \
          (sf.velocity(X, Y + e)[1] - sf.velocity(X, Y - e)[1]) / (2 * e)
    vx, _ = sf.velocity(X, Y)
    assert np.abs(div).max() < 1e-6 * np.abs(vx).max()


def test_pulse_ranges():
    for seed in range(5):
        L = 126.0
        pu = inputs.gaussian_pulse(seed, L)
        assert 0.4 * L <= pu.xc <= 0.6 * L and 0.4 * L <= pu.yc <= 0.6 * L
        assert 0.05 * L <= pu.sigma <= 0.1 * L
        assert pu(pu.xc, pu.yc) == 1.0
