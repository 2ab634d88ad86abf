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


def test_pore_flow_vanishes_at_grains_and_is_divergence_free():
    """v = curl(psi phi): zero on and inside the grains, the rotated
    gradient of psi phi (so divergence-free), and the plain stream-function
    flow farther than the wall width from every grain."""
    L = 400.0
    sf = inputs.stream_function(11, L)
    centers = np.array([[150.0, 160.0], [182.0, 160.0], [260.0, 250.0]])
    radii = np.array([12.0, 15.0, 9.0])
    flow = inputs.PoreFlow(sf, centers, radii, width=6.0)
    ax = np.arange(100.0, 300.0, 0.5)
    vx, vy = flow.velocity_grid(ax, ax)
    Y, X = np.meshgrid(ax, ax, indexing="ij")
    dist = np.min([np.hypot(X - c[0], Y - c[1]) - r for c, r in zip(centers, radii)], axis=0)
    speed = np.hypot(vx, vy)
    assert speed[dist <= 0].max() == 0.0
    # continuity at the surface: phi and its gradient vanish there, so the
    # speed fades to zero approaching a grain
    assert speed[(dist > 0) & (dist < 0.1)].max() < 0.1 * speed.max()
    assert speed[(dist > 0) & (dist < 0.1)].max() < speed[(dist > 0.4) & (dist < 0.6)].max()
    # far field equals the stream-function flow
    ux, uy = sf.velocity(X, Y)
    far = dist > 6.0
    assert np.allclose(vx[far], ux[far], atol=1e-15) and np.allclose(vy[far], uy[far], atol=1e-15)
    # v is the rotated gradient of psi * phi: compare with central differences
    phi, _, _ = inputs.wall_factor(ax, ax, centers, radii, 6.0)
    chi = sf.psi(X, Y) * phi
    h = ax[1] - ax[0]
    dchi_dy = (chi[2:, 1:-1] - chi[:-2, 1:-1]) / (2 * h)
    dchi_dx = (chi[1:-1, 2:] - chi[1:-1, :-2]) / (2 * h)
    scale = speed.max()
    # central differences at h = 0.5 agree to O(h^2) of the layer scale
    assert np.abs(vx[1:-1, 1:-1] - dchi_dy).max() < 0.1 * scale
    assert np.abs(vy[1:-1, 1:-1] + dchi_dx).max() < 0.1 * scale
    ax2 = np.arange(100.0, 300.0, 0.25)
    vx2, vy2 = flow.velocity_grid(ax2, ax2)
    Y2, X2 = np.meshgrid(ax2, ax2, indexing="ij")
    phi2, _, _ = inputs.wall_factor(ax2, ax2, centers, radii, 6.0)
    chi2 = sf.psi(X2, Y2) * phi2
    err2 = np.abs(vx2[1:-1, 1:-1] - (chi2[2:, 1:-1] - chi2[:-2, 1:-1]) / 0.5).max()
    # the difference quotients converge to v (at least first order: the
    # smoothstep is C^1, its second derivative jumps at both ends)
    assert err2 < 0.6 * np.abs(vx[1:-1, 1:-1] - dchi_dy).max()
    # hence the discrete divergence is small next to |v| / h
    div = (vx[1:-1, 2:] - vx[1:-1, :-2]) / (2 * h) + (vy[2:, 1:-1] - vy[:-2, 1:-1]) / (2 * h)
    assert np.abs(div).max() < 5e-2 * scale / h


def test_pore_workload_velocity_stays_out_of_solids():
    cfg = configs.SMALL.replace(N=300, M=10, porosity=0.7, velocity="stream")
    p = configs.build_problem(cfg)
    solid = p.solid != 0
    assert np.abs(p.vx[solid]).max() == 0 and np.abs(p.vy[solid]).max() == 0
    sp = np.hypot(p.vx, p.vy)
    assert abs(float(sp[~solid].max()) - cfg.v_max) < 1e-7
    # fluid nodes next to a grain move slowly (the flow fades towards the surface)
    nb = np.zeros_like(solid)
    nb[1:-1, 1:-1] = solid[:-2, 1:-1] | solid[2:, 1:-1] | solid[1:-1, :-2] | solid[1:-1, 2:]
    adj = nb & ~solid
    assert float(sp[adj].max()) < 0.6 * cfg.v_max
