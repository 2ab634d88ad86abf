"""Pins of the oracle's coupling loop (Algorithm 1).  The hybrid result as
a whole has no printed 2-D value to compare with (the paper's 2-D
examples are figures only); these tests pin the pieces of the loop that a
closed form fixes."""
import dataclasses

import numpy as np

from paper_1601_02708_amd import configs


def _constant_problem(value, porosity=None, N=48, M=12):
    cfg = configs.SMALL.replace(N=N, M=M, porosity=porosity, velocity="stream" if porosity else "uniform",
                                v_uniform=(0.0, 0.0), eta=5)
    p = configs.build_problem(cfg)
    p.vx[:] = 0.0
    p.vy[:] = 0.0
    p.u0_fine[:] = value
    p.u0_fine[p.solid != 0] = 0.0
    p.u0_coarse[:] = value
    return p


def test_constant_state_is_preserved(orc):
    """A constant concentration with v = 0 on the lattice is a fixed point of
    every part of the loop: equilibrium populations stream onto themselves,
    bounce-back returns w_i u, the maxent closure returns w_i u^p, the
    transfers interpolate a constant exactly and the FEM step (any coarse
    velocity, no reaction) maps a constant with constant Dirichlet data to
    itself.  A mis-weighted transfer or eq. (MTS) whose weights do not add
    to one breaks it."""
    for porosity in (None, 0.75):
        p = _constant_problem(1.7, porosity)
        o = orc.HybridOracle(p, outer_value=1.7, max_iter=3)
        o.run(4)
        u = o.fine_concentration()
        fluid = p.solid == 0
        assert np.allclose(u[fluid], 1.7, rtol=1e-13)
        assert np.allclose(o.d, 1.7, rtol=1e-13)
        assert o.infeasible == 0


def test_interface_follows_mts_interpolation(orc):
    """After fine step j of a coarse step, every perimeter node carries the
    interface value of eq. (MTS), (1 - j/eta) a + (j/eta) b, exactly: the
    Dirichlet closure enforces sum f = u^p and the readout sum f*/(1 - k)
    returns that sum."""
    cfg = configs.SMALL.replace(N=32, M=8, eta=6, k=2e-3)
    p = configs.build_problem(cfg)
    o = orc.HybridOracle(p)
    rng = np.random.default_rng(3)
    P = 4 * (cfg.N - 1)
    a = 0.5 + rng.uniform(0, 1, P)
    b = 0.5 + rng.uniform(0, 1, P)
    ii, jj = orc.perimeter_nodes(cfg.N)
    F = o.fstar
    for j in range(1, cfg.eta + 1):
        lam = j / cfg.eta
        F, _ = o.lat.substep(F, (1 - lam) * a + lam * b)
        u = o.lat.concentration(F)
        assert np.allclose(u[jj, ii], (1 - lam) * a + lam * b, rtol=1e-13)


def test_schwarz_converges_by_finite_propagation(orc):
    """With the restart-from-t_n reading, the f->c data of iteration it >= 2
    are read at coarse nodes at least h_c lattice units inside the patch,
    which eta fine steps cannot reach from the perimeter when eta <= h_c
    (a D2Q9 population moves one node per step).  So iterations beyond the
    second change nothing, bit for bit, on the small workload (h_c = 7.875,
    eta = 4)."""
    p = configs.build_problem(configs.SMALL)
    o2 = orc.HybridOracle(p, max_iter=2).run(5)
    o3 = orc.HybridOracle(p, max_iter=3).run(5)
    o1 = orc.HybridOracle(p, max_iter=1).run(5)
    assert np.array_equal(o2.fstar, o3.fstar) and np.array_equal(o2.d, o3.d)
    assert not np.array_equal(o1.d, o2.d)


def test_coupling_consistent_resolved_pulse(orc):
    """Qualitative (the 2-D hybrid is parity-unpinned beyond its parts):
    with a pulse the coarse mesh resolves (sigma = 0.15 L), the coarse
    interpolant and the fine solution agree in the overlap to a few
    percent of the peak after 25 coarse steps."""
    from paper_1601_02708_amd import inputs
    p = configs.build_problem(configs.SMALL)
    pulse = inputs.Pulse(xc=0.5 * p.L, yc=0.5 * p.L, sigma=0.15 * p.L)
    X, Y = inputs.fine_coords(p.cfg.N)
    XC, YC = inputs.coarse_coords(p.cfg.M, p.L)
    p.u0_fine[:] = pulse(X, Y)
    p.u0_coarse[:] = pulse(XC, YC).ravel()
    o = orc.HybridOracle(p).run(25)
    u = o.fine_concentration()
    assert np.isfinite(u).all() and np.isfinite(o.d).all()
    N = p.cfg.N
    sl = slice(8, N - 8, 4)
    jj, ii = np.meshgrid(np.arange(N)[sl], np.arange(N)[sl], indexing="ij")
    uc = orc.fem_interpolate(p.cfg.M, p.L, o.d, p.x0 + ii.ravel(), p.y0 + jj.ravel())
    assert np.abs(uc - u[jj, ii].ravel()).max() < 0.08 * u.max()


def test_natural_outer_edges_keep_a_constant(orc):
    """With every outer edge natural (zero diffusive flux) and no flow or
    reaction, a constant state stays constant whatever the outer value;
    with Dirichlet edges at another value it does not."""
    from paper_1601_02708_amd import configs
    cfg = configs.SMALL.replace(v_uniform=(0.0, 0.0))
    p = configs.build_problem(cfg)
    c = 0.6
    p.u0_fine[:] = c
    p.u0_coarse[:] = c
    o = orc.HybridOracle(p, outer_value=0.0, outer_natural=15).run(3)
    assert np.abs(o.d - c).max() <= 1e-13
    assert np.abs(o.fine_concentration() - c).max() <= 1e-13
    o2 = orc.HybridOracle(p, outer_value=0.0, outer_natural=0).run(3)
    assert np.abs(o2.d - c).max() > 1e-2


def test_inlet_with_natural_edges_is_mirror_symmetric(orc):
    """Inlet edge x = 0 held at 1, the other three natural, flow along x:
    the problem is symmetric about y = L/2, and so is the solution
    (populations mirrored in y: q 2 <-> 4, 5 <-> 8, 6 <-> 7)."""
    from paper_1601_02708_amd import configs, inputs
    cfg = configs.SMALL.replace(v_uniform=(0.05, 0.0))
    p = configs.build_problem(cfg)
    pulse = inputs.Pulse(xc=0.45 * p.L, yc=0.5 * p.L, sigma=0.1 * p.L)
    X, Y = inputs.fine_coords(cfg.N)
    XC, YC = inputs.coarse_coords(cfg.M, p.L)
    p.u0_fine[:] = pulse(X, Y)
    p.u0_coarse[:] = pulse(XC, YC).ravel()
    o = orc.HybridOracle(p, outer_value=1.0, outer_natural=14).run(3)
    d = o.d.reshape(cfg.M + 1, cfg.M + 1)
    assert np.abs(d - d[::-1, :]).max() <= 1e-12 * np.abs(d).max()
    F = o.fstar
    mirror_q = [0, 1, 4, 3, 2, 8, 7, 6, 5]
    assert np.abs(F - F[mirror_q][:, ::-1, :]).max() <= 1e-12 * np.abs(F).max()
    assert np.abs(d[:, 0] - 1.0).max() <= 1e-12 and d[:, -1].max() < 0.99   # the inlet holds, the far edge is free
