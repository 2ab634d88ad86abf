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


# ----------------------------------------------------------------------------
# Algorithm 1 against the free-space advected Gaussian (closed form)
# ----------------------------------------------------------------------------

_TAU = 0.6                    # D_lattice = (tau - 1/2)/3 = 1/30
_D_PHYS = 1e-3                # in units of the unit square
_V_PHYS = (0.2, 0.05)
_C0, _S0 = (0.55, 0.47), 0.06


def _gaussian(X, Y, t, L):
    """The advected, spreading Gaussian of the ADE in free space, in the
    lattice units of a domain of side L (t in fine steps): with diffusive
    scaling a unit of physical time is D_phys L^2 / D_lattice fine steps."""
    Dl = (_TAU - 0.5) / 3.0
    vl = np.array(_V_PHYS) * Dl / _D_PHYS / L
    s0 = _S0 * L
    s2 = s0 ** 2 + 2.0 * Dl * t
    cx, cy = _C0[0] * L + vl[0] * t, _C0[1] * L + vl[1] * t
    return s0 ** 2 / s2 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * s2)), vl


def _gaussian_problem(L, eta):
    """Patch of L/2 + 1 nodes in a domain of side L (h_c = 4 h_f), uniform
    flow, the Gaussian as initial condition on both grids, outer Dirichlet
    0 (the pulse stays > 5 sigma from the outer edge)."""
    from paper_1601_02708_amd import inputs
    N, M = L // 2 + 1, L // 4
    cfg = configs.SMALL.replace(N=N, M=M, D=(_TAU - 0.5) / 3.0, eta=eta, max_iter=2, tau=_TAU)
    p = configs.build_problem(cfg)
    X, Y = inputs.fine_coords(N)
    XC, YC = inputs.coarse_coords(M, p.L)
    p.u0_fine, vl = _gaussian(X, Y, 0.0, p.L)
    p.u0_coarse = _gaussian(XC, YC, 0.0, p.L)[0].ravel()
    p.vx[:], p.vy[:] = vl[0], vl[1]
    p.vc[:, 0], p.vc[:, 1] = vl[0], vl[1]
    return p, (X, Y, XC, YC)


def _planted(kind):
    """Algorithm 1 with one planted mistake (test only)."""
    def step(h):
        ufc = h.fine_to_coarse(h.fstar)
        a = h.coarse_to_fine(h.d)
        F = h.fstar
        for _ in range(h.max_iter):
            d1 = h.coarse_step(h.d, ufc)
            b = h.coarse_to_fine(d1)
            if kind == "mts_swapped":                 # (j/eta) a + (1 - j/eta) b
                F = h.lbm_substeps(h.fstar, b, a)
            elif kind == "no_restart":                # each pass continues the last
                F = h.lbm_substeps(F, a, b)
            else:
                F = h.lbm_substeps(h.fstar, a, b)
            if kind != "f2c_from_t_n":                # f->c data always from f*(t_n)
                ufc = h.fine_to_coarse(F)
        h.fstar = F
        h.d = d1
    return step


def _gaussian_errors(orc, L, kind=None):
    """Max-norm errors (fine, coarse) of the hybrid at t = L^2/64 fine
    steps (0.52 time units), eta = L/16 so that the coarse step shrinks like
    h (Delta t_c = eta dt_f with dt_f ~ h^2)."""
    from oracle.hybrid import algorithm1_step
    eta = L // 16
    p, (X, Y, XC, YC) = _gaussian_problem(L, eta)
    o = orc.HybridOracle(p)
    n = L * L // 64
    step = algorithm1_step if kind is None else _planted(kind)
    for _ in range(n // eta):
        step(o)
    ef = float(np.abs(o.fine_concentration() - _gaussian(X, Y, n, p.L)[0]).max())
    ec = float(np.abs(o.d - _gaussian(XC, YC, n, p.L)[0].ravel()).max())
    return ef, ec


def _gaussian_pin(errs):
    """The bar: at L = 256 both errors below 3e-3 (about 2x the measured
    1.3e-3 / 1.0e-3) and, from L = 128 to 256, observed orders of at least
    1.4 (fine) and 1.5 (coarse); measured 1.6 and 2.0.  The paper reports
    first order for its coarse domain (Sec. 7.1); this loop does better."""
    (f1, c1), (f2, c2) = errs
    return f2 < 3e-3 and c2 < 3e-3 and np.log2(f1 / f2) >= 1.4 and np.log2(c1 / c2) >= 1.5


def test_algorithm1_converges_to_the_advected_gaussian(orc):
    """Algorithm 1 as a whole (Sec. 6.2: eq. MTS at every fine step, both
    transfers, the restart from t_n and the f->c data of the previous pass)
    on a pulse that advects and spreads across the patch's right interface,
    against the closed-form ADE solution, refined in space (h_f, h_c = 4 h_f)
    and in the coarse step (Delta t_c ~ h).  Every mistake planted in the
    loop's bookkeeping fails the bar (next test)."""
    errs = [_gaussian_errors(orc, L) for L in (128, 256)]
    print(f"\nfine/coarse max errors at L = 128, 256: {errs}")
    assert _gaussian_pin(errs), errs


def test_algorithm1_gaussian_pin_catches_planted_mistakes(orc):
    """Interface values of eq. (MTS) with a and b swapped, f->c data always
    taken from f*(t_n), or passes that do not restart from t_n: each lags
    the exchange by O(Delta t_c) (first order under this scaling) or
    advances the fine subdomain too far, and fails the bar."""
    for kind in ("mts_swapped", "f2c_from_t_n", "no_restart"):
        errs = [_gaussian_errors(orc, L, kind) for L in (128, 256)]
        print(f"\n{kind}: {errs}")
        assert not _gaussian_pin(errs), (kind, errs)
