"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle
on identical seeded inputs.  FP64 must agree to 1e-12 relative L2 (the
bound the method's specification sets); FP32 errors are reported and held
to a loose regression bound only."""
import functools

import numpy as np
import pytest

from paper_1601_02708_amd import configs, inputs

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_02708_amd import hyb
    return hyb


def rel_l2(a, b, mask=None):
    a, b = np.asarray(a, float), np.asarray(b, float)
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@functools.lru_cache(maxsize=None)
def problem(name, **over):
    cfg = configs.CONFIGS[name]
    if over:
        cfg = cfg.replace(**over)
    return configs.build_problem(cfg)


def _lattice_case(N, seed, porosity=0.7, k_field=False, tau=0.56, vmax=0.05):
    rng = np.random.default_rng(seed)
    solid = inputs.random_disks(N, porosity, seed=seed, r_min=2, r_max=6).solid if porosity < 1 else None
    vx = rng.uniform(-vmax, vmax, (N, N)).astype(np.float32)
    vy = rng.uniform(-vmax, vmax, (N, N)).astype(np.float32)
    if solid is not None:
        vx[solid != 0] = 0
        vy[solid != 0] = 0
    kf = rng.uniform(0, 2e-3, (N, N)) if k_field else None
    return solid, vx, vy, kf, tau


# ----------------------------------------------------------------------------
# single fine steps from random populations (lattice only)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N,clamp,k_field", [(67, 0, False), (130, 1, True), (3, 0, False), (4, 0, True)])
def test_substeps_random_state(orc, precision, N, clamp, k_field):
    hyb = _gpu()
    solid, vx, vy, kf, tau = _lattice_case(N, 100 + N, porosity=0.75 if N > 8 else 1.0, k_field=k_field)
    eta = 3
    rng = np.random.default_rng(N)
    P = 4 * (N - 1)
    kind = rng.integers(0, 2, P).astype(np.int8)
    a = rng.uniform(0.2, 1.5, P)
    b = rng.uniform(0.2, 1.5, P)
    # Neumann slots get small fluxes of both signs
    a[kind == 1] = rng.uniform(-0.05, 0.05, (kind == 1).sum())
    b[kind == 1] = rng.uniform(-0.05, 0.05, (kind == 1).sum())
    f0 = inputs.random_populations(N, 7 + N, lo=0.05, hi=0.4)
    if solid is not None:
        f0[:, solid != 0] = 0.0
    g = hyb.Hybrid(N=N, x0=0, y0=0, u0=np.zeros((N, N)), vx=vx, vy=vy, D=(tau - 0.5) / 3, eta=eta,
                   precision=precision, tau=tau, solid=solid, k=0.0 if k_field else 1e-3, k_field=kf,
                   bc_clamp=clamp)
    g.set_populations(f0)
    g.set_boundary(a, b, kind)
    lat = orc.Lattice(N, tau, vx.astype(np.float64), vy.astype(np.float64), solid=solid,
                      k=kf if k_field else 1e-3, bc_kind=kind, clamp=clamp)
    f = f0 if precision == "fp64" else f0.astype(np.float32).astype(np.float64)
    for j in range(1, eta + 1):
        g.lbm_substeps(1, restart=0)
        lam = j / eta
        f, _ = lat.substep(f, (1 - lam) * a + lam * b)
        got = g.get_populations()
        err = np.abs(got - f).max() / np.abs(f).max()
        tol = 1e-13 if precision == "fp64" else 2e-6
        assert err <= tol, (j, err)


def test_substeps_many_commits_fp64(orc):
    """200 fine steps in 20 coarse steps of 10 (Dirichlet + Neumann slots,
    solids, per-node reaction)."""
    hyb = _gpu()
    N = 96
    solid, vx, vy, kf, tau = _lattice_case(N, 5, k_field=True, tau=0.53)
    rng = np.random.default_rng(1)
    P = 4 * (N - 1)
    ii = np.arange(P)
    kind = (ii % 5 == 0).astype(np.int8)
    u0 = inputs.gaussian_pulse(3, N)(*np.meshgrid(np.arange(N) * 1.0, np.arange(N) * 1.0, indexing="xy"))
    g = hyb.Hybrid(N=N, x0=0, y0=0, u0=u0, vx=vx, vy=vy, D=(tau - 0.5) / 3, eta=10, tau=tau, solid=solid,
                   k_field=kf)
    lat = orc.Lattice(N, tau, vx.astype(float), vy.astype(float), solid=solid, k=kf, bc_kind=kind)
    f = lat.init(u0)
    a = rng.uniform(0, 0.2, P)
    for step in range(20):
        b = a + rng.uniform(-0.02, 0.02, P)
        av, bv = a.copy(), b.copy()
        av[kind == 1] = 0.0
        bv[kind == 1] = 0.0
        g.set_boundary(av, bv, kind)
        g.lbm_substeps(10, restart=1)
        g.commit()
        for j in range(1, 11):
            f, _ = lat.substep(f, (1 - j / 10) * av + j / 10 * bv)
        a = b
    fluid = solid == 0
    assert rel_l2(g.get_populations(), f, fluid) <= 1e-12
    assert rel_l2(g.concentration(), lat.concentration(f), fluid) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N,clamp,k_field,eta", [(67, 0, False, 5), (130, 1, True, 4), (3, 0, False, 3),
                                                  (4, 0, True, 2), (200, 0, False, 7), (65, 1, False, 6)])
def test_two_step_sweep(orc, precision, N, clamp, k_field, eta):
    """Fine steps taken in temporally blocked pairs (two steps per launch,
    plus a single step for an odd count) against the oracle and against the
    single-step sweep: random states, solids, every perimeter slot
    Dirichlet with interface values that make some closures infeasible.
    Sizes cover several tiles with ragged edges in x and y, and lattices
    smaller than one tile."""
    hyb = _gpu()
    solid, vx, vy, kf, tau = _lattice_case(N, 300 + N, porosity=0.75 if N > 8 else 1.0, k_field=k_field)
    rng = np.random.default_rng(3 * N + eta)
    P = 4 * (N - 1)
    a = rng.uniform(0.2, 1.5, P)
    b = rng.uniform(0.2, 1.5, P)
    f0 = inputs.random_populations(N, 11 + N, lo=0.05, hi=0.4)
    if solid is not None:
        f0[:, solid != 0] = 0.0
    lat = orc.Lattice(N, tau, vx.astype(np.float64), vy.astype(np.float64), solid=solid,
                      k=kf if k_field else 1e-3, clamp=clamp)
    f = f0 if precision == "fp64" else f0.astype(np.float32).astype(np.float64)
    bad = 0
    for j in range(1, eta + 1):
        lam = j / eta
        f, nb = lat.substep(f, (1 - lam) * a + lam * b)
        bad += nb
    assert bad > 0                      # the infeasible branch is exercised
    got = {}
    for spl in (1, 2):
        g = hyb.Hybrid(N=N, x0=0, y0=0, u0=np.zeros((N, N)), vx=vx, vy=vy, D=(tau - 0.5) / 3, eta=eta,
                       precision=precision, tau=tau, solid=solid, k=0.0 if k_field else 1e-3, k_field=kf,
                       bc_clamp=clamp)
        g.set_steps_per_launch(spl)
        g.set_populations(f0)
        g.set_boundary(a, b)
        g.lbm_substeps(eta, restart=1)
        g.commit()
        got[spl] = g.get_populations()
        assert g.stats()["infeasible"] == bad, spl
        err = np.abs(got[spl] - f).max() / np.abs(f).max()
        assert err <= (1e-13 if precision == "fp64" else 2e-6), (spl, err)
    d = np.abs(got[2] - got[1]).max() / np.abs(got[1]).max()
    assert d <= (1e-14 if precision == "fp64" else 1e-6), d


@pytest.mark.parametrize("N,clamp,k_field,eta", [(67, 0, False, 5), (130, 1, True, 9), (3, 0, False, 3),
                                                  (4, 0, True, 6), (200, 0, False, 7), (65, 1, False, 10),
                                                  (131, 0, True, 8)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("spl", [3, 4, 5])
def test_three_step_sweep(orc, spl, precision, N, clamp, k_field, eta):
    """Fine steps taken three or four per launch (hyb_set_steps_per_launch;
    the pass's plan with 3: eta = 5 -> 3 + 2, 9 -> 3 + 3 + 3, 3 -> 3,
    6 -> 3 + 3, 7 -> 3 + 2 + 2, 10 -> 3 + 3 + 2 + 2, 8 -> 3 + 3 + 2; with 4:
    5 -> 3 + 2, 9 -> 4 + 3 + 2, 3 -> 3, 6 -> 3 + 3, 7 -> 4 + 3, 10 -> 4 + 3 + 3,
    8 -> 4 + 4; with 5: 9 -> 5 + 4, 10 -> 5 + 5, 8 -> 4 + 4, 7 -> 4 + 3) against the oracle and against the single-step sweep: random states, solids, every perimeter
    slot Dirichlet with interface values that make some closures infeasible
    (counted once per owned node, as by single steps), ragged tiles and
    lattices smaller than one tile."""
    hyb = _gpu()
    solid, vx, vy, kf, tau = _lattice_case(N, 500 + N, porosity=0.75 if N > 8 else 1.0, k_field=k_field)
    rng = np.random.default_rng(7 * N + eta)
    P = 4 * (N - 1)
    a = rng.uniform(0.2, 1.5, P)
    b = rng.uniform(0.2, 1.5, P)
    f0 = inputs.random_populations(N, 13 + N, lo=0.05, hi=0.4)
    if solid is not None:
        f0[:, solid != 0] = 0.0
    lat = orc.Lattice(N, tau, vx.astype(np.float64), vy.astype(np.float64), solid=solid,
                      k=kf if k_field else 1e-3, clamp=clamp)
    f = f0 if precision == "fp64" else f0.astype(np.float32).astype(np.float64)
    bad = 0
    for j in range(1, eta + 1):
        lam = j / eta
        f, nb = lat.substep(f, (1 - lam) * a + lam * b)
        bad += nb
    assert bad > 0
    got = {}
    for s in (1, spl):
        g = hyb.Hybrid(N=N, x0=0, y0=0, u0=np.zeros((N, N)), vx=vx, vy=vy, D=(tau - 0.5) / 3, eta=eta,
                       precision=precision, tau=tau, solid=solid, k=0.0 if k_field else 1e-3, k_field=kf,
                       bc_clamp=clamp)
        g.set_steps_per_launch(s)
        g.set_populations(f0)
        g.set_boundary(a, b)
        g.lbm_substeps(eta, restart=1)
        g.commit()
        got[s] = g.get_populations()
        assert g.stats()["infeasible"] == bad, s
        err = np.abs(got[s] - f).max() / np.abs(f).max()
        assert err <= (1e-13 if precision == "fp64" else 2e-6), (s, err)
        g.close()
    d = np.abs(got[spl] - got[1]).max() / np.abs(got[1]).max()
    assert d <= (1e-14 if precision == "fp64" else 1e-6), d


@pytest.mark.parametrize("N", [97, 200])
@pytest.mark.parametrize("spl", [3, 4, 5])
def test_three_step_fp16s_matches_single_steps(spl, N):
    """FP16 shifted storage, three to five steps per launch: a launch keeps
    its intermediate states in FP32 and rounds to binary16 only at the
    store, single steps round after every step; the two agree to a few
    binary16 roundings.  At N = 200 some tiles' regions stay clear of the
    perimeter (the stages' interior copy); at N = 97 none does."""
    hyb = _gpu()
    eta = 10
    solid, vx, vy, kf, tau = _lattice_case(N, 777, porosity=0.7)
    rng = np.random.default_rng(778)
    P = 4 * (N - 1)
    a = rng.uniform(0.2, 0.6, P)
    b = rng.uniform(0.2, 0.6, P)
    u0 = np.full((N, N), 0.4)
    got = {}
    for s in (1, spl):
        g = hyb.Hybrid(N=N, x0=0, y0=0, u0=u0, vx=vx, vy=vy, D=(tau - 0.5) / 3, eta=eta, precision="fp16s",
                       tau=tau, solid=solid, k=1e-3)
        g.set_steps_per_launch(s)
        g.set_boundary(a, b)
        g.lbm_substeps(eta, restart=1)
        g.commit()
        got[s] = g.get_populations()
        g.close()
    d = np.abs(got[spl] - got[1]).max() / np.abs(got[1]).max()
    assert d <= 4e-3, d


@pytest.mark.parametrize("spl,over,steps,depths", [(3, {"N": 600, "M": 32}, 3, (1, 2, 3, 4)),
                                                   (3, {"N": 1026, "M": 32}, 2, (1, 2, 4)),
                                                   (3, {"N": 257, "M": 32, "eta": 7}, 3, (1, 2, 3)),
                                                   (4, {"N": 600, "M": 32}, 3, (1, 2, 3)),
                                                   (4, {"N": 1027, "M": 32}, 2, (1, 3)),
                                                   (4, {"N": 600, "M": 32, "eta": 9}, 2, (1, 2, 3)),
                                                   (5, {"N": 600, "M": 32}, 3, (1, 2)),
                                                   (5, {"N": 1029, "M": 32, "eta": 9}, 2, (1, 2))])
def test_three_step_overlapped_step_is_bit_identical(spl, over, steps, depths):
    """hyb_step with three-step launches (plan 3 + 3 + 2 + 2 at eta = 10,
    3 + 2 + 2 at eta = 7) and the deep tiles of the first launches on the
    side stream equals the serial order bit for bit at every depth; the
    pass's two-step launches take the rectangles of the three-step ones
    (at N = 1026 the one- and two-node-ring rectangles differ by a tile, so
    rectangles that did not nest would read unwritten tiles).  Against
    two-step launches the state agrees to FP32 rounding."""
    hyb = _gpu()
    p = problem("pore2048", **over)
    out = []
    for ov in (0,) + tuple(depths):
        g = hyb.Hybrid.from_problem(p, precision="fp32")
        g.set_steps_per_launch(spl)
        g.set_overlap(ov)
        for _ in range(steps):
            g.step(p.cfg.max_iter)
        out.append((g.get_populations(), g.concentration(hyb.HYB_COARSE), g.stats()["infeasible"]))
        g.close()
    for d, o in zip(depths, out[1:]):
        assert np.array_equal(o[0], out[0][0]), d
        assert np.array_equal(o[1], out[0][1]), d
        assert o[2] == out[0][2], d
    g = hyb.Hybrid.from_problem(p, precision="fp32")
    g.set_steps_per_launch(2)
    g.set_overlap(0)
    for _ in range(steps):
        g.step(p.cfg.max_iter)
    two = g.get_populations()
    fluid = p.solid == 0
    err = rel_l2(out[0][0], two, fluid)
    print(f"\nthree-step vs two-step launches, {over}: rel L2 {err:.2e}")
    assert err <= 1e-6, err


def test_three_steps_fp64_equal_two_steps():
    """FP64 storage, overlapped steps: three-step launches (512 lanes per
    workgroup) give the two-step launches' state bit for bit."""
    hyb = _gpu()
    p = problem("pore2048", N=257, M=32)
    out = []
    for spl in (2, 3):
        g = hyb.Hybrid.from_problem(p, precision="fp64")
        g.set_steps_per_launch(spl)
        g.set_overlap(2)
        for _ in range(2):
            g.step(p.cfg.max_iter)
        out.append(g.get_populations())
        g.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("name,over,precision,steps,depths",
                         [("small", {}, "fp64", 6, (1, 2)),
                          ("pore2048", {"N": 257, "M": 32}, "fp32", 4, (1, 2, 5)),
                          ("pore2048", {"N": 131, "M": 16, "eta": 5}, "fp64", 3, (1, 2, 3)),
                          ("pore2048", {"N": 600, "M": 32}, "fp32", 3, (1, 2, 3, 4, 5, 8)),
                          ("pore2048", {"N": 600, "M": 32, "eta": 7}, "fp64", 2, (2, 3, 4)),
                          ("pore4096", {"N": 1536}, "fp32", 3, (1, 2, 3))])
def test_overlapped_step_is_bit_identical(name, over, precision, steps, depths):
    """hyb_step with the deep tiles of each pass's first launches on the
    handle's side stream (overlapping the coarse solve) equals the serial
    order bit for bit, for every overlap depth (depths past eta / 2 are
    capped; 600^2 keeps the depth-3 rectangle non-empty, 257^2 empties it at
    depth 1); odd eta mixes two-step and single-step launches; with eta = 4
    and depth 2 every launch of a pass is split, so the pass must end by
    joining the side stream (large deep launches make a missing join show)."""
    hyb = _gpu()
    p = problem(name, **over)
    out = []
    for ov in (0,) + tuple(depths):
        g = hyb.Hybrid.from_problem(p, precision=precision)
        g.set_overlap(ov)
        for _ in range(steps):
            g.step(p.cfg.max_iter)
        out.append((g.get_populations(), g.concentration(hyb.HYB_COARSE), g.stats()["infeasible"]))
        g.close()
    for d, o in zip(depths, out[1:]):
        assert np.array_equal(o[0], out[0][0]), d
        assert np.array_equal(o[1], out[0][1]), d
        assert o[2] == out[0][2], d


def test_overlap_rejects_negative_depth():
    hyb = _gpu()
    N = 8
    z = np.zeros((N, N))
    g = hyb.Hybrid(N=N, x0=0, y0=0, u0=z, vx=z, vy=z, D=0.1, eta=2)
    g.set_overlap(hyb.HYB_OVERLAP_AUTO)
    with pytest.raises(hyb.HybError):
        g.set_overlap(-2)


@pytest.mark.parametrize("spl,D", [(2, 5), (3, 4), (4, 3), (5, 2)])
def test_overlap_auto_tunes_then_keeps_a_depth(spl, D):
    """HYB_OVERLAP_AUTO (the default): one serial step, then three rounds
    over depths 0 .. D (D = the pass's multi-step launches at eta = 10:
    5 pairs, or 3 + 3 + 2 + 2), then one depth in 0 .. D stays; the states
    equal the serial order's bit for bit throughout."""
    hyb = _gpu()
    p = problem("pore2048", N=600, M=32)
    n_tune = 1 + 3 * (D + 1)
    ref = hyb.Hybrid.from_problem(p, precision="fp32")
    ref.set_steps_per_launch(spl)
    ref.set_overlap(0)
    g = hyb.Hybrid.from_problem(p, precision="fp32")
    g.set_steps_per_launch(spl)
    assert g.stats()["overlap_depth"] == -1
    for k in range(n_tune + 2):
        ref.step(p.cfg.max_iter)
        g.step(p.cfg.max_iter)
        d = g.stats()["overlap_depth"]
        assert (d == -1) if k < n_tune - 1 else (0 <= d <= D), (k, d)
    assert np.array_equal(g.get_populations(), ref.get_populations())
    assert ref.stats()["overlap_depth"] == 0


def test_steps_per_launch_rejects_other_values():
    hyb = _gpu()
    N = 8
    z = np.zeros((N, N))
    g = hyb.Hybrid(N=N, x0=0, y0=0, u0=z, vx=z, vy=z, D=0.1, eta=2)
    for bad in (0, 6, -1):
        with pytest.raises(hyb.HybError):
            g.set_steps_per_launch(bad)


@pytest.mark.parametrize("clamp", [0, 1])
def test_paper_example_e01(orc, clamp):
    """Sec. 4.1.2 example on the GPU (Neumann at x = 0, Dirichlet 0
    elsewhere, tau ~ 1), Table LBM_p1 case 1 discretisation."""
    hyb = _gpu()
    D = 4 / (5 * np.pi ** 2)
    N, dt = 26, 3.3e-3
    h = 1 / (N - 1)
    n = int(np.floor(0.25 / dt))
    tau = 0.5 + 3 * D * dt / h ** 2
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = np.sin(np.pi * Y) * np.cos(np.pi * X / 2)
    ii, jj = orc.perimeter_nodes(N)
    kind = np.where((ii == 0) & (jj > 0) & (jj < N - 1), 1, 0).astype(np.int8)
    z = np.zeros((N, N), np.float32)
    g = hyb.Hybrid(N=N, x0=0, y0=0, u0=u0, vx=z, vy=z, D=1.0, eta=n, tau=tau, bc_clamp=clamp)
    g.set_boundary(np.zeros(4 * (N - 1)), None, kind)
    g.lbm_substeps(n, restart=1)
    g.commit()
    lat = orc.Lattice(N, tau, np.zeros((N, N)), np.zeros((N, N)), bc_kind=kind, clamp=clamp)
    f = lat.init(u0)
    for _ in range(n):
        f, _ = lat.substep(f, np.zeros(4 * (N - 1)))
    assert rel_l2(g.concentration(), lat.concentration(f)) <= 1e-12
    st = g.stats()
    assert st["infeasible"] > 0   # u = 0 walls are infeasible for f >= 0


def test_neumann_box_corners(orc):
    """All-Neumann box: flat edges are closed form, the corners (diagonal
    normal, mixed e.n) need the Newton iteration on the GPU and bisection in
    the oracle."""
    hyb = _gpu()
    N, tau = 40, 0.8
    rng = np.random.default_rng(9)
    vx = rng.uniform(-0.02, 0.02, (N, N)).astype(np.float32)
    vy = rng.uniform(-0.02, 0.02, (N, N)).astype(np.float32)
    u0 = 1.0 + 0.3 * rng.uniform(size=(N, N))
    P = 4 * (N - 1)
    kind = np.ones(P, np.int8)
    q = rng.uniform(-0.02, 0.02, P)
    g = hyb.Hybrid(N=N, x0=0, y0=0, u0=u0, vx=vx, vy=vy, D=0.1, eta=50, tau=tau)
    g.set_boundary(q, None, kind)
    g.lbm_substeps(50, restart=1)
    lat = orc.Lattice(N, tau, vx.astype(float), vy.astype(float), bc_kind=kind)
    f = lat.init(u0)
    for _ in range(50):
        f, _ = lat.substep(f, q)
    assert rel_l2(g.get_populations(), f) <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_wall_closure_lattice_matches_oracle(orc, precision, tol):
    """The maximum-entropy zero-flux closure at grain walls (eq. LBM_Neu with
    the grains' normals, FP64 Newton on the GPU, bisection in the oracle)
    against the oracle over 30 fine steps in three commits: populations,
    concentration and the infeasible-node count; switching the closure off
    restores bounce-back."""
    hyb = _gpu()
    N = 97
    pack = inputs.random_disks(N, 0.7, seed=14, r_min=3, r_max=8)
    solid = pack.solid
    wn = inputs.wall_normals(pack)
    rng = np.random.default_rng(15)
    vx = rng.uniform(-0.04, 0.04, (N, N)).astype(np.float32)
    vy = rng.uniform(-0.04, 0.04, (N, N)).astype(np.float32)
    vx[solid != 0] = 0
    vy[solid != 0] = 0
    tau = 0.6
    P = 4 * (N - 1)
    u0 = inputs.gaussian_pulse(4, N)(*np.meshgrid(np.arange(N) * 1.0, np.arange(N) * 1.0, indexing="xy"))
    u0[solid != 0] = 0.0
    g = hyb.Hybrid(N=N, x0=0, y0=0, u0=u0, vx=vx, vy=vy, D=(tau - 0.5) / 3, eta=10, tau=tau, solid=solid,
                   precision=precision, wall_closure=True)
    g.set_wall_normals(wn)
    lat = orc.Lattice(N, tau, vx.astype(float), vy.astype(float), solid=solid, wall_normals=wn)
    f = lat.init(u0)
    if precision == "fp32":
        f = f.astype(np.float32).astype(np.float64)
    a = rng.uniform(0.0, 0.3, P)
    inf = 0
    fluid = solid == 0
    for step in range(3):
        b = a + rng.uniform(-0.02, 0.02, P)
        g.set_boundary(a, b)
        g.lbm_substeps(10, restart=1)
        g.commit()
        for j in range(1, 11):
            f, k = lat.substep(f, (1 - j / 10) * a + j / 10 * b)
            inf += k
        a = b
        e = rel_l2(g.get_populations(), f, fluid)
        print(f"\nwall closure {precision} after {10 * (step + 1)} fine steps: rel L2 {e:.3e}, infeasible {inf}")
        assert e <= tol
    assert rel_l2(g.concentration(), lat.concentration(f), fluid) <= tol
    if precision == "fp64":
        assert g.stats()["infeasible"] == inf
    # back to bounce-back: the next fine steps equal the oracle's bounce-back ones
    g.set_wall_normals(None)
    bb = orc.Lattice(N, tau, vx.astype(float), vy.astype(float), solid=solid)
    g.set_boundary(a, a)
    g.lbm_substeps(10, restart=1)
    g.commit()
    for _ in range(10):
        f, _ = bb.substep(f, a)
    assert rel_l2(g.get_populations(), f, fluid) <= tol
    g.close()


def test_wall_closure_hybrid_matches_oracle(orc):
    """Algorithm 1 on the 129^2 pore workload (32^2 mesh) with the wall
    closure at every grain, FP64, four coarse steps, against the oracle."""
    hyb = _gpu()
    p = problem("pore2048", N=129, M=32)
    wn = inputs.wall_normals(p.pack)
    o = orc.HybridOracle(p, wall_normals=wn)
    g = hyb.Hybrid.from_problem(p, precision="fp64", wall_closure=True)
    g.set_wall_normals(wn)
    o.run(4)
    for _ in range(4):
        g.step(p.cfg.max_iter)
    fluid = p.solid == 0
    e_f = rel_l2(g.concentration(), o.fine_concentration(), fluid)
    e_c = rel_l2(g.concentration(hyb.HYB_COARSE), o.d)
    print(f"\nwall-closure hybrid 129^2: fine {e_f:.3e} coarse {e_c:.3e}, infeasible {o.infeasible}")
    assert e_f <= 1e-12 and e_c <= 1e-12
    assert g.stats()["infeasible"] == o.infeasible
    g.close()


def test_wall_closure_rejects():
    hyb = _gpu()
    p = problem("pore2048", N=65, M=16, eta=3)
    wn = inputs.wall_normals(p.pack)
    plain = hyb.Hybrid.from_problem(p, precision="fp64")
    with pytest.raises(hyb.HybError):                     # no reserved workspace
        plain.set_wall_normals(wn)
    g = hyb.Hybrid.from_problem(p, precision="fp64", wall_closure=True)
    bad = wn.copy()
    j, i = np.argwhere(np.hypot(wn[0], wn[1]) > 0)[0]
    bad[:, j, i] *= 0.5                                   # not a unit normal
    with pytest.raises(hyb.HybError):
        g.set_wall_normals(bad)
    g.set_wall_normals(wn)
    tape = g.adjoint_tape(3)
    with pytest.raises(hyb.HybError):                     # no reverse mode with the wall closure
        g.substeps_record(3, tape)
    plain.close()
    g.close()


# ----------------------------------------------------------------------------
# coarse solve and the full coupling loop
# ----------------------------------------------------------------------------

def _oracle_hybrid(orc, p, steps, **kw):
    o = orc.HybridOracle(p, **kw)
    o.run(steps)
    return o


def _gpu_hybrid(hyb, p, precision, steps, max_schwarz=None):
    g = hyb.Hybrid.from_problem(p, precision=precision)
    for _ in range(steps):
        g.step(max_schwarz or p.cfg.max_iter)
    return g


def test_coarse_solve_matches_direct(orc):
    """One coarse step (BiCGSTAB + sparse approximate inverse on the GPU)
    against the oracle's banded LU on the 128^2 mesh of the 2048^2 workload."""
    hyb = _gpu()
    p = problem("pore2048")
    g = hyb.Hybrid.from_problem(p, precision="fp32")
    g.interface_exchange(hyb.HYB_F2C)
    g.coarse_step()
    d1 = g.concentration(hyb.HYB_COARSE)
    st = g.stats()
    o = orc.HybridOracle(p)
    ufc = o.fine_to_coarse(o.fstar)
    ref = o.coarse_step(o.d, ufc)
    # the fp32 lattice only enters through the f->c data; use the oracle's
    # values read from the same fp32-rounded state to isolate the solver
    assert st["krylov_converged"] == 1 and st["krylov_iters"] < 40
    assert rel_l2(d1, ref) <= 1e-6
    g64 = hyb.Hybrid.from_problem(p, precision="fp64")
    g64.interface_exchange(hyb.HYB_F2C)
    g64.coarse_step()
    assert rel_l2(g64.concentration(hyb.HYB_COARSE), ref) <= 1e-13


@pytest.mark.parametrize("name,over,steps", [("small", {}, 20), ("pore2048", {"N": 129, "M": 16}, 6)])
def test_library_derives_tau_from_D(orc, name, over, steps):
    """The relaxation time comes from each side's own reading of Sec. 4.1:
    the binding passes tau = 0, so hyb_create derives it from D, and the
    oracle derives it from its lattice tables; the two runs agree to 1e-12."""
    hyb = _gpu()
    p = problem(name, **over)
    assert p.cfg.tau is None
    g = hyb.Hybrid.from_problem(p, precision="fp64")
    assert g.lat.tau == 0.0
    for _ in range(steps):
        g.step(p.cfg.max_iter)
    o = _oracle_hybrid(orc, p, steps)
    fluid = p.solid == 0
    assert rel_l2(g.concentration(), o.fine_concentration(), fluid) <= 1e-12
    assert rel_l2(g.concentration(hyb.HYB_COARSE), o.d) <= 1e-12
    g.close()


def test_hybrid_small_fp64_full_run(orc):
    """The 64^2 / 16^2 workload, all 100 coarse steps, FP64."""
    hyb = _gpu()
    p = problem("small")
    o = _oracle_hybrid(orc, p, p.cfg.steps)
    g = _gpu_hybrid(hyb, p, "fp64", p.cfg.steps)
    assert rel_l2(g.concentration(), o.fine_concentration()) <= 1e-12
    assert rel_l2(g.concentration(hyb.HYB_COARSE), o.d) <= 1e-12
    assert g.stats()["infeasible"] == o.infeasible


def test_hybrid_small_clamped_fp64(orc):
    hyb = _gpu()
    p = configs.build_problem(configs.SMALL.replace(bc_clamp=1))
    o = _oracle_hybrid(orc, p, 30)
    g = _gpu_hybrid(hyb, p, "fp64", 30)
    assert rel_l2(g.concentration(), o.fine_concentration()) <= 1e-12
    assert rel_l2(g.concentration(hyb.HYB_COARSE), o.d) <= 1e-12


def test_hybrid_pore_reduced_fp64(orc):
    """Pore geometry, stream-function velocity and reaction at 257^2 (a
    ragged size) on a 32^2 mesh, 12 coarse steps of 10 fine steps."""
    hyb = _gpu()
    p = problem("pore2048", N=257, M=32)
    o = _oracle_hybrid(orc, p, 12)
    g = _gpu_hybrid(hyb, p, "fp64", 12)
    fluid = p.solid == 0
    assert rel_l2(g.concentration(), o.fine_concentration(), fluid) <= 1e-12
    assert rel_l2(g.concentration(hyb.HYB_COARSE), o.d) <= 1e-12


def test_hybrid_small_fp32_error_stated(orc):
    hyb = _gpu()
    p = problem("small")
    o = _oracle_hybrid(orc, p, p.cfg.steps)
    g = _gpu_hybrid(hyb, p, "fp32", p.cfg.steps)
    e_f = rel_l2(g.concentration(), o.fine_concentration())
    e_c = rel_l2(g.concentration(hyb.HYB_COARSE), o.d)
    print(f"\nsmall fp32 vs fp64 oracle after {p.cfg.steps} coarse steps: fine {e_f:.3e} coarse {e_c:.3e}")
    assert e_f < 1e-4 and e_c < 1e-4


@pytest.mark.parametrize("name,steps", [("pore2048", 1), ("pore4096", 1)])
def test_full_size_first_step(orc, name, steps):
    """Full-size workloads in the launch configuration the benchmark times:
    the first coarse step (all Schwarz passes) against the oracle."""
    hyb = _gpu()
    p = problem(name)
    o = _oracle_hybrid(orc, p, steps)
    fluid = p.solid == 0
    uo = o.fine_concentration()
    for precision, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        g = _gpu_hybrid(hyb, p, precision, steps)
        e_f = rel_l2(g.concentration(), uo, fluid)
        e_c = rel_l2(g.concentration(hyb.HYB_COARSE), o.d)
        print(f"\n{name} {precision}: fine {e_f:.3e} coarse {e_c:.3e}")
        assert e_f <= tol and e_c <= tol
        g.close()
        del g


# ----------------------------------------------------------------------------
# error handling (forced from the host)
# ----------------------------------------------------------------------------

def test_nonfinite_boundary_is_reported_and_retry_is_exact(orc):
    hyb = _gpu()
    N = 48
    solid, vx, vy, _, tau = _lattice_case(N, 77)
    u0 = np.full((N, N), 0.5)
    P = 4 * (N - 1)
    good = np.full(P, 0.4)
    bad = good.copy()
    bad[5] = np.nan

    def make():
        return hyb.Hybrid(N=N, x0=0, y0=0, u0=u0, vx=vx, vy=vy, D=0.02, eta=6, tau=tau, solid=solid)

    clean = make()
    clean.set_boundary(good)
    clean.lbm_substeps(6, 1)
    clean.commit()
    ref = clean.get_populations()

    g = make()
    g.set_boundary(bad)
    g.lbm_substeps(6, 1)
    with pytest.raises(hyb.HybError) as e:
        g.commit()
    assert e.value.code == hyb.HYB_ENONFINITE
    g.set_boundary(good)
    g.lbm_substeps(6, 1)
    g.commit()
    assert np.array_equal(g.get_populations(), ref)


def test_coarse_nonconvergence_is_reported():
    hyb = _gpu()
    p = problem("small")
    g = hyb.Hybrid.from_problem(p)
    before = g.get_populations()
    g.interface_exchange(hyb.HYB_F2C)
    g.coarse_step(max_iter=1)
    g.interface_exchange(hyb.HYB_C2F)
    g.lbm_substeps(p.cfg.eta, 1)
    with pytest.raises(hyb.HybError) as e:
        g.commit()
    assert e.value.code == hyb.HYB_ENOCONV
    g.lbm_substeps(0, 1)                # back to the committed state
    assert np.array_equal(g.get_populations(), before)


def test_invalid_arguments():
    hyb = _gpu()
    N = 8
    z = np.zeros((N, N))
    with pytest.raises(hyb.HybError):
        hyb.Hybrid(N=N, x0=0, y0=0, u0=z, vx=z, vy=z, D=0.1, eta=2, tau=0.5)
    solid = np.zeros((N, N), np.uint8)
    solid[0, 3] = 1
    with pytest.raises(hyb.HybError):
        hyb.Hybrid(N=N, x0=0, y0=0, u0=z, vx=z, vy=z, D=0.1, eta=2, solid=solid)
    g = hyb.Hybrid(N=N, x0=0, y0=0, u0=z, vx=z, vy=z, D=0.1, eta=2)
    with pytest.raises(hyb.HybError):
        g.lbm_substeps(3, 1)
    with pytest.raises(hyb.HybError):
        g.interface_exchange(hyb.HYB_F2C)      # lattice-only handle


# ----------------------------------------------------------------------------
# FP16 shifted storage (binary16 g = (f - w c_ref) 2^s, FP32 arithmetic)
# ----------------------------------------------------------------------------

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def fp16s_params(u0, solid):
    """c_ref and the power-of-two scale the library derives from u0."""
    fluid = np.ones(u0.shape, bool) if solid is None else solid == 0
    cref = float(u0[fluid].mean())
    U = max(1.0, float(np.abs(u0[fluid] - cref).max()))
    s = int(np.floor(np.log2(16384.0 / (4.0 / 9.0 * U))))
    return np.float32(cref), np.float32(2.0 ** s)


def fp16s_roundtrip(f, cref, scale):
    """What binary16 storage keeps of f: encode in FP32, round to nearest
    even, decode in FP32."""
    wc = (W9.astype(np.float32) * cref)[:, None, None]
    g = ((f.astype(np.float32) - wc) * scale).astype(np.float16)
    return (g.astype(np.float32) * (np.float32(1) / scale) + wc).astype(np.float64)


def test_fp16s_storage_roundtrip():
    """set/get populations: exactly the binary16 round trip of the stated
    encoding (c_ref = fluid mean of u0, power-of-two scale)."""
    hyb = _gpu()
    N = 40
    solid, vx, vy, _, tau = _lattice_case(N, 9)
    rng = np.random.default_rng(2)
    u0 = rng.uniform(0.0, 3.0, (N, N))
    g = hyb.Hybrid(N=N, x0=0, y0=0, u0=u0, vx=vx, vy=vy, D=0.02, eta=2, precision="fp16s", tau=tau, solid=solid)
    cref, scale = fp16s_params(u0, solid)
    f = inputs.random_populations(N, 5, lo=-0.1, hi=1.2)
    f[:, solid != 0] = 0.0
    g.set_populations(f)
    got = g.get_populations()
    want = fp16s_roundtrip(f, cref, scale)
    want[:, solid != 0] = 0.0
    assert np.array_equal(got, want)


@pytest.mark.parametrize("N,eta", [(67, 5), (130, 4), (200, 10)])
def test_fp16s_substeps_error_stated(orc, N, eta):
    """Random states through eta fine steps with FP16 shifted storage, in
    single steps and in launches of two to five steps, against the FP64
    oracle started from the stored (rounded) state.  Single steps round
    through binary16 after every fine step, a multi-step launch only at its
    store; the error against the oracle is printed and held to 2e-3 (about
    four binary16 roundings), and the paths agree to a few roundings."""
    hyb = _gpu()
    solid, vx, vy, _, tau = _lattice_case(N, 500 + N)
    rng = np.random.default_rng(N)
    P = 4 * (N - 1)
    a = rng.uniform(0.2, 0.6, P)
    b = rng.uniform(0.2, 0.6, P)
    u0 = np.full((N, N), 0.4)
    # near-equilibrium state: f = w u (1 + 5% noise), u in [0.3, 0.5]
    uf = rng.uniform(0.3, 0.5, (N, N))
    f0 = W9[:, None, None] * uf[None] * (1 + 0.05 * rng.standard_normal((9, N, N)))
    f0[:, solid != 0] = 0.0
    cref, scale = fp16s_params(u0, solid)
    lat = orc.Lattice(N, tau, vx.astype(np.float64), vy.astype(np.float64), solid=solid, k=1e-3)
    f = fp16s_roundtrip(f0, cref, scale)
    f[:, solid != 0] = 0.0
    for j in range(1, eta + 1):
        f, _ = lat.substep(f, (1 - j / eta) * a + j / eta * b)
    fluid = solid == 0
    got = {}
    for spl in (1, 2, 3, 4, 5):
        g = hyb.Hybrid(N=N, x0=0, y0=0, u0=u0, vx=vx, vy=vy, D=(tau - 0.5) / 3, eta=eta, precision="fp16s",
                       tau=tau, solid=solid, k=1e-3)
        g.set_steps_per_launch(spl)
        g.set_populations(f0)
        g.set_boundary(a, b)
        g.lbm_substeps(eta, restart=1)
        g.commit()
        got[spl] = g.get_populations()
        err = rel_l2(got[spl], f, fluid)
        print(f"\nfp16s N={N} eta={eta} steps/launch={spl}: rel L2 vs FP64 oracle {err:.3e}")
        assert err <= 2e-3
    for spl in (2, 3, 4, 5):
        d = np.abs(got[spl] - got[1]).max() / np.abs(got[1]).max()
        assert d <= 4e-3, (spl, d)


def test_fp16s_hybrid_small_error_stated(orc):
    """The 64^2 / 16^2 workload, all 100 coarse steps, FP16 shifted storage."""
    hyb = _gpu()
    p = problem("small")
    o = _oracle_hybrid(orc, p, p.cfg.steps)
    g = _gpu_hybrid(hyb, p, "fp16s", p.cfg.steps)
    e_f = rel_l2(g.concentration(), o.fine_concentration())
    e_c = rel_l2(g.concentration(hyb.HYB_COARSE), o.d)
    print(f"\nsmall fp16s vs fp64 oracle after {p.cfg.steps} coarse steps: fine {e_f:.3e} coarse {e_c:.3e}")
    assert e_f < 2e-2 and e_c < 2e-2


def test_fp16s_full_size_first_step(orc):
    """pore2048, first coarse step (2 Schwarz passes x 10 fine steps), FP16
    shifted storage, against the oracle."""
    hyb = _gpu()
    p = problem("pore2048")
    o = _oracle_hybrid(orc, p, 1)
    g = _gpu_hybrid(hyb, p, "fp16s", 1)
    fluid = p.solid == 0
    e_f = rel_l2(g.concentration(), o.fine_concentration(), fluid)
    e_c = rel_l2(g.concentration(hyb.HYB_COARSE), o.d)
    print(f"\npore2048 fp16s first step: fine {e_f:.3e} coarse {e_c:.3e}")
    assert e_f < 1e-2 and e_c < 1e-2
