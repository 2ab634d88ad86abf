"""GPU reverse mode of one whole coarse step (C ABI hyb_step_record /
hyb_step_adjoint): against the oracle's adjoint of Algorithm 1 on the same
state, the dot-product identity of the GPU's own forward and adjoint, and
the rejected configurations."""
import numpy as np
import pytest

from paper_1601_02708_amd import configs

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_02708_amd import hyb
    return hyb, torch


def _rel(x, y):
    return float(np.abs(x - y).max() / max(np.abs(y).max(), 1e-300))


def _problem(name, **over):
    return configs.build_problem(configs.CONFIGS[name].replace(**over))


def _cotangents(p, N, M, seed):
    rng = np.random.default_rng(seed)
    lam_f = rng.standard_normal((9, N, N))
    if p.solid is not None:
        lam_f[:, p.solid != 0] = 0.0
    lam_d = rng.standard_normal((M + 1) ** 2)
    return lam_f, lam_d


def _gpu_adjoint(hyb, torch, g, p, passes, lam_f, lam_d, with_k=True):
    N, M = p.cfg.N, p.cfg.M
    dev = g.dev
    lf = torch.from_numpy(lam_f).to(dev)
    ld = torch.from_numpy(lam_d).to(dev)
    lf_out = torch.empty_like(lf)
    ld_out = torch.empty_like(ld)
    gk = torch.zeros((N, N), dtype=torch.float64, device=dev) if with_k else None
    tape = g.step_tape(passes)
    g.step_record(passes, tape)
    g.step_adjoint(tape, lf, ld, lf_out, ld_out, gk)
    torch.cuda.synchronize()
    return lf_out.cpu().numpy(), ld_out.cpu().numpy(), (gk.cpu().numpy() if with_k else None)


@pytest.mark.parametrize("name,over,precision,tol", [
    ("small", {"k": 2e-3}, "fp64", 1e-11),
    ("pore2048", {"N": 97, "M": 16, "eta": 3}, "fp64", 1e-11),
    ("small", {"k": 2e-3}, "fp32", 1e-4),
])
def test_step_adjoint_matches_oracle(orc, name, over, precision, tol):
    from oracle.hybrid_adjoint import HybridStepAdjoint
    hyb, torch = _gpu()
    p = _problem(name, **over)
    N, M = p.cfg.N, p.cfg.M
    g = hyb.Hybrid.from_problem(p, precision=precision)
    F0 = g.get_populations()
    d0 = g.concentration(hyb.HYB_COARSE).reshape(-1)
    lam_f, lam_d = _cotangents(p, N, M, 11)
    lF, ld, gk = _gpu_adjoint(hyb, torch, g, p, p.cfg.max_iter, lam_f, lam_d)
    o = orc.HybridOracle(p)
    adj = HybridStepAdjoint(o)
    F1, d1, tape = adj.forward(F0, d0)
    # the recorded step committed the same state as the oracle's step
    fwd_tol = 1e-12 if precision == "fp64" else 1e-5
    assert _rel(g.get_populations(), F1) <= fwd_tol
    assert _rel(g.concentration(hyb.HYB_COARSE).reshape(-1), d1) <= fwd_tol
    oF, od, ok = adj.adjoint(tape, lam_f, lam_d)
    errs = {"f": _rel(lF, oF), "d": _rel(ld, od), "k": _rel(gk, ok)}
    print(f"\nstep adjoint {name} {precision}: {errs}")
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("name,over,precision,spl,tol", [
    ("small", {"k": 2e-3, "eta": 5}, "fp64", 2, 1e-11),     # pairs: 5 = 2 + 2 + 1
    ("small", {"k": 2e-3, "eta": 5}, "fp64", 1, 1e-11),     # single reversed steps
    ("pore2048", {"N": 97, "M": 16, "eta": 4}, "fp64", 2, 1e-11),
    ("small", {"k": 2e-3, "eta": 5}, "fp32", 2, 1e-4),
])
def test_step_adjoint_substep_cotangent_matches_oracle(orc, name, over, precision, spl, tol):
    """A cotangent at every intermediate fine state of the committed pass
    (hyb_step_adjoint's lam_sub: an objective that integrates over every
    fine step), in paired and single reversed steps, against the oracle's
    adjoint with the same lam_sub."""
    from oracle.hybrid_adjoint import HybridStepAdjoint
    hyb, torch = _gpu()
    p = _problem(name, **over)
    N, M = p.cfg.N, p.cfg.M
    g = hyb.Hybrid.from_problem(p, precision=precision)
    g.set_steps_per_launch(spl)
    F0 = g.get_populations()
    d0 = g.concentration(hyb.HYB_COARSE).reshape(-1)
    lam_f, lam_d = _cotangents(p, N, M, 31)
    w, _ = _cotangents(p, N, M, 32)
    dev = g.dev
    lf, ld = torch.from_numpy(lam_f).to(dev), torch.from_numpy(lam_d).to(dev)
    lw = torch.from_numpy(w).to(dev)
    lf_out, ld_out = torch.empty_like(lf), torch.empty_like(ld)
    gk = torch.zeros((N, N), dtype=torch.float64, device=dev)
    tape = g.step_tape(p.cfg.max_iter)
    g.step_record(p.cfg.max_iter, tape)
    g.step_adjoint(tape, lf, ld, lf_out, ld_out, gk, lam_sub=lw)
    torch.cuda.synchronize()
    adj = HybridStepAdjoint(orc.HybridOracle(p))
    _, _, otape = adj.forward(F0, d0)
    oF, od, ok = adj.adjoint(otape, lam_f, lam_d, lam_sub=w)
    errs = {"f": _rel(lf_out.cpu().numpy(), oF), "d": _rel(ld_out.cpu().numpy(), od), "k": _rel(gk.cpu().numpy(), ok)}
    print(f"\nstep adjoint with substep cotangent {name} {precision} spl={spl}: {errs}")
    assert max(errs.values()) <= tol, errs
    g.close()


def test_step_adjoint_dot_product_identity_on_gpu():
    """<(lam_f, lam_d), Step(F, d)> = <lam_F, F> + <lam_dn, d> with the GPU
    forward (recorded step) and adjoint, 257^2 patch on a 32^2 mesh (ragged
    tiles, solids), two Schwarz passes, no clamp, zero outer data."""
    hyb, torch = _gpu()
    p = _problem("pore2048", N=257, M=32, eta=6)
    N, M = p.cfg.N, p.cfg.M
    g = hyb.Hybrid.from_problem(p, precision="fp64")
    rng = np.random.default_rng(21)
    F0 = rng.uniform(0.0, 0.2, (9, N, N))
    F0[:, p.solid != 0] = 0.0
    g.set_populations(F0)
    d0 = g.concentration(hyb.HYB_COARSE).reshape(-1)
    lam_f, lam_d = _cotangents(p, N, M, 22)
    lF, ld, _ = _gpu_adjoint(hyb, torch, g, p, 2, lam_f, lam_d, with_k=False)
    F1 = g.get_populations()
    d1 = g.concentration(hyb.HYB_COARSE).reshape(-1)
    lhs = float(np.sum(lam_f * F1)) + float(lam_d @ d1)
    rhs = float(np.sum(lF * F0)) + float(ld @ d0)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0), (lhs, rhs)


def test_step_adjoint_lam_d_null_and_aliasing():
    """lam_d = NULL means zero; lam_f_out may alias lam_f."""
    hyb, torch = _gpu()
    p = _problem("small", k=1e-3)
    N, M = p.cfg.N, p.cfg.M
    lam_f, _ = _cotangents(p, N, M, 31)
    res = []
    for alias in (False, True):
        g = hyb.Hybrid.from_problem(p, precision="fp64")
        lf = torch.from_numpy(lam_f).to(g.dev)
        out = lf if alias else torch.empty_like(lf)
        ld_out = torch.empty((M + 1) ** 2, dtype=torch.float64, device=g.dev)
        tape = g.step_tape(p.cfg.max_iter)
        g.step_record(p.cfg.max_iter, tape)
        g.step_adjoint(tape, lf, None, out, ld_out)
        res.append((out.cpu().numpy(), ld_out.cpu().numpy()))
        g.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_step_adjoint_rejects():
    hyb, torch = _gpu()
    p = _problem("small")
    g = hyb.Hybrid.from_problem(p, precision="fp16s")
    tape = g.step_tape(1)
    with pytest.raises(hyb.HybError):
        g.step_record(1, tape)
    g = hyb.Hybrid.from_problem(p, precision="fp64")
    tape = g.step_tape(2)
    lf = torch.zeros((9, p.cfg.N, p.cfg.N), dtype=torch.float64, device=g.dev)
    ld = torch.zeros((p.cfg.M + 1) ** 2, dtype=torch.float64, device=g.dev)
    with pytest.raises(hyb.HybError):                     # nothing recorded yet
        g.step_adjoint(tape, lf, ld, lf, ld)
    g.step_record(2, tape)
    other = g.step_tape(2)
    with pytest.raises(hyb.HybError):                     # not the recorded tape
        g.step_adjoint(other, lf, ld, lf, ld)
    z = np.zeros((8, 8))
    g2 = hyb.Hybrid(N=8, x0=0, y0=0, u0=z, vx=z, vy=z, D=0.1, eta=2)
    with pytest.raises(hyb.HybError):                     # no coarse mesh
        g2.step_record(1, g.step_tape(1))


def test_step_adjoint_requires_the_recorded_handle():
    """f*(t_n) and the step's end state stay in the handle's buffers: a call
    that changes the handle between hyb_step_record and hyb_step_adjoint
    (another step, fine steps, a commit, new populations or interface values)
    makes the adjoint fail; reading the state does not."""
    hyb, torch = _gpu()
    p = _problem("small")
    N, M = p.cfg.N, p.cfg.M
    g = hyb.Hybrid.from_problem(p, precision="fp64")
    tape = g.step_tape(2)
    lf = torch.ones((9, N, N), dtype=torch.float64, device=g.dev)
    ld = torch.zeros((M + 1) ** 2, dtype=torch.float64, device=g.dev)
    of, od = torch.empty_like(lf), torch.empty_like(ld)
    changes = [lambda: g.step(2),
               lambda: g.lbm_substeps(1, restart=1),
               lambda: g.commit(),
               lambda: g.set_populations(g.get_populations()),
               lambda: g.interface_exchange(hyb.HYB_C2F)]
    for change in changes:
        g.step_record(2, tape)
        change()
        with pytest.raises(hyb.HybError):
            g.step_adjoint(tape, lf, ld, of, od)
    g.step_record(2, tape)
    g.get_populations()
    g.concentration(hyb.HYB_COARSE)
    g.step_adjoint(tape, lf, ld, of, od)
    torch.cuda.synchronize()
    assert torch.isfinite(of).all() and torch.isfinite(od).all()
    g.close()


def test_set_coarse_round_trip():
    hyb, torch = _gpu()
    p = _problem("small")
    g = hyb.Hybrid.from_problem(p, precision="fp64")
    d = np.random.default_rng(41).standard_normal((p.cfg.M + 1) ** 2)
    g.set_coarse(d)
    assert np.array_equal(g.concentration(hyb.HYB_COARSE).reshape(-1), d)
    with pytest.raises(ValueError):
        g.set_coarse(d[:-1])


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
def test_steps_adjoint_matches_oracle_over_a_trajectory(orc, precision, tol):
    """Three coarse steps, a cotangent on the state after every step
    (a trajectory objective), checkpoints every two steps (segments of two
    and one steps): the GPU reverse sweep equals the oracle's composition of
    one-step adjoints, including dJ/dk and dJ/d(outer values)."""
    from oracle.hybrid_adjoint import HybridStepAdjoint
    hyb, torch = _gpu()
    p = _problem("small", k=2e-3)
    N, M, P = p.cfg.N, p.cfg.M, p.cfg.max_iter
    n_steps = 3
    g = hyb.Hybrid.from_problem(p, precision=precision)
    F0 = g.get_populations()
    d0 = g.concentration(hyb.HYB_COARSE).reshape(-1)

    def cot(n, F, d):
        rng = np.random.default_rng(100 + n)
        return rng.standard_normal((9, N, N)), rng.standard_normal((M + 1) ** 2)

    lF, ld, gk, go = hyb.steps_adjoint(g, n_steps, cot, P, checkpoint_every=2)
    o = orc.HybridOracle(p)
    adj = HybridStepAdjoint(o)
    F, d = F0, d0
    tapes, states = [], []
    for _ in range(n_steps):
        F, d, tp = adj.forward(F, d)
        tapes.append(tp)
        states.append((F, d))
    # the handle ends at the rollout's end state
    assert _rel(g.get_populations(), F) <= (1e-12 if precision == "fp64" else 1e-5)
    oF = np.zeros((9, N, N))
    od = np.zeros((M + 1) ** 2)
    ok = np.zeros((N, N))
    oo = np.zeros((M + 1) ** 2)
    for n in range(n_steps - 1, -1, -1):
        cf, cd = cot(n + 1, *states[n])
        oF, od, k, out = adj.adjoint(tapes[n], oF + cf, od + cd, outer=True)
        ok += k
        oo += out
    errs = {"F": _rel(lF, oF), "d": _rel(ld, od), "k": _rel(gk, ok), "outer": _rel(go, oo)}
    print(f"\nsteps adjoint {precision}: {errs}")
    assert max(errs.values()) <= tol, errs


def test_rollout_autograd_by_central_differences():
    """torch.autograd through two coarse steps: the gradient of
    J = <w, F_2> + <v, d_2> along random directions equals central
    differences of the GPU rollout (the map is linear: exact up to the
    coarse solver's tolerance)."""
    hyb, torch = _gpu()
    p = _problem("small", k=1e-3)
    N, M, P = p.cfg.N, p.cfg.M, p.cfg.max_iter
    g = hyb.Hybrid.from_problem(p, precision="fp64")
    Rollout = hyb.rollout_function()
    rng = np.random.default_rng(51)
    dev = g.dev
    F0 = torch.from_numpy(g.get_populations()).to(dev).requires_grad_(True)
    d0 = torch.from_numpy(g.concentration(hyb.HYB_COARSE).copy()).to(dev).requires_grad_(True)
    w = torch.from_numpy(rng.standard_normal((9, N, N))).to(dev)
    v = torch.from_numpy(rng.standard_normal((M + 1) ** 2)).to(dev)
    F2, d2 = Rollout.apply(g, 2, P, F0, d0)
    J = (w * F2).sum() + (v * d2).sum()
    J.backward()
    dF = torch.from_numpy(rng.standard_normal((9, N, N)) * 1e-2).to(dev)
    dd = torch.from_numpy(rng.standard_normal((M + 1) ** 2) * 1e-2).to(dev)
    with torch.no_grad():
        Fp, dp = Rollout.apply(g, 2, P, F0 + dF, d0 + dd)
        Fm, dm = Rollout.apply(g, 2, P, F0 - dF, d0 - dd)
        fd = float(((w * (Fp - Fm)).sum() + (v * (dp - dm)).sum()) / 2)
    an = float((F0.grad * dF).sum() + (d0.grad * dd).sum())
    assert abs(fd - an) <= 1e-9 * max(1.0, abs(an)), (fd, an)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 1e-6)])
def test_step_adjoint_paired_reversed_steps(precision, tol):
    """The whole-step adjoint with its fine steps reversed in pairs (the
    default) against one reversed step per launch: same cotangents and
    gradients to rounding (eta = 5: two pairs and a single step per pass)."""
    hyb, torch = _gpu()
    p = _problem("pore2048", N=97, M=16, eta=5)
    N, M = p.cfg.N, p.cfg.M
    lam_f, lam_d = _cotangents(p, N, M, 71)
    out = {}
    for spl in (1, 4):
        g = hyb.Hybrid.from_problem(p, precision=precision)
        g.set_steps_per_launch(spl)
        out[spl] = _gpu_adjoint(hyb, torch, g, p, p.cfg.max_iter, lam_f, lam_d)
        g.close()
    errs = [_rel(x, y) for x, y in zip(out[4], out[1])]
    print(f"\nstep adjoint paired vs single {precision}: {errs}")
    assert max(errs) <= tol, errs
