"""Pins of the oracle's reverse mode of a coarse step with dissolving
solids (oracle/dissolution_adjoint.py): the recorded forward is the
dissolving step, the replay reproduces it, the adjoint satisfies the
dot-product identity of the recorded (affine) map including the conversion,
and its reaction-rate gradient matches central differences."""
import numpy as np
import pytest

from paper_1601_02708_amd import configs


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def _hybrid(orc):
    from oracle.dissolution import DissolvingHybrid
    p = configs.build_problem(configs.PORE2048.replace(N=65, M=16, eta=3))
    mass = np.random.default_rng(7).uniform(0.002, 0.01, p.solid.shape)
    return p, mass, (lambda: DissolvingHybrid(p, mass, kappa_s=0.2, c_sat=1.0))


@pytest.fixture(scope="module")
def recorded(orc):
    from oracle.dissolution_adjoint import DissolvingStepAdjoint
    p, mass, make = _hybrid(orc)
    o = make()
    adj = DissolvingStepAdjoint(o)
    F0, d0 = o.fstar.copy(), o.d.copy()
    F1, d1, tape = adj.forward(F0, d0)
    return p, make, o, adj, F0, d0, F1, d1, tape


def test_recorded_forward_is_the_dissolving_step(recorded):
    p, make, o, adj, F0, d0, F1, d1, tape = recorded
    o2 = make()
    o2.step()
    assert np.array_equal(F1, o2.fstar) and np.array_equal(d1, o2.d)
    assert np.array_equal(o.solid, o2.solid) and np.array_equal(o.mass, o2.mass)
    assert tape["conv"].sum() == o2.converted > 0


def test_replay_reproduces_the_recorded_step(recorded):
    p, make, o, adj, F0, d0, F1, d1, tape = recorded
    F, d = adj.replay(tape, F0, d0)
    assert np.array_equal(F, F1) and np.array_equal(d, d1)


def test_dissolving_step_dot_product_identity(recorded):
    """The recorded step is affine in (F, d) (reaction towards c_sat and the
    conversion with its set fixed): <lam, M(x) - M(0)> = <M^T lam, x>."""
    p, make, o, adj, F0, d0, F1, d1, tape = recorded
    N, n1 = o.N, (o.M + 1) ** 2
    rng = np.random.default_rng(5)
    fluid = tape["solid"] == 0
    F = rng.uniform(0.0, 0.2, (9, N, N)) * fluid
    d = rng.standard_normal(n1)
    lam_f = rng.standard_normal((9, N, N)) * (o.solid == 0)
    lam_d = rng.standard_normal(n1)
    Fa, da = adj.replay(tape, F, d)
    Fz, dz = adj.replay(tape, np.zeros_like(F), np.zeros_like(d))
    lF, ld, _ = adj.adjoint(tape, lam_f, lam_d)
    lhs = float(np.sum(lam_f * (Fa - Fz))) + float(lam_d @ (da - dz))
    rhs = float(np.sum(lF * F)) + float(ld @ d)
    assert _rel(lhs, rhs) <= 1e-11, (lhs, rhs)
    # the converted nodes' cotangent reaches their fluid neighbours
    conv = tape["conv"]
    assert conv.any()
    lF0, _, _ = adj.adjoint(tape, lam_f * ~conv, lam_d)
    assert not np.array_equal(lF0, lF)


def test_dissolving_step_rate_gradient_by_central_differences(recorded):
    p, make, o, adj, F0, d0, F1, d1, tape = recorded
    N, n1 = o.N, (o.M + 1) ** 2
    rng = np.random.default_rng(6)
    lam_f = rng.standard_normal((9, N, N)) * (o.solid == 0)
    lam_d = rng.standard_normal(n1)
    _, _, gk = adj.adjoint(tape, lam_f, lam_d)
    k0 = np.full((N, N), p.cfg.k)
    dk = rng.standard_normal((N, N))
    eps = 1e-5

    def J(kf):
        F, d = adj.replay(tape, F0, d0, kfield=kf)
        return float(np.sum(lam_f * F)) + float(lam_d @ d)

    fd = (J(k0 + eps * dk) - J(k0 - eps * dk)) / (2 * eps)
    assert _rel(fd, float(np.sum(gk * dk))) <= 1e-7
    # the conversion's own rate terms matter: without them the check fails
    _, gk_conv = adj.conversion_T(tape, lam_f)
    assert _rel(fd, float(np.sum((gk - gk_conv) * dk))) > 1e-6
