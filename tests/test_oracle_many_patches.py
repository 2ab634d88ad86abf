"""Pins of the oracle's Algorithm 2 with one coarse subdomain and several
fine patches (oracle/many_patches.py): one patch is Algorithm 1 bit for
bit; two patches mirrored about the domain's centre line give a mirrored
solution; a constant state with matching outer data stays constant."""
import numpy as np
import pytest

from paper_1601_02708_amd import configs, inputs


def test_one_patch_is_algorithm_1(orc):
    from oracle.many_patches import ManyPatchOracle
    cfg = configs.SMALL
    p = configs.build_problem(cfg)
    mp = configs.build_multi(cfg.N, cfg.M, p.L, [(p.x0, p.y0)], D=cfg.D, k=cfg.k, eta=cfg.eta,
                             max_iter=cfg.max_iter, velocity=cfg.v_uniform, pulse=inputs.gaussian_pulse(cfg.seed, p.L))
    assert np.array_equal(mp.patches[0].u0_fine, p.u0_fine) and np.array_equal(mp.u0_coarse, p.u0_coarse)
    o1 = orc.HybridOracle(p).run(3)
    o2 = ManyPatchOracle(mp).run(3)
    assert np.array_equal(o2.fstar[0], o1.fstar) and np.array_equal(o2.d, o1.d)


def _mirror_pair(v=(0.0, 0.0)):
    L, N, M = 128.0, 33, 16
    pulse = inputs.Pulse(xc=64.0, yc=64.0, sigma=20.0)
    return configs.build_multi(N, M, L, [(16.0, 48.0), (80.0, 48.0)], D=1e-2, eta=4, max_iter=2, velocity=v,
                               pulse=pulse)


def test_mirrored_patches_give_a_mirrored_solution(orc):
    """Reflection x -> L - x maps patch A onto patch B and the pulse onto
    itself (no flow): the coarse solution is symmetric and B's populations
    are A's with the x direction reversed (q: 1 <-> 3, 5 <-> 6, 7 <-> 8)."""
    from oracle.many_patches import ManyPatchOracle
    mp = _mirror_pair()
    o = ManyPatchOracle(mp).run(3)
    M, N = mp.M, mp.patches[0].N
    d = o.d.reshape(M + 1, M + 1)
    assert np.abs(d - d[:, ::-1]).max() <= 1e-13 * np.abs(d).max()
    mirror_q = [0, 3, 2, 1, 4, 6, 5, 8, 7]
    A, B = o.fstar
    assert np.abs(B - A[mirror_q][:, :, ::-1]).max() <= 1e-13 * np.abs(A).max()
    # the coupling matters: the patches differ from their first state
    assert np.abs(A - ManyPatchOracle(mp).fstar[0]).max() > 1e-3


def test_constant_state_is_preserved(orc):
    """No flow (the closure's unknowns are at rest), no reaction: every
    transfer weight set and eq. (MTS) reproduce a constant exactly."""
    from oracle.many_patches import ManyPatchOracle
    mp = _mirror_pair()
    c = 0.7
    for p in mp.patches:
        p.u0_fine[:] = c
    mp.u0_coarse[:] = c
    o = ManyPatchOracle(mp, outer_value=c).run(3)
    assert np.abs(o.d - c).max() <= 1e-13
    for lat, F in zip(o.lat, o.fstar):
        assert np.abs(lat.concentration(F) - c).max() <= 1e-13
