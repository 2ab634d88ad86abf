"""Pins of the oracle's adjoint (reverse mode) of the fine step.

The fine step with the Dirichlet closure applied as printed is linear and
homogeneous in (f*(t), u^p) for fixed velocity, tau and reaction rate, so
its adjoint is fixed exactly by the dot-product identity
<c, F(x)> = <F^T c, x> and by brute-force columns of the step's matrix.
Over n steps the objective is a polynomial of degree n in the reaction
rate k, so its k-gradient is fixed by central differences to O(eps^2).
Clamped closures are piecewise linear and are checked by one-sided
differences that switch no closure.
"""
import numpy as np
import pytest


def _case(orc, N, seed, solid=True, k_field=True, clamp=False, periodic=False, vmax=0.08, tau=0.57):
    rng = np.random.default_rng(seed)
    sol = None
    if solid:
        sol = np.zeros((N, N), np.uint8)
        # a few solid blocks away from the perimeter
        for (i0, j0, w, h) in ((3, 4, 3, 2), (N - 7, N - 6, 2, 3), (N // 2, N // 2 - 1, 2, 2)):
            sol[j0:j0 + h, i0:i0 + w] = 1
    vx = rng.uniform(-vmax, vmax, (N, N))
    vy = rng.uniform(-vmax, vmax, (N, N))
    if sol is not None:
        vx[sol != 0] = 0
        vy[sol != 0] = 0
    k = rng.uniform(0.0, 0.02, (N, N)) if k_field else 0.01
    lat = orc.Lattice(N, tau, vx, vy, solid=sol, k=k, clamp=clamp, periodic_x=periodic, periodic_y=periodic)
    return lat, sol, rng


def _run(lat, f0, bcs):
    f = f0
    for bc in bcs:
        f, _ = lat.substep(f, bc)
    return f


def _adjoint(lat, f0, bcs, c):
    """Reverse sweep over the steps: returns dJ/df0, [dJ/du^p per step], dJ/dk."""
    states = [f0]
    for bc in bcs[:-1]:
        states.append(lat.substep(states[-1], bc)[0])
    lam = c
    gk = np.zeros((lat.N, lat.N))
    gbc = [None] * len(bcs)
    for t in reversed(range(len(bcs))):
        lam, g, k = lat.adjoint_substep(states[t], bcs[t], lam)
        gbc[t] = g
        gk += k
    return lam, gbc, gk


@pytest.mark.parametrize("N,steps,solid,periodic", [(12, 1, True, False), (13, 4, True, False),
                                                    (10, 3, False, False), (11, 3, True, True)])
def test_adjoint_dot_product(orc, N, steps, solid, periodic):
    lat, sol, rng = _case(orc, N, 10 + N, solid=solid, periodic=periodic)
    P = 4 * (N - 1)
    x0 = rng.standard_normal((9, N, N))
    bcs = [rng.standard_normal(P) for _ in range(steps)]
    if sol is not None:
        x0[:, sol != 0] = 0.0
    c = rng.standard_normal((9, N, N))
    lhs = float(np.sum(c * _run(lat, x0, bcs)))
    lam, gbc, _ = _adjoint(lat, np.zeros_like(x0), [np.zeros(P)] * steps, c)
    rhs = float(np.sum(lam * x0)) + sum(float(np.dot(g, b)) for g, b in zip(gbc, bcs))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs)), (lhs, rhs)


def test_adjoint_matches_single_entries(orc):
    """Brute force on a tiny lattice: column n of the step's matrix (response
    to a unit population) dotted with c equals entry n of the adjoint."""
    N = 5
    lat, _, rng = _case(orc, N, 3, solid=False)
    P = 4 * (N - 1)
    c = rng.standard_normal((9, N, N))
    lam, gbc, _ = lat.adjoint_substep(np.zeros((9, N, N)), np.zeros(P), c)
    for idx in [(0, 2, 2), (1, 0, 0), (5, 4, 1), (8, 2, 4), (3, 1, 3)]:
        e = np.zeros((9, N, N))
        e[idx] = 1.0
        col, _ = lat.substep(e, np.zeros(P))
        assert abs(float(np.sum(c * col)) - lam[idx]) <= 1e-14
    for p in (0, 3, P - 1):
        bc = np.zeros(P)
        bc[p] = 1.0
        col, _ = lat.substep(np.zeros((9, N, N)), bc)
        assert abs(float(np.sum(c * col)) - gbc[p]) <= 1e-14


def test_adjoint_reaction_rate_by_central_differences(orc):
    N, steps = 12, 3
    lat, sol, rng = _case(orc, N, 77)
    P = 4 * (N - 1)
    f0 = np.abs(rng.standard_normal((9, N, N))) * 0.1
    f0[:, sol != 0] = 0.0
    bcs = [rng.uniform(0.1, 0.5, P) for _ in range(steps)]
    c = rng.standard_normal((9, N, N))
    _, _, gk = _adjoint(lat, f0, bcs, c)
    dk = rng.standard_normal((N, N))
    dk[sol != 0] = 0.0
    k0 = lat.kfield.copy()
    eps = 1e-4

    def J(kf):
        l2 = orc.Lattice(N, lat.tau, lat.vx, lat.vy, solid=sol, k=kf)
        return float(np.sum(c * _run(l2, f0, bcs)))

    fd = (J(k0 + eps * dk) - J(k0 - eps * dk)) / (2 * eps)
    an = float(np.sum(gk * dk))
    # J is a polynomial of degree `steps` in k: central differences err by O(eps^2)
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)


def test_adjoint_clamped_closure_one_sided(orc):
    """With clamp, closures with R < 0 give constant unknowns: the adjoint
    is that of the active branch (checked by small one-sided differences
    that switch no closure)."""
    N, steps = 10, 2
    lat, sol, rng = _case(orc, N, 5, solid=False, clamp=True)
    P = 4 * (N - 1)
    f0 = np.abs(rng.standard_normal((9, N, N))) * 0.2 + 0.05
    bcs = [rng.uniform(-0.2, 0.6, P) for _ in range(steps)]     # some R < 0, some R > 0
    nb = sum(lat.substep(f0, b)[1] for b in bcs[:1])
    assert nb > 0
    c = rng.standard_normal((9, N, N))
    lam, gbc, _ = _adjoint(lat, f0, bcs, c)
    d0 = rng.standard_normal((9, N, N))
    db = [rng.standard_normal(P) for _ in range(steps)]
    eps = 1e-7
    Jp = float(np.sum(c * _run(lat, f0 + eps * d0, [b + eps * d for b, d in zip(bcs, db)])))
    J0 = float(np.sum(c * _run(lat, f0, bcs)))
    fd = (Jp - J0) / eps
    an = float(np.sum(lam * d0)) + sum(float(np.dot(g, d)) for g, d in zip(gbc, db))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_adjoint_rejects_neumann(orc):
    N = 6
    kind = np.zeros(4 * (N - 1), np.int8)
    kind[3] = 1
    lat = orc.Lattice(N, 0.6, np.zeros((N, N)), np.zeros((N, N)), bc_kind=kind)
    with pytest.raises(ValueError):
        lat.adjoint_substep(np.zeros((9, N, N)), np.zeros(4 * (N - 1)), np.zeros((9, N, N)))


def test_adjoint_of_pulse_transport_drives_sensitivity_upstream(orc):
    """A physical sanity check: with a uniform flow in +x, the sensitivity of
    the total mass in the right half after n steps to the initial state lies
    upstream (to the left) of that region, shifted by about n |v|."""
    N, steps = 40, 20
    v = 0.3
    lat = orc.Lattice(N, 0.8, np.full((N, N), v), np.zeros((N, N)), k=0.0, periodic_x=True, periodic_y=True)
    c = np.zeros((9, N, N))
    c[:, :, 20:30] = 1.0             # mass in columns 20..29 at the end
    lam, _, _ = _adjoint(lat, np.zeros((9, N, N)), [np.zeros(4 * (N - 1))] * steps, c)
    prof = lam.sum(axis=(0, 1))
    centre = float(np.sum(prof * np.arange(N)) / np.sum(prof))
    assert abs(centre - (24.5 - steps * v)) < 1.0
