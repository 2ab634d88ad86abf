"""P5: the paper's worked LBM example (Sec. 4.1.2, Table LBM_p1).

Exact solution u = exp(-t) sin(pi y) cos(pi x/2), since
D (pi^2 + pi^2/4) = 1 for D = 4/(5 pi^2).  Reading of the table: nodes lie
on the boundary (h = 1/(N-1)), the run takes n = floor(0.25/dt) steps of
the printed dt with tau = 1/2 + 3 D dt / h^2 (Sec. 4.1), and the
Dirichlet closure is eq. (LBM_Dir) as printed (no clamp at zero, which
the u = 0 walls would trigger everywhere).  The oracle must land within a
factor 1.5 of each printed error and converge at second order.
"""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
D = 4.0 / (5.0 * np.pi ** 2)


def load_table():
    rows = []
    for line in open(os.path.join(HERE, "golden", "lbm_p1_table.txt")):
        if line.strip() and not line.startswith("#"):
            c, h, dt, E = line.split()
            rows.append((int(c), float(h), float(dt), float(E)))
    return rows


def e01_error(orc, h, dt, clamp=False):
    N = int(round(1.0 / h)) + 1
    n = int(np.floor(0.25 / dt))
    tau = 0.5 + 3.0 * D * dt / h ** 2
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = np.sin(np.pi * Y) * np.cos(np.pi * X / 2)
    ii, jj = orc.perimeter_nodes(N)
    kind = np.where((ii == 0) & (jj > 0) & (jj < N - 1), 1, 0).astype(np.int8)
    lat = orc.Lattice(N, tau, np.zeros((N, N)), np.zeros((N, N)), bc_kind=kind, clamp=clamp)
    fs = lat.init(u0)
    bc = np.zeros(4 * (N - 1))
    for _ in range(n):
        fs, _ = lat.substep(fs, bc)
    u = lat.concentration(fs)
    return float(np.abs(u - np.exp(-0.25) * u0).max())


@pytest.mark.parametrize("case", [1, 2, 3, 4])
def test_table_lbm_p1(orc, case):
    """Cases 1-3 within a factor 1.5.  Case 4 is held to a factor 3: with
    the printed dt = 5.2e-5, stopping at floor(0.25/dt) steps alone leaves
    t short of 0.25 by 3.6e-5, an error of 2.8e-5 > the printed 1.7e-5, so
    the two-digit dt cannot be the one the paper ran (0.25 h^2/(6D)-based
    steps give 5.14e-5, which would print as 5.1e-5)."""
    row = [r for r in load_table() if r[0] == case][0]
    _, h, dt, E_paper = row
    E = e01_error(orc, h, dt)
    fac = 1.5 if case < 4 else 3.0
    assert E_paper / fac <= E <= E_paper * fac, (E, E_paper)


def test_table_lbm_p1_order(orc):
    rows = load_table()[:3]
    E = [e01_error(orc, h, dt) for _, h, dt, _ in rows]
    orders = np.log2(np.asarray(E[:-1]) / np.asarray(E[1:]))
    assert np.all(orders > 1.7), orders


def test_clamped_closure_is_first_order(orc):
    """The non-negativity clamp cannot meet u = 0 walls: the wall keeps the
    mass of its known populations and the error becomes first order,
    tens of times the printed values.  This is why the default reading
    applies eq. (LBM_Dir) as printed."""
    E1 = e01_error(orc, 4e-2, 3.3e-3, clamp=True)
    E2 = e01_error(orc, 2e-2, 8.2e-4, clamp=True)
    assert E1 > 10 * 2.5e-3
    assert 1.5 < E1 / E2 < 2.5
