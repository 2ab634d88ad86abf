"""The one-dimensional hybrid (D1Q2 fine, linear Galerkin coarse) driven by
the oracle's Algorithm 1 loop, against the errors printed for the advected
Gaussian hill (Sec. 7.1, tests/golden/gauss1d_tables.txt).

Pinned: the fine-domain error at the finest printed resolutions (the
floor set by the zero-flux wall's reflection, which the printed values
reach), and the two trends the paper states -- refining only the fine grid
lowers the fine-domain error, refining only the coarse grid leaves it
unchanged.  Not reproduced: the printed coarse-domain errors, which are
first order in h_c and 10-100 times larger than this implementation's
(the paper's exchange evidently carries an O(h_c) interface error that its
text does not specify)."""
import os

import numpy as np
import pytest

from oracle.hybrid1d import Hybrid1D

HERE = os.path.dirname(__file__)
T_END = 0.4


def _rows():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "gauss1d_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        t, r, hc, hf, L, mi, ec, ef = line.split()
        rows[f"{t}r{r}"] = (float(hc), float(hf), float(L), int(mi), float(ec), float(ef))
    return rows


ROWS = _rows()


def _run(key):
    hc, hf, L, mi, _, _ = ROWS[key]
    return Hybrid1D(hc, hf, L, mi).run(T_END).errors()


@pytest.mark.parametrize("key,tol", [("T5r3", 0.05), ("T4r4", 0.12), ("T6r4", 0.12)])
def test_fine_error_at_finest_rows(key, tol):
    _, ef = _run(key)
    printed = ROWS[key][5]
    assert abs(ef / printed - 1.0) <= tol, (ef, printed)


def test_reflection_floor_is_the_wall_image():
    """The floor is the image source of the zero-flux wall at x = 1: the
    exact half-line solution minus the free-space one at x = 1."""
    phi, s0, x0, v, D = 0.1, 1e-2, 0.3, 1.0, 1e-2
    s2 = s0 ** 2 + 2 * D * T_END
    image = phi / np.sqrt(2 * np.pi * s2) * np.exp(-(1.0 - (2.0 - x0 - v * T_END)) ** 2 / (2 * s2))
    assert abs(image / ROWS["T5r3"][5] - 1.0) < 0.05


def test_fine_refinement_lowers_fine_error():
    e = [_run(k)[1] for k in ("T1r1", "T1r2", "T1r3")]
    assert e[0] > e[1] > e[2]
    # the paper's fine errors fall the same way (printed column)
    p = [ROWS[k][5] for k in ("T1r1", "T1r2", "T1r3")]
    assert p[0] > p[1] > p[2]


def test_coarse_refinement_leaves_fine_error():
    base = _run("T1r3")[1]
    for k in ("T2r2", "T2r3"):
        assert abs(_run(k)[1] / base - 1.0) < 0.05
    p = [ROWS[k][5] for k in ("T1r3", "T2r2", "T2r3")]
    assert max(p) / min(p) < 1.1
