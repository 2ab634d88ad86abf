"""The 1-D hybrid of Sec. 7.1 on the GPU (include/hyb1d.h) against the
oracle's Hybrid1D (oracle/hybrid1d.py, driven by the same Algorithm 1 loop
as the 2-D oracle) on rows of the printed Gaussian-hill tables: the coarse
and fine states after the whole run agree to FP64 rounding, so the GPU run
reproduces what the oracle reproduces of the printed errors."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(__file__)
T_END = 0.4


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_02708_amd import hyb
    return hyb


def _rows():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "gauss1d_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        t, r, hc, hf, L, mi, ec, ef = line.split()
        rows[f"{t}r{r}"] = (float(hc), float(hf), float(L), int(mi), float(ec), float(ef))
    return rows


ROWS = _rows()


def _rel(x, y):
    return float(np.abs(x - y).max() / np.abs(y).max())


@pytest.mark.parametrize("key", ["T1r1", "T1r3", "T2r3", "T5r3", "T6r4"])
def test_hybrid1d_matches_oracle(orc, key):
    from oracle.hybrid1d import Hybrid1D, gaussian_exact
    hyb = _gpu()
    hc, hf, L, mi, _, ef_printed = ROWS[key]
    o = Hybrid1D(hc, hf, L, mi)
    n = int(round(T_END / o.dt_c))
    g = hyb.Hybrid1D(hc, hf, L, mi, lambda x: gaussian_exact(x, 0.0, 0.1, 1e-2, 0.3, 1.0, 1e-2))
    assert (g.nc, g.nf, g.eta) == (len(o.xc), len(o.xf), o.eta)
    assert np.array_equal(g.xf, o.xf) and np.array_equal(g.xc, o.xc)
    g.run(n)
    o.run(T_END)
    d, u = g.state()
    uo = o.fstar[0] + o.fstar[1]
    errs = {"d": _rel(d, o.d), "u": _rel(u, uo)}
    print(f"\n1-D hybrid {key} ({n} coarse steps, eta {g.eta}): {errs}")
    assert max(errs.values()) <= 1e-12, errs
    # the fine-domain error of the GPU run against the exact solution
    ef = float(np.abs(u - o.exact(o.xf, o.t)).max())
    assert abs(ef / o.errors()[1] - 1.0) <= 1e-9
    if key in ("T5r3",):
        assert abs(ef / ef_printed - 1.0) <= 0.05


def test_hybrid1d_runs_compose():
    """Two calls of n/2 steps equal one call of n steps bit for bit."""
    from oracle.hybrid1d import gaussian_exact
    hyb = _gpu()
    hc, hf, L, mi = ROWS["T1r2"][:4]
    init = lambda x: gaussian_exact(x, 0.0, 0.1, 1e-2, 0.3, 1.0, 1e-2)
    a = hyb.Hybrid1D(hc, hf, L, mi, init)
    b = hyb.Hybrid1D(hc, hf, L, mi, init)
    a.run(40)
    b.run(20)
    b.run(20)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
