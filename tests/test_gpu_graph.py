"""A Schwarz pass's fine steps (hyb_lbm_substeps, restart from the
committed state) and the allocation-free diagnostics captured in one HIP
graph on the handle's stream and replayed: every replay equals the eager
pass, with the pass's destination buffers cleared, other work and
synchronisations in between (so a replay that did nothing would fail)."""
import ctypes

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


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_pass_and_diagnostics_replay_in_a_hip_graph(precision):
    hyb, torch = _gpu()
    lib = hyb.load()
    p = configs.build_problem(configs.PORE2048.replace(N=257, M=32, eta=10))
    side = torch.cuda.Stream()                   # capture needs a stream other than the legacy default one
    with torch.cuda.stream(side):
        g = hyb.Hybrid.from_problem(p, precision=precision)
    assert g.stream.cuda_stream == side.cuda_stream
    for _ in range(2):
        g.step(p.cfg.max_iter)
    # interface values of the next coarse step, then the eager pass
    g.interface_exchange(hyb.HYB_F2C)
    g.coarse_step()
    g.interface_exchange(hyb.HYB_C2F)
    before = [b.clone() for b in g.fbuf]
    g.lbm_substeps(p.cfg.eta, restart=1)
    ref = g.get_populations()
    ref_diag = g.diagnostics()
    changed = [k for k in range(3) if not torch.equal(before[k], g.fbuf[k])]
    assert len(changed) == 2                     # the committed buffer is only read

    out = torch.full((4,), -1.0, dtype=torch.float64, device=g.dev)
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=g.stream):
        g.lbm_substeps(p.cfg.eta, restart=1)
        assert lib.hyb_diagnostics_noalloc(g.h, ctypes.c_void_p(out.data_ptr())) == hyb.HYB_OK
    for r in range(3):
        for k in changed:
            g.fbuf[k].zero_()
        out.fill_(-1.0)
        other = torch.randn(1 << 20, device=g.dev).sum()      # unrelated eager work
        torch.cuda.synchronize()
        assert float(other) == float(other)
        graph.replay()
        torch.cuda.synchronize()
        got = g.get_populations()
        assert np.array_equal(got, ref), r
        v = out.cpu().numpy()
        assert (v[0], v[1], v[2], v[3]) == (ref_diag["mass"], ref_diag["min_f"], ref_diag["h_function"],
                                            ref_diag["nonfinite"]), r
    del graph
    g.close()
