"""Full-size workloads against the oracle at their final coarse step: the
2048^2 pore workload over all 200 coarse steps and the 4096^2 precision
form over all 100, in the launch configuration the benchmark times (the
library's default plan and overlap).  FP64 must agree to 1e-12 relative L2
on the fine concentration (fluid nodes) and the coarse solution; the FP32
and FP16-shifted-storage errors against the FP64 oracle are stated and held
to loose regression bounds.  The oracle runs on every host thread OpenMP
gives it (its results do not depend on the thread count)."""
import time

import numpy as np
import pytest

from paper_1601_02708_amd import configs

pytestmark = pytest.mark.gpu

_ORACLE = {}


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_02708_amd import hyb
    return hyb


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _oracle_final(orc, name):
    """(problem, fine concentration, coarse solution, infeasible count) of
    the oracle after all of the workload's coarse steps (cached)."""
    if name not in _ORACLE:
        p = configs.build_problem(configs.CONFIGS[name])
        o = orc.HybridOracle(p)
        t0 = time.perf_counter()
        for s in range(p.cfg.steps):
            o.step()
            if s % 20 == 19:
                print(f"[oracle] {name}: coarse step {s + 1}/{p.cfg.steps}, {time.perf_counter() - t0:.0f} s",
                      flush=True)
        print(f"[oracle] {name}: {p.cfg.steps} coarse steps on {orc.get_threads()} threads in "
              f"{time.perf_counter() - t0:.1f} s", flush=True)
        _ORACLE[name] = (p, o.fine_concentration(), o.d.copy(), o.infeasible)
        del o
    return _ORACLE[name]


def _gpu_final(hyb, p, precision):
    g = hyb.Hybrid.from_problem(p, precision=precision)
    for _ in range(p.cfg.steps):
        g.step(p.cfg.max_iter)
    fine, coarse = g.concentration(), g.concentration(hyb.HYB_COARSE).reshape(-1)
    st = g.stats()
    g.close()
    return fine, coarse, st


@pytest.mark.parametrize("name,precisions", [
    ("pore2048", (("fp64", 1e-12), ("fp32", 1e-4))),
    ("pore4096", (("fp64", 1e-12), ("fp32", 1e-4), ("fp16s", 5e-3))),
])
def test_final_step_against_oracle(orc, name, precisions):
    hyb = _gpu()
    p, uo, do, inf_o = _oracle_final(orc, name)
    fluid = p.solid == 0
    for precision, tol in precisions:
        fine, coarse, st = _gpu_final(hyb, p, precision)
        e_f = rel_l2(fine[fluid], uo[fluid])
        e_c = rel_l2(coarse, do)
        print(f"\n{name} {precision} after {p.cfg.steps} coarse steps vs the FP64 oracle: "
              f"fine {e_f:.3e} coarse {e_c:.3e}", flush=True)
        assert e_f <= tol and e_c <= tol, (precision, e_f, e_c)
        assert st["nonfinite"] == 0
        if precision == "fp64":
            assert st["infeasible"] == inf_o
