"""Host logic of the measurement, on the CPU: the counter-record writers of
paper_1601_02708_amd/profiling.py (copy-calibrated HBM traffic, the SQ
limiter reading), the bench's check that a committed record belongs to the
current kernel source, its per-launch byte model and launch plan, and its
refusal of more than one GPU."""
import csv
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1601_02708_amd import profiling  # noqa: E402

SWEEP0 = "void hyb::(anonymous namespace)::lbm_sweep4_kernel<double, 64, 8, 512, 0>(hyb::LbmArgs, hyb::TileMap)"
SWEEP1 = "void hyb::(anonymous namespace)::lbm_sweep4_kernel<double, 64, 8, 512, 1>(hyb::LbmArgs, hyb::TileMap)"
COPY = "__amd_rocclr_copyBuffer"


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kernel, counter, value in rows:
            w.writerow({"Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_record_scales_the_sweep_by_the_copy(tmp_path):
    """bytes per launch = (mean FETCH_SIZE x s_f + mean WRITE_SIZE x s_w) KiB,
    s = the copy's known size over what the same counter read for it (the
    largest copy dispatch); only the whole-patch launch (part 0) counts."""
    fetch, write, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _counter_csv(fetch, [(SWEEP0, "FETCH_SIZE", 1000.0), (SWEEP0, "FETCH_SIZE", 1200.0),
                         (SWEEP1, "FETCH_SIZE", 9999.0), (COPY, "FETCH_SIZE", 100.0), (COPY, "FETCH_SIZE", 512.0)])
    _counter_csv(write, [(SWEEP0, "WRITE_SIZE", 500.0), (SWEEP0, "WRITE_SIZE", 700.0),
                         (SWEEP1, "WRITE_SIZE", 9999.0), (COPY, "WRITE_SIZE", 1024.0)])
    profiling.traffic(str(fetch), str(write), str(out), "w", "fp64", "1", "cmd", "lbm_sweep4_kernel")
    rec = json.load(open(out))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0      # 1 MiB copy = 1024 KiB
    assert rec["bytes_per_launch"] == (1100.0 * 2.0 + 600.0 * 1.0) * 1024
    assert rec["launches"] == 2 and rec["kernel"].startswith(SWEEP0[:60])
    assert rec["kernel_sha"] == profiling.kernel_hash("lbm_sweep4_kernel")


def _sq_rows(kernel, valu_busy):
    xcd_cycles = 240000.0                       # 100 us at 2.4 GHz
    quads = 256 * 4 * xcd_cycles / 4.0
    vals = {"GRBM_GUI_ACTIVE": 8 * xcd_cycles, "SQ_ACTIVE_INST_VALU": valu_busy * quads,
            "SQ_WAVE_CYCLES": 4.0e6, "SQ_BUSY_CU_CYCLES": 1.0e6, "SQ_WAIT_INST_ANY": 1.0e6,
            "SQ_LDS_BANK_CONFLICT": 10.0, "SQ_LDS_IDX_ACTIVE": 100.0, "SQ_INSTS_VALU": 8.0e5,
            "SQ_INSTS_SALU": 2.0e5, "SQ_WAVES": 1000.0}
    return [(kernel, c, v) for c, v in vals.items()]


@pytest.mark.parametrize("busy,bound", [(0.5, "latency"), (0.8, "alu")])
def test_sq_record_reads_the_limiter(tmp_path, busy, bound):
    """VALU busy = issue cycles over SIMD quad-cycles (256 CUs x 4 SIMDs);
    waves per CU = 4 x wave quad-cycles over busy CU cycles; at 70% VALU
    the kernel counts as ALU-bound, below as bound by latency."""
    path, out = tmp_path / "a.csv", tmp_path / "sq.json"
    _counter_csv(path, _sq_rows(SWEEP0, busy) + _sq_rows(SWEEP1, 0.1))
    profiling.sq(str(out), "w", "fp64", "lbm_sweep4_kernel", "cmd", str(path))
    rec = json.load(open(out))
    assert rec["valu_busy"] == pytest.approx(busy)
    assert rec["duration_us"] == pytest.approx(100.0)
    assert rec["waves_per_cu"] == pytest.approx(16.0)
    assert rec["mem_wait"] == pytest.approx(0.25) and rec["lds_conflict"] == pytest.approx(0.1)
    assert rec["valu_insts_per_wave"] == pytest.approx(800.0)
    assert rec["bound"] == bound


def test_bench_uses_a_record_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    kernel = "lbm_sweep4_kernel<double, 64, 8, 512, 0>"
    path = tmp_path / "profiles" / "sq_w_fp64.json"

    def put(sha, name=SWEEP0):
        json.dump({"kernel": name, "kernel_sha": sha, "bound": "latency", "limiter": "x"}, open(path, "w"))

    assert bench.load_limiter("w", "fp64", kernel) is None                      # no record
    put(profiling.kernel_hash("lbm_sweep4_kernel"))
    assert bench.load_limiter("w", "fp64", kernel) == {"bound": "latency", "limiter": "x"}
    put("0" * 16)                                                               # source changed since
    assert bench.load_limiter("w", "fp64", kernel) is None
    put(profiling.kernel_hash("lbm_sweep4_kernel"), SWEEP0.replace("sweep4", "sweep3"))
    assert bench.load_limiter("w", "fp64", kernel) is None                      # another kernel's record
    # the reversed-step kernel's records are keyed by its own source
    assert profiling.kernel_hash("adj_step2_kernel") != profiling.kernel_hash("lbm_sweep4_kernel")


def test_sweep_byte_model():
    """Per fluid node 9 loads and 9 stores of the storage type, two FP32
    velocity components and the flag word; a solid node its flag word; a
    perimeter slot its two FP64 interface values."""
    class Cfg:
        N = 5

    class Problem:
        cfg = Cfg()
        solid = np.zeros((5, 5), dtype=np.uint8)

    Problem.solid[2, 1:4] = 1
    total, fluid, solid, per_fluid = bench.sweep_bytes(Problem, 8)
    assert (fluid, solid, per_fluid) == (22, 3, 18 * 8 + 10)
    assert total == 22 * 154 + 3 * 2 + 4 * 4 * 16
    assert bench.sweep_bytes(Problem, 2)[3] == 18 * 2 + 10


@pytest.mark.parametrize("spl,plans", [
    (3, {5: [3, 2], 9: [3, 3, 3], 3: [3], 6: [3, 3], 7: [3, 2, 2], 10: [3, 3, 2, 2], 8: [3, 3, 2]}),
    (4, {5: [3, 2], 9: [4, 3, 2], 3: [3], 6: [3, 3], 7: [4, 3], 10: [4, 3, 3], 8: [4, 4], 4: [4]}),
    (5, {9: [5, 4], 10: [5, 5], 8: [4, 4], 7: [4, 3], 20: [5, 5, 5, 5]}),
    (2, {10: [2, 2, 2, 2, 2], 5: [2, 2, 1]}),
])
def test_bench_launch_plan_is_the_librarys(spl, plans):
    """The plans the bench prices its roofline with: the library's pass plans
    that the K-step parity tests run (as many steps as allowed, no lone
    single step where it can be avoided)."""
    for eta, plan in plans.items():
        assert bench.launch_plan(eta, spl) == plan, (spl, eta)
    for eta in range(1, 41):
        p = bench.launch_plan(eta, spl)
        assert sum(p) == eta and max(p) <= spl
        assert eta < 2 or spl < 2 or 1 not in p or (spl == 2 and eta % 2 == 1)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and r.stdout == ""
