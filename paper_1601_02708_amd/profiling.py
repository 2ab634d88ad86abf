"""Summarise rocprofv3 output of bench.py runs into the short text records
kept under profiles/ (run on the host after the GPU job).

    python -m paper_1601_02708_amd.profiling stats  <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1601_02708_amd.profiling traffic <fetch_counter_collection.csv> \
        <write_counter_collection.csv> <out.json> <workload> <precision> <copy_mib> "<commands>" [kernel]
    python -m paper_1601_02708_amd.profiling sq <out.json> <workload> <precision> <kernel> "<commands>" \
        <counter_collection.csv> ...

The traffic record scales the FETCH_SIZE / WRITE_SIZE counters of the
lattice-sweep kernel by what the same counters read for the plain copy
bench.py --copy-mib performs in the same run (a copy of known size), and
stores the sweep kernel's source hash so that bench.py drops the figure
once the kernel changes.
"""
import csv
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the source of a kernel and the header it is built with: a counter record
# stays valid while neither changes (the reversed-step kernels live in
# adjoint_kernels.hip, the sweeps in lbm_kernels.hip)
def _srcs(kernel):
    f = "adjoint_kernels.hip" if kernel.startswith("adj_") else "lbm_kernels.hip"
    return [os.path.join(ROOT, "paper_1601_02708_amd", "csrc", n) for n in (f, "hyb_impl.h")]


def kernel_hash(kernel="lbm_sweep"):
    h = hashlib.sha256()
    for path in _srcs(kernel):
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def stats(csv_path, out_path, command):
    rows = list(csv.DictReader(open(csv_path)))
    lines = ["# rocprofv3 kernel statistics", "", f"command: `{command}`", "",
             "| kernel | calls | avg us | min us | max us | total ms | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    open(out_path, "w").write("\n".join(lines) + "\n")


def _per_kernel(path, counter):
    out = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def traffic(fetch_csv, write_csv, out_path, workload, precision, copy_mib, commands, kernel="lbm_sweep3_kernel"):
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    tname = {"fp32": "float", "fp64": "double", "fp16s": "_Float16"}[precision]
    # the dominant sweep kernel: the whole-patch launch (tile part 0) of
    # `kernel` (the bench's dominant kind) when it ran, else the whole-patch
    # two-step launch, else the single-step one
    mname = {"fp32": "f", "fp64": "d", "fp16s": "DF16_"}[precision]
    # demangled, or (where the demangler gives up, as for _Float16) mangled
    sweep = [k for k in fetch if (f"{kernel}<" in k and f"<{tname}" in k and ", 0>" in k) or
             (f"{kernel}I{mname}Li" in k and "ELi0EEEv" in k)]
    sweep = sweep or [k for k in fetch if "lbm_sweep2_kernel" in k and f"<{tname}" in k and ", 0>" in k]
    sweep = sweep or [k for k in fetch if "lbm_sweep_kernel" in k and f"<{tname}" in k]
    if not sweep:
        raise SystemExit("no sweep kernel in the counter file")
    # the calibration copy is the largest copyBuffer dispatch; it reads and
    # writes copy_mib MiB each
    copy_f = max(v for k, vs in fetch.items() if "copyBuffer" in k for v in vs)
    copy_w = max(v for k, vs in write.items() if "copyBuffer" in k for v in vs)
    copy_bytes_kib = float(copy_mib) * 1024.0
    f_scale = copy_bytes_kib / copy_f
    w_scale = copy_bytes_kib / copy_w
    k = sweep[0]
    f = statistics.mean(fetch[k])
    w = statistics.mean(write[k])
    rec = {
        "kernel": k[:120], "workload": workload, "precision": precision, "kernel_sha": kernel_hash(kernel),
        "fetch_kib_per_launch": f, "write_kib_per_launch": w,
        "copy_kib": copy_bytes_kib, "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "bytes_per_launch": int(round((f * f_scale + w * w_scale) * 1024)),
        "launches": len(fetch[k]), "commands": commands,
    }
    json.dump(rec, open(out_path, "w"), indent=1)
    print(json.dumps(rec))


def _per_kernel_all(paths):
    out = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            out.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return out


def sq(out_path, workload, precision, kernel, commands, *csv_paths):
    """Shader-sequencer counters of the dominant sweep kernel (whole-patch
    launches of `kernel`, mean per dispatch) from several --pmc passes, with
    the derived utilisations and the limiter they point to:
      valu_busy   VALU issue cycles per SIMD cycle (one wave instruction per
                  4 cycles per SIMD, 4 SIMDs per CU, 256 CUs)
      waves_per_cu  mean resident waves per CU (SQ_WAVE_CYCLES counts
                  quad-cycles, SQ_BUSY_CU_CYCLES cycles)
      mem_wait    share of wave time waiting at s_waitcnt
      lds_conflict  LDS bank-conflict cycles per LDS-active cycle
    """
    data = _per_kernel_all(csv_paths)
    tname = {"fp32": "float", "fp64": "double", "fp16s": "_Float16"}[precision]
    mname = {"fp32": "f", "fp64": "d", "fp16s": "DF16_"}[precision]
    # the whole-patch launch (tile part 0) of a sweep; the reversed-step
    # kernels have no parts
    whole = kernel.startswith("adj_")
    ks = [k for k in data if (f"{kernel}<{tname}" in k and (whole or ", 0>" in k)) or
          (kernel in k and f"I{mname}" in k and (whole or "Li0EEE" in k))]
    if not ks:
        raise SystemExit("kernel not found in the counter files")
    m = {c: statistics.mean(v) for c, v in data[ks[0]].items()}
    xcd_cycles = m["GRBM_GUI_ACTIVE"] / 8.0             # the counter sums the 8 XCDs
    simd_quads = 256 * 4 * xcd_cycles / 4.0
    rec = {
        "kernel": ks[0][:120], "workload": workload, "precision": precision, "kernel_sha": kernel_hash(kernel),
        "counters": {c: m[c] for c in sorted(m)},
        "duration_us": xcd_cycles / 2400.0,
        "valu_busy": m["SQ_ACTIVE_INST_VALU"] / simd_quads,
        "waves_per_cu": 4.0 * m["SQ_WAVE_CYCLES"] / m["SQ_BUSY_CU_CYCLES"],
        "mem_wait": m["SQ_WAIT_INST_ANY"] / m["SQ_WAVE_CYCLES"],
        "lds_conflict": m["SQ_LDS_BANK_CONFLICT"] / m["SQ_LDS_IDX_ACTIVE"],
        "valu_insts_per_wave": m["SQ_INSTS_VALU"] / m["SQ_WAVES"],
        "salu_insts_per_wave": m["SQ_INSTS_SALU"] / m["SQ_WAVES"],
        "commands": commands,
    }
    busy = rec["valu_busy"]
    if busy >= 0.7:
        rec["bound"] = "alu"
        rec["limiter"] = (f"VALU issue: {100 * busy:.0f}% of SIMD issue slots, {rec['waves_per_cu']:.1f} waves/CU, "
                          f"{100 * rec['mem_wait']:.0f}% of wave time in memory waits")
    else:
        rec["bound"] = "latency"
        rec["limiter"] = (f"latency and occupancy: VALU {100 * busy:.0f}% of SIMD issue slots, "
                          f"{rec['waves_per_cu']:.1f} waves/CU, {100 * rec['mem_wait']:.0f}% of wave time in "
                          f"memory waits, LDS conflicts {100 * rec['lds_conflict']:.0f}%")
    json.dump(rec, open(out_path, "w"), indent=1)
    print(json.dumps({k: v for k, v in rec.items() if k != "counters"}))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:10])
    elif sys.argv[1] == "sq":
        sq(*sys.argv[2:])
