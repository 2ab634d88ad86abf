"""Benchmark: the hybrid multi-time-step FEM/LBM step on one MI355X.

A "step" is one coarse step of Algorithm 1.  By default the workload is the
precision form at 4096^2 (pore4096: D2Q9 lattice with random solid disks at
porosity 0.6, seeded 8-mode stream-function velocity, D = 1e-2, 16^2 Q1
mesh, eta = 4 fine steps per coarse step, 2 Schwarz passes) in FP64:
2 x {fine-to-coarse transfer, FP64 coarse solve, coarse-to-fine transfer,
4 lattice sweeps}, then commit.  Inputs are synthetic and seeded and
already resident in HBM when the timed region starts.

The printed JSON line reports lattice updates per second over all nodes
(MLUPS); the roofline of the dominant lattice-sweep kernel (algorithmic
bytes per launch over its average duration, timed with HIP events on its
stream, next to the HBM bytes the counters measured for it); FP32 and FP16
shifted storage on the same GPU, with their relative L2 errors against FP64
after the timed steps and after all of the workload's coarse steps; and the
CPU oracle timed on a bounded sample on this host (all threads and one).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1601_02708_amd.profiling import kernel_hash  # noqa: E402

METRIC = "ADE-LBM MLUPS + % HBM peak; FP32/adjoint vs FP64 plain at stated L2 error"
HBM_PEAK_GBS = 8000.0

def sweep_bytes(problem, elem_bytes):
    """Algorithmic HBM bytes of one lattice-sweep launch (every node of the
    patch): per fluid node 9 population loads + 9 stores, 2 FP32 velocity
    components and the 16-bit flag word; a solid node reads only its flag
    word; each perimeter slot also reads its two FP64 interface values.
    The two-step launch needs the same bytes (the state between its two
    fine steps never leaves the chip), for twice the lattice updates."""
    N = problem.cfg.N
    fluid = int((problem.solid == 0).sum())
    solid = N * N - fluid
    per_fluid = 18 * elem_bytes + 8 + 2
    return fluid * per_fluid + solid * 2 + 4 * (N - 1) * 16, fluid, solid, per_fluid


ELEM = {"fp64": 8, "fp32": 4, "fp16s": 2}


def launch_plan(eta, steps_per_launch):
    """Fine steps of each sweep launch of one Schwarz pass of eta fine steps,
    as the library plans a pass (hyb_set_steps_per_launch; fixed solids,
    every slot Dirichlet): as many steps as allowed, with no lone single
    step where it can be avoided (eta = 10: 4 + 3 + 3 at 4, 3 + 3 + 2 + 2 at
    3, five pairs at 2)."""
    out, rem = [], eta
    while rem > 0:
        if rem <= 1 or steps_per_launch == 1:
            t = 1
        elif steps_per_launch == 2 or rem == 2:
            t = 2
        elif steps_per_launch == 3:
            t = 2 if rem == 4 else 3
        elif steps_per_launch == 4:
            t = 3 if rem in (3, 5, 6) else 4
        else:
            t = 3 if rem == 6 else 4 if rem in (7, 8) else min(rem, 5)
        out.append(t)
        rem -= t
    return out


def default_steps_per_launch(precision):
    """The library's default (hyb_set_steps_per_launch): 5 for FP32, 4 for
    FP64, 4 for FP16 shifted storage."""
    return {"fp32": 5, "fp64": 4, "fp16s": 4}[precision]


def sweep_kernel(elem_bytes, take):
    """Symbol of the whole-patch launch (tile part 0) of the sweep that
    takes `take` fine steps per launch."""
    t = {8: "double", 4: "float", 2: "_Float16"}[elem_bytes]
    nt = 512 if elem_bytes == 8 or take >= 3 else 256
    if take >= 2:
        return f"lbm_sweep{take}_kernel<{t}, 64, 8, {nt}, 0>"
    return f"lbm_sweep_kernel<{t}>"


def _profile_record(kind, workload, precision, kernel):
    """A committed counter record profiles/<kind>_<workload>_<precision>.json
    of this kernel, or None when there is none or the kernel source changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    name = kernel.split("<")[0]
    if rec.get("kernel_sha") != kernel_hash(name) or not (name + "<" in rec.get("kernel", "") or
                                                         name + "I" in rec.get("kernel", "")):
        return None
    return rec


def load_traffic(workload, precision, kernel):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE
    record of this kernel (scaled by a plain copy's counters), or None."""
    rec = _profile_record("traffic", workload, precision, kernel)
    return None if rec is None else rec.get("bytes_per_launch")


def load_limiter(workload, precision, kernel, kind="sq"):
    """The limiter the committed SQ counter record of this kernel names
    (its 'bound' and a one-line 'limiter' reading of the counters), or
    None."""
    rec = _profile_record(kind, workload, precision, kernel)
    return None if rec is None else {"bound": rec.get("bound"), "limiter": rec.get("limiter")}


def final_step_errors(problem, ref_precision, others):
    """Each precision's fine (fluid nodes) and coarse concentration after
    all of the workload's coarse steps, each from a fresh handle at the
    library's default launch plan; relative L2 of the others against
    ref_precision's.  (The parity tests hold the FP64 path to the oracle at
    1e-12 at this step.)"""
    import numpy as np
    from paper_1601_02708_amd import hyb
    cfg = problem.cfg
    fluid = problem.solid == 0
    res = {}
    for prec in [ref_precision] + list(others):
        g = hyb.Hybrid.from_problem(problem, precision=prec, device="cuda:0")
        for _ in range(cfg.steps):
            g.step(cfg.max_iter)
        res[prec] = (g.concentration()[fluid], g.concentration(hyb.HYB_COARSE).reshape(-1))
        g.close()
    uf, dc = res[ref_precision]
    return {p: {"fine": float(np.linalg.norm(res[p][0] - uf) / np.linalg.norm(uf)),
                "coarse": float(np.linalg.norm(res[p][1] - dc) / np.linalg.norm(dc)),
                "coarse_steps": cfg.steps} for p in others}


def tune_overlap(problem, precision, steps_per_launch=None):
    """Overlap depth the library's own tuning picks for this workload, found
    on a throwaway handle (its steps are not part of any measurement)."""
    from paper_1601_02708_amd import hyb
    g = hyb.Hybrid.from_problem(problem, precision=precision, device="cuda:0")
    g.set_steps_per_launch(steps_per_launch or default_steps_per_launch(precision))
    g.set_overlap(hyb.HYB_OVERLAP_AUTO)
    for _ in range(2 + 3 * (problem.cfg.eta // 2 + 1)):
        if g.stats()["overlap_depth"] >= 0:
            break
        g.step(problem.cfg.max_iter)
    depth = g.stats()["overlap_depth"]
    g.close()
    return depth


def run_gpu(problem, precision, steps, warmup, steps_per_launch=None, depth=None, timing_steps=10):
    """W warmup and K timed coarse steps at the given overlap depth; then
    timing_steps more at depth 0 with kernel timing (every sweep launch
    whole and on the handle's stream: the sweep time of a step), and, for
    each kind of launch in the pass's plan, timing_steps chains of that
    kind alone, for its average launch duration: restarted passes of as
    many of its fine steps as fit in eta, taken by that kind only (eta = 10,
    three-step launches: 9 steps in three launches, each reading the
    previous one's output as inside a pass; a launch repeated on one source
    buffer would re-read data left in the 256 MB last-level cache and look
    faster than it runs in a pass), each call bracketed by HIP events on the
    handle's stream.  Returns the average launch duration (ms) per kind."""
    import torch
    from paper_1601_02708_amd import hyb
    steps_per_launch = steps_per_launch or default_steps_per_launch(precision)
    g = hyb.Hybrid.from_problem(problem, precision=precision, device="cuda:0")
    g.set_steps_per_launch(steps_per_launch)
    if depth is None:
        depth = tune_overlap(problem, precision, steps_per_launch)
    g.set_overlap(depth)
    mi = problem.cfg.max_iter
    for _ in range(warmup):
        g.step(mi)
    stream = g.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        g.step(mi)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    st = g.stats()
    kms, launches = 0.0, 0
    if timing_steps > 0:
        g.set_overlap(0)
        g.kernel_timing(True)
        for _ in range(timing_steps):
            g.step(mi)
        torch.cuda.synchronize()
        kms, launches = g.kernel_time()
        kinds = {}
        eta = problem.cfg.eta
        for take in sorted(set(launch_plan(eta, steps_per_launch))):
            g.set_steps_per_launch(take)
            for _ in range(timing_steps):
                g.lbm_substeps(take * (eta // take), restart=1)
            torch.cuda.synchronize()
            ms_k, n_k = g.kernel_time()
            kinds[take] = (ms_k / max(n_k, 1), n_k)
        g.kernel_timing(False)
        g.set_steps_per_launch(steps_per_launch)
        g.lbm_substeps(0, restart=1)          # back to the committed state
        g.set_overlap(depth)
    else:
        kinds = {}
    return g, wall, gpu_ms, kms, launches, st, depth, kinds


def dominant(kinds, eta, steps_per_launch):
    """(fine steps per launch, average launch ms, launches timed) of the
    launch kind with the most sweep time per pass."""
    plan = launch_plan(eta, steps_per_launch)
    take = max(kinds, key=lambda t: plan.count(t) * kinds[t][0])
    return take, kinds[take][0], kinds[take][1]


def adjoint_rate(problem, precision, reps=3):
    """Reverse mode of one coarse step's fine steps (hyb_lbm_substeps_record,
    then hyb_lbm_adjoint) on the same workload; MLUPS of the adjoint sweep
    (all nodes x eta fine steps) and of the recording forward sweep."""
    import torch
    from paper_1601_02708_amd import hyb
    g = hyb.Hybrid.from_problem(problem, precision=precision, device="cuda:0")
    g.interface_exchange(hyb.HYB_F2C)
    g.coarse_step()
    g.interface_exchange(hyb.HYB_C2F)
    eta, N = problem.cfg.eta, problem.cfg.N
    tape = g.adjoint_tape(eta)
    P = 4 * (N - 1)
    lam = torch.ones((9, N, N), dtype=torch.float64, device=g.dev)
    lam_out = torch.empty_like(lam)
    ga = torch.zeros(P, dtype=torch.float64, device=g.dev)
    gb = torch.zeros_like(ga)
    gk = torch.zeros((N, N), dtype=torch.float64, device=g.dev)
    s = g.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    rec_ms = adj_ms = 0.0
    for r in range(reps + 1):
        ev[0].record(s)
        g.substeps_record(eta, tape)
        ev[1].record(s)
        g.adjoint(eta, tape, lam, lam_out, ga, gb, gk)
        ev[2].record(s)
        torch.cuda.synchronize()
        if r > 0:                       # the first pass warms up
            rec_ms += ev[0].elapsed_time(ev[1])
            adj_ms += ev[1].elapsed_time(ev[2])
    lups = eta * N * N * reps
    # algorithmic bytes of one reversed fine step (reversed in pairs, two
    # per launch of adj_step2_kernel, the cotangent between them on chip): per
    # fluid node the cotangent read and the result written (9 values each),
    # the recorded u of the step's collision (one value, for dJ/dk), flags,
    # velocity and the FP64 dJ/dk read-modify-write; per solid node its flags
    # and the zeros written
    s = 8 if precision == "fp64" else 4
    nfl = int((problem.solid == 0).sum())
    step_bytes = nfl * (19 * s + 2 + 8 + 16) + (N * N - nfl) * (2 + 9 * s)
    kernel = f"adj_step2_kernel<{'double, 64, 8, 512' if s == 8 else 'float, 64, 8, 256'}>"
    lim = load_limiter(problem.cfg.name, precision, kernel, kind="sq_adjoint")
    step_ms = adj_ms / (reps * eta)
    out = {"precision": precision, "value": round(lups / (adj_ms / 1e3) / 1e6, 1), "unit": "MLUPS",
           "ms_per_fine_step": round(step_ms, 4),
           "record_forward_mlups": round(lups / (rec_ms / 1e3) / 1e6, 1),
           "roofline": {"kernel": kernel + " (two reversed steps per launch)",
                        "bound": lim["bound"] if lim else "hbm", "limiter": lim["limiter"] if lim else None,
                        "algorithmic_bytes_per_step": int(step_bytes),
                        "achieved": round(step_bytes / (step_ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(step_bytes / (step_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        "note": "time per reversed fine step of the whole call (the dense FP64 cotangent is "
                                "read and written by the first and last reversed launches, no packing passes)"},
           "note": "dJ/df*, dJ/da, dJ/db, dJ/dk over one coarse step's fine steps (tape of eta + 4 states and eta recorded u planes)"}
    g.close()
    return out


def step_adjoint_rate(problem, precision, reps=3):
    """Reverse mode of one whole coarse step (hyb_step_record, then
    hyb_step_adjoint: every Schwarz pass's fine steps, transfers and coarse
    solve transposed); MLUPS over the step's lattice updates (passes x eta x
    all nodes) for the adjoint and for the recording forward."""
    import torch
    from paper_1601_02708_amd import hyb
    g = hyb.Hybrid.from_problem(problem, precision=precision, device="cuda:0")
    cfg = problem.cfg
    passes, eta, N = cfg.max_iter, cfg.eta, cfg.N
    tape = g.step_tape(passes)
    lam_f = torch.ones((9, N, N), dtype=torch.float64, device=g.dev)
    lam_d = torch.ones((cfg.M + 1) ** 2, dtype=torch.float64, device=g.dev)
    out_f = torch.empty_like(lam_f)
    out_d = torch.empty_like(lam_d)
    gk = torch.zeros((N, N), dtype=torch.float64, device=g.dev)
    s = g.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    rec_ms = adj_ms = 0.0
    for r in range(reps + 1):
        ev[0].record(s)
        g.step_record(passes, tape)
        ev[1].record(s)
        g.step_adjoint(tape, lam_f, lam_d, out_f, out_d, gk)
        ev[2].record(s)
        torch.cuda.synchronize()
        if r > 0:                       # the first pass warms up
            rec_ms += ev[0].elapsed_time(ev[1])
            adj_ms += ev[1].elapsed_time(ev[2])
    lups = passes * eta * N * N * reps
    res = {"precision": precision, "value": round(lups / (adj_ms / 1e3) / 1e6, 1), "unit": "MLUPS",
           "ms_per_coarse_step": round(adj_ms / reps, 4),
           "record_forward_mlups": round(lups / (rec_ms / 1e3) / 1e6, 1),
           "tape_bytes": int(tape.numel()),
           "note": "dJ/df*(t_n), dJ/dd^n, dJ/dk through one coarse step of Algorithm 1 "
                   "(fine steps, transfers and the transposed coarse solve of every Schwarz pass)"}
    g.close()
    return res


def dissolution_adjoint(g, cfg, substeps=1000, checkpoint_every=10):
    """Reverse mode over the last `substeps` fine steps of the dissolving run
    (substeps / eta coarse steps from the handle's state, each with its
    Schwarz passes): J = sum of all populations after them (the fluid's
    total concentration times 1 - k), gradient with respect to the per-node
    reaction rate k, the initial state and the coarse state, through
    steps_adjoint (device checkpoints of populations, coarse state, solids
    and masses every `checkpoint_every` steps; every step re-run once,
    recorded, and reversed on the GPU).  Also one record + adjoint pair timed
    alone with HIP events."""
    import numpy as np
    import torch
    from paper_1601_02708_amd import hyb
    N, P = cfg.N, cfg.max_iter
    n = substeps // cfg.eta
    ones = np.ones((9, N, N))
    conv0 = g.dissolution_state()[2]
    t0 = time.perf_counter()
    lF, ld, gk, _ = hyb.steps_adjoint(g, n, lambda k, F, d: (ones, None) if k == n else (None, None), P,
                                      checkpoint_every=checkpoint_every, state_in_cotangent=False)
    wall = time.perf_counter() - t0
    conv1 = g.dissolution_state()[2]
    # one step's record and adjoint alone, on the GPU clock
    tape = g.step_tape(P)
    lf = torch.ones((9, N, N), dtype=torch.float64, device=g.dev)
    lfo = torch.empty_like(lf)
    ld_ = torch.zeros((cfg.M + 1) ** 2, dtype=torch.float64, device=g.dev)
    ldo = torch.empty_like(ld_)
    gk1 = torch.zeros((N, N), dtype=torch.float64, device=g.dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(g.stream)
    g.step_record(P, tape)
    ev[1].record(g.stream)
    g.step_adjoint(tape, lf, ld_, lfo, ldo, gk1)
    ev[2].record(g.stream)
    torch.cuda.synchronize()
    rec_ms, adj_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    lups = P * cfg.eta * N * N
    tape_bytes = int(tape.numel())
    del tape
    return {"substeps": n * cfg.eta, "coarse_steps": n, "checkpoint_every": checkpoint_every,
            "objective": "sum of all populations after the last step", "wrt": "per-node reaction rate k, f*(t0), d(t0)",
            "wall_s": round(wall, 2), "solids_converted_in_window": int(conv1 - conv0),
            "grad_k_l2": float(np.linalg.norm(gk)), "grad_k_finite": bool(np.isfinite(gk).all()),
            "step_record_ms": round(rec_ms, 3), "step_adjoint_ms": round(adj_ms, 3),
            "step_adjoint_mlups": round(lups / (adj_ms / 1e3) / 1e6, 1), "tape_bytes": tape_bytes,
            "mlups_whole_reverse": round(n * lups / wall / 1e6, 1),
            "note": "wall time: forward rollout with checkpoints, segment re-runs, every step's record and "
                    "reverse; step_* are one coarse step's record and reverse alone on the GPU clock"}


def differentiation(directions=2, eps=1e-3):
    """The differentiation workload (diff512: 512^2 patch, porosity 0.6, in a
    64^2 mesh; inlet x = 0 held at 1, the other outer edges natural; fine
    rate field U[0, 2e-4]; 200 coarse steps of 10 substeps, one Schwarz
    pass): J = the outflow moment through the patch's right edge summed over
    every one of the 2000 fine steps (the time integral at the fine step),
    and its gradient in (k field, inlet value) through
    hyb.trajectory_functional(every_substep=True) (checkpoints every 10
    coarse steps = 100 substeps).  Per precision: the forward's MLUPS (J accumulated on the
    device each step), the gradient's wall time and MLUPS over the
    trajectory's lattice updates (backward = checkpointed forward, segment
    re-runs, every step recorded and reversed), their ratio; FP64 also
    central differences along `directions` seeded directions, and FP32's
    gradient against FP64's."""
    import numpy as np
    import torch
    from paper_1601_02708_amd import configs, hyb
    cfg = configs.DIFF512
    p = configs.build_problem(cfg)
    N = cfg.N
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], np.float64)
    w = np.zeros((9, N, N))
    w[:, :, N - 1] = ex[:, None]
    w[:, p.solid != 0] = 0.0
    lups = cfg.steps * cfg.eta * cfg.max_iter * N * N
    Functional = hyb.trajectory_functional(every_substep=True)
    out, grads = {}, {}
    for prec in ("fp64", "fp32"):
        g = hyb.Hybrid.from_problem(p, precision=prec, device="cuda:0")
        start = g.checkpoint()

        def J_of(kf, gv):
            g.restore(start)
            return Functional.apply(g, cfg.steps, cfg.max_iter, 10, w, None, kf, gv)

        with torch.no_grad():                                  # warm-up
            J_of(torch.from_numpy(p.k_field), torch.tensor(cfg.outer_value, dtype=torch.float64))
        k = torch.tensor(p.k_field, dtype=torch.float64, requires_grad=True)
        gv = torch.tensor(cfg.outer_value, dtype=torch.float64, requires_grad=True)
        g.restore(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = Functional.apply(g, cfg.steps, cfg.max_iter, 10, w, None, k, gv)
        Jv = float(J.detach())
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gk = k.grad.numpy().copy()
        grads[prec] = (gk, float(gv.grad))
        rec = {"J": Jv, "forward_s": round(t1 - t0, 4), "forward_mlups": round(lups / (t1 - t0) / 1e6, 1),
               "gradient_s": round(t2 - t1, 4), "gradient_mlups": round(lups / (t2 - t1) / 1e6, 1),
               "gradient_over_forward": round((t2 - t1) / (t1 - t0), 2),
               "dJ_dg": float(gv.grad), "grad_k_l2": float(np.linalg.norm(gk))}
        if prec == "fp64":
            rng = np.random.default_rng(cfg.seed + 7000)
            rels = []
            with torch.no_grad():
                for _ in range(directions):
                    dk = rng.uniform(-1.0, 1.0, (N, N)) * p.k_field
                    dk[p.solid != 0] = 0.0
                    dg = float(rng.uniform(-1.0, 1.0))
                    jp = float(J_of(torch.from_numpy(p.k_field + eps * dk),
                                    torch.tensor(cfg.outer_value + eps * dg, dtype=torch.float64)))
                    jm = float(J_of(torch.from_numpy(p.k_field - eps * dk),
                                    torch.tensor(cfg.outer_value - eps * dg, dtype=torch.float64)))
                    fd = (jp - jm) / (2 * eps)
                    an = float(np.sum(gk * dk)) + grads[prec][1] * dg
                    rels.append(abs(fd - an) / abs(fd))
            rec["central_difference_rel"] = [float(f"{r:.3g}") for r in rels]
        out[prec] = rec
        g.close()
    ref = grads["fp64"][0]
    out["fp32"]["grad_k_rel_vs_fp64"] = float(np.abs(grads["fp32"][0] - ref).max() / np.abs(ref).max())
    out["workload"] = (f"diff512: {N}^2 lattice (porosity {p.porosity:.4f}), {cfg.M}^2 mesh, inlet x=0 at "
                       f"{cfg.outer_value}, other edges natural, k field U[0, {cfg.k_field_max}], "
                       f"{cfg.steps} coarse steps x {cfg.eta} substeps, MaxIter {cfg.max_iter}")
    out["note"] = ("J = sum over all fine steps of the x-moment of f* on the patch's right edge; the forward reads "
                   "every fine state (single-step launches); gradient wall time includes the checkpointed re-run, "
                   "every step's record and reverse with the cotangent injected at every fine state (checkpoints "
                   "every 100 substeps); MLUPS over the trajectory's lattice updates")
    return out


def dissolution_rate(steps=20, warmup=2, timing_steps=3, adjoint=True):
    """The dissolving-solid workload (4096^2, porosity 0.5, FP32, eta = 20,
    256^2 mesh, 2 Schwarz passes, surface reaction at every fluid-solid link,
    seeded per-solid masses): K timed coarse steps after W warmup steps on
    the caller's stream (the commit's mass update, conversions and flag
    rebuild included), MLUPS over all nodes, the solids converted, and the
    sweep's average launch duration with its algorithmic bytes (fluid nodes
    as in the plain sweep, for the launch's fine steps -- five at eta = 20
    with the library's default; each solid node with a fluid neighbour also
    reads and writes its FP64 link-flux sum once per launch)."""
    import numpy as np
    import torch
    from paper_1601_02708_amd import configs, hyb
    cfg = configs.DISSOLVE4096
    p = configs.build_problem(cfg)
    N = cfg.N
    g = hyb.Hybrid.from_problem(p, precision="fp32", device="cuda:0", dissolution=True)
    g.set_dissolution(cfg.kappa_s, cfg.c_sat, configs.solid_mass(cfg, p.solid))
    for _ in range(warmup):
        g.step(cfg.max_iter)
    _, _, conv0 = g.dissolution_state()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(g.stream)
    for _ in range(steps):
        g.step(cfg.max_iter)
    e1.record(g.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sol, _, conv1 = g.dissolution_state()
    g.kernel_timing(True)
    for _ in range(timing_steps):
        g.step(cfg.max_iter)
    kms, launches = g.kernel_time()
    g.kernel_timing(False)
    sol2, _, conv2 = g.dissolution_state()
    adj = None
    if adjoint:
        print("[bench] dissolving solids: reverse mode over the last 1000 fine steps", file=sys.stderr, flush=True)
        adj = dissolution_adjoint(g, cfg)
    # geometry of the timing steps (their own commits convert after them)
    s = sol != 0
    pad = np.pad(~s, 1, constant_values=False)
    fluid_nb = np.zeros_like(s)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if di or dj:
                fluid_nb |= pad[1 + dj:1 + dj + N, 1 + di:1 + di + N]
    surface = int((s & fluid_nb).sum())
    nfl = int((~s).sum())
    plan = launch_plan(cfg.eta, default_steps_per_launch("fp32"))
    k_avg = cfg.eta / len(plan)             # fine steps per launch (uniform at eta = 20: 5)
    launch_bytes = k_avg * (nfl * (18 * 4 + 8 + 2) + (N * N - nfl) * 2 + 4 * (N - 1) * 16) + surface * 16
    avg = kms / max(launches, 1)
    lups = steps * cfg.max_iter * cfg.eta * N * N
    g.close()
    out_adj = {} if adj is None else {"adjoint_fp32": adj}
    return {"workload": (f"{cfg.name}: {N}^2 D2Q9 lattice, random disks (porosity {p.porosity:.4f}), 8-mode "
                         f"stream-function velocity max 0.05, D={cfg.D}, k={cfg.k}, {cfg.M}^2 Q1 SUPG mesh, "
                         f"eta={cfg.eta}, {cfg.max_iter} Schwarz passes; surface reaction kappa_s={cfg.kappa_s} "
                         f"towards c_sat={cfg.c_sat}, solid masses U{list(cfg.mass_range)}"),
            "precision": "fp32", "value": round(lups / (ms / 1e3) / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(ms / steps, 4), "steps": steps, "warmup": warmup,
            "converted_in_timed_steps": int(conv1 - conv0), "converted_total": int(conv2),
            "solid_nodes_now": int(sol2.sum()),
            "sweep_kernel": (f"lbm_sweepk_flux_kernel<float, 64, 8, 512, {plan[0]}> (launches {plan}, link fluxes at "
                             "solid nodes)" if plan[0] >= 3 else
                             "lbm_sweep2_flux_kernel<float, 64, 8, 256> (two fine steps, link fluxes at solid nodes)"),
            "sweep_avg_launch_ms": round(avg, 5),
            "sweep_algorithmic_bytes_per_launch": int(launch_bytes),
            "sweep_achieved_gbs": round(launch_bytes / (avg / 1e3) / 1e9, 1),
            "sweep_frac": round(launch_bytes / (avg / 1e3) / 1e9 / HBM_PEAK_GBS, 4), **out_adj}


def hybrid1d_tables():
    """The 1-D hybrid of Sec. 7.1 on the GPU for every printed row of the
    Gaussian-hill tables (tests/golden/gauss1d_tables.txt): the run to
    T = 0.4 in one launch per row (one workgroup), its coarse and fine
    max-norm errors against the closed-form solution next to the printed
    ones, and the GPU time per coarse step; the oracle (NumPy, one thread)
    timed on one row."""
    import numpy as np
    import torch
    from paper_1601_02708_amd import hyb, inputs
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "gauss1d_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        t, r, hc, hf, L, mi, ec, ef = line.split()
        rows.append((f"{t}r{r}", float(hc), float(hf), float(L), int(mi), float(ec), float(ef)))
    hybrid1d_tables.rows = rows
    out = []
    T = 0.4
    for key, hc, hf, L, mi, ec_p, ef_p in rows:
        g = hyb.Hybrid1D(hc, hf, L, mi, lambda x: inputs.gaussian_hill_1d(x, 0.0))
        n = int(round(T / g.dt_c))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(g.stream)
        g.run(n)
        e1.record(g.stream)
        d, u = g.state()
        ms = e0.elapsed_time(e1)
        ec = float(np.abs(d - inputs.gaussian_hill_1d(g.xc, T)).max())
        ef = float(np.abs(u - inputs.gaussian_hill_1d(g.xf, T)).max())
        out.append({"row": key, "h_c": hc, "h_f": hf, "L_ov": L, "max_iter": mi, "eta": g.eta, "coarse_steps": n,
                    "E_c": ec, "E_f": ef, "printed_E_c": ec_p, "printed_E_f": ef_p, "gpu_ms": round(ms, 3),
                    "us_per_coarse_step": round(1e3 * ms / n, 2)})
        g.close()
    return {"rows": out, "note": "E_f reproduces the printed fine-domain floor at the finest rows; the printed "
                                 "E_c are not reproduced (see the oracle's pins)"}


def cpu_baseline_1d(row, gpu_rows):
    """The 1-D oracle (NumPy, one thread) on one table row to T = 0.4."""
    from oracle.hybrid1d import Hybrid1D
    hc, hf, L, mi = row[1:5]
    o = Hybrid1D(hc, hf, L, mi)
    t0 = time.perf_counter()
    o.run(0.4)
    dt = time.perf_counter() - t0
    gpu = [r for r in gpu_rows if r["row"] == row[0]][0]
    return {"row": row[0], "seconds": round(dt, 3), "cores": 1, "kind": "oracle",
            "gpu_seconds": round(gpu["gpu_ms"] / 1e3, 4)}


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or 'unknown'."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_steps(problem, threads, min_seconds, max_steps):
    """Whole coarse steps of the oracle on `threads` threads (None: the
    OpenMP default) until min_seconds have been timed; (steps, seconds,
    threads used)."""
    import oracle
    if threads is not None:
        oracle.set_threads(threads)
    used = oracle.get_threads()
    o = oracle.HybridOracle(problem)
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step()
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or steps >= max_steps:
            break
    return steps, dt, used


def cpu_baseline(problem, min_seconds=8.0, max_steps=6):
    """The oracle as it stands on this host (its lattice loops split over
    rows by OpenMP, the rest serial): whole coarse steps (Schwarz passes x
    eta fine steps, FP64) of the same workload with every thread OpenMP
    gives it, then on one thread, each repeated until min_seconds of CPU
    work have been timed."""
    import oracle
    cfg = problem.cfg
    lups_step = cfg.max_iter * cfg.eta * cfg.N ** 2
    steps, dt, used = _oracle_steps(problem, None, min_seconds, max_steps)
    steps1, dt1, _ = _oracle_steps(problem, 1, min_seconds, max_steps)
    oracle.set_threads(used)
    what = (f"{cfg.name}: first {{}} coarse steps ({cfg.max_iter} Schwarz passes x {cfg.eta} fine steps on "
            f"{cfg.N}^2 nodes, plus the {cfg.M}^2 coarse solves, per step), FP64, {{}} thread(s), {{:.1f}} s")
    return {"value": round(steps * lups_step / dt / 1e6, 3), "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": what.format(steps, used, dt), "cpu_model": cpu_model(), "cpu_count": os.cpu_count(),
            "single_thread": {"value": round(steps1 * lups_step / dt1 / 1e6, 3), "unit": "MLUPS", "cores": 1,
                              "sample": what.format(steps1, 1, dt1)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pore4096")
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp64", "fp16s"])
    ap.add_argument("--steps-per-launch", type=int, default=None, choices=[1, 2, 3, 4, 5],
                    help="most fine steps per lattice-sweep launch (temporal blocking; eta = 10 runs 5 + 5 at 5, "
                         "4 + 3 + 3 at 4); default: the library's (5 fp32, 4 fp64, 4 fp16s)")
    ap.add_argument("--overlap", type=int, default=-1,
                    help="overlap depth of hyb_step (-1: the library's tuning, on a separate handle)")
    ap.add_argument("--timing-steps", type=int, default=10,
                    help="coarse steps at overlap depth 0 after the timed ones, for the sweep kernel's "
                         "average launch duration (roofline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode measurement")
    ap.add_argument("--no-compare", action="store_true", help="skip the other-precision runs")
    ap.add_argument("--no-dissolution", action="store_true", help="skip the dissolving-solid workload")
    ap.add_argument("--no-hybrid1d", action="store_true", help="skip the 1-D hybrid tables")
    ap.add_argument("--no-differentiation", action="store_true",
                    help="skip the differentiation workload (diff512) of the reverse-mode records")
    ap.add_argument("--dissolution-only", action="store_true",
                    help="run only the dissolving-solid workload and print its record (for profiling)")
    ap.add_argument("--differentiation-only", action="store_true",
                    help="run only the differentiation workload (diff512 gradient) and print its record")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (a plain copy kernel of "
                         "known size, for calibrating HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the lattice patch is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_1601_02708_amd import configs, hyb

    if args.differentiation_only:
        print(json.dumps({"differentiation": differentiation()}), flush=True)
        return
    if args.dissolution_only:
        print(json.dumps({"dissolution": dissolution_rate(adjoint=not args.no_adjoint)}), flush=True)
        return
    cfg = configs.CONFIGS[args.workload]
    problem = configs.build_problem(cfg)
    N = cfg.N
    lups_step = cfg.max_iter * cfg.eta * N * N
    fluid_frac = float((problem.solid == 0).mean())
    elem = ELEM[args.precision]
    print(f"[bench] {cfg.name} {args.precision}: {args.warmup} warmup + {args.steps} timed coarse steps",
          file=sys.stderr, flush=True)
    spl = args.steps_per_launch
    depth = tune_overlap(problem, args.precision, spl) if args.overlap < 0 else args.overlap
    print(f"[bench] overlap depth {depth}", file=sys.stderr, flush=True)
    g, wall, gpu_ms, kms, launches, st, _, kinds = run_gpu(problem, args.precision, args.steps, args.warmup,
                                                           spl, depth, args.timing_steps)
    ms_step = gpu_ms / args.steps
    value = lups_step * args.steps / (gpu_ms / 1e3) / 1e6
    bbytes, nfl, nsol, per_fluid = sweep_bytes(problem, elem)
    spl = spl or default_steps_per_launch(args.precision)
    steps_launch, avg_kernel_ms, dom_n = dominant(kinds, cfg.eta, spl)
    kname = sweep_kernel(elem, steps_launch)
    # algorithmic bytes per launch = bytes per fluid lattice update x the
    # updates one launch performs (its fine steps over every fluid node)
    launch_bytes = bbytes * steps_launch
    achieved = launch_bytes / (avg_kernel_ms / 1e3) / 1e9
    traffic = load_traffic(cfg.name, args.precision, kname)
    lim = load_limiter(cfg.name, args.precision, kname)
    res = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{cfg.name}: {N}^2 D2Q9 lattice, random disks (porosity {problem.porosity:.4f}), "
                         f"8-mode stream-function velocity max 0.05, D={cfg.D}, k={cfg.k}, {cfg.M}^2 Q1 SUPG mesh, "
                         f"eta={cfg.eta}, {cfg.max_iter} Schwarz passes per coarse step"),
            "lattice": N, "mesh": cfg.M, "eta": cfg.eta, "schwarz": cfg.max_iter, "precision": args.precision,
            "storage": {"fp64": "f64", "fp32": "f32", "fp16s": "f16 shifted"}[args.precision],
        },
        "mflups": round(value * fluid_frac, 1),
        "roofline": {
            "bound": lim["bound"] if lim else "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            # what the kernel really moves: the counters' bytes over the same
            # launch duration (the algorithmic figure counts every fine step
            # of a temporally blocked launch, the state crosses HBM once)
            "hbm_achieved": None if traffic is None else round(traffic / (avg_kernel_ms / 1e3) / 1e9, 1),
            "hbm_frac": None if traffic is None else round(traffic / (avg_kernel_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "limiter": lim["limiter"] if lim else None,
            "kernel": kname,
            "fine_steps_per_launch": steps_launch,
            "fluid_updates_per_launch": int(nfl * steps_launch),
            "bytes_per_fluid_update": round(bbytes / nfl, 2),
            "algorithmic_bytes_per_launch": int(launch_bytes),
            "avg_launch_ms": round(avg_kernel_ms, 5),
            "launches_timed": dom_n,
            "pass_plan": launch_plan(cfg.eta, spl),
            "avg_launch_ms_by_steps": {str(t): round(v[0], 5) for t, v in sorted(kinds.items())},
        },
        # sweep kernel time per coarse step (depth-0 timing steps) over the
        # step time of the timed (overlapped) steps
        "sweep_time_frac": round(kms / max(args.timing_steps, 1) / ms_step, 4),
        "overlap_depth": depth,
        "wall_s": round(wall, 3),
        "krylov_iters_last": st["krylov_iters"],
        "infeasible_closures": st["infeasible"],
    }
    if not args.no_compare:
        fluid = problem.solid == 0
        conc = {args.precision: g.concentration()}
        for other in [p for p in ("fp64", "fp16s", "fp32") if p != args.precision]:
            print(f"[bench] comparison run {other}", file=sys.stderr, flush=True)
            g2, _, gpu_ms2, kms2, launches2, _, d2, kinds2 = run_gpu(problem, other, args.steps, args.warmup,
                                                                     args.steps_per_launch, None, args.timing_steps)
            conc[other] = g2.concentration()
            e2 = ELEM[other]
            b2, _, _, _ = sweep_bytes(problem, e2)
            take2, k2, _ = dominant(kinds2, cfg.eta, args.steps_per_launch or default_steps_per_launch(other))
            kname2 = sweep_kernel(e2, take2)
            res[other] = {"value": round(lups_step * args.steps / (gpu_ms2 / 1e3) / 1e6, 1), "unit": "MLUPS",
                          "ms_per_step": round(gpu_ms2 / args.steps, 4), "overlap_depth": d2,
                          "sweep_kernel": kname2,
                          "sweep_achieved_gbs": round(b2 * take2 / (k2 / 1e3) / 1e9, 1),
                          "sweep_avg_launch_ms": round(k2, 5)}
            g2.close()
            del g2
        ref = conc["fp64"]
        nref = np.linalg.norm(ref[fluid])
        for p_, u_ in conc.items():
            if p_ != "fp64":
                key = "fp32_rel_l2_vs_fp64" if p_ == "fp32" else f"{p_}_rel_l2_vs_fp64"
                res[key] = float(np.linalg.norm((u_ - ref)[fluid]) / nref)
        print(f"[bench] final-step errors ({cfg.steps} coarse steps)", file=sys.stderr, flush=True)
        res["final_step_rel_l2_vs_fp64"] = final_step_errors(problem, "fp64", ["fp32", "fp16s"])
    if not args.no_adjoint and args.precision in ("fp32", "fp64"):
        print("[bench] adjoint", file=sys.stderr, flush=True)
        res["adjoint"] = adjoint_rate(problem, args.precision)
        res["step_adjoint"] = step_adjoint_rate(problem, args.precision)
        if not args.no_differentiation:
            print("[bench] differentiation workload (diff512)", file=sys.stderr, flush=True)
            res["differentiation"] = differentiation()
    if not args.no_hybrid1d:
        print("[bench] 1-D hybrid tables", file=sys.stderr, flush=True)
        res["hybrid1d"] = hybrid1d_tables()
    if not args.no_dissolution:
        print("[bench] dissolving solids (dissolve4096, fp32)", file=sys.stderr, flush=True)
        g.close()
        res["dissolution"] = dissolution_rate(adjoint=not args.no_adjoint)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, all threads and one thread)", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(problem)
        if "hybrid1d" in res:
            row = [r for r in hybrid1d_tables.rows if r[0] == "T1r3"][0]
            res["cpu_baseline"]["hybrid1d"] = cpu_baseline_1d(row, res["hybrid1d"]["rows"])
    if args.copy_mib > 0:
        import torch
        nbytes = args.copy_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = nbytes
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
