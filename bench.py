"""Benchmark of the HB residual + Runge-Kutta hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch32_mixed]

The batched kernel's launch configuration is autotuned first (outside the
timed region).  One step = one pseudo-time iteration of the whole hot path
over the workload: four Runge-Kutta stages (ghosts, MUSCL/Roe and viscous fluxes, HB
source D.Q, local time step, update), the residual norm and the force
coefficients of every body, as hb_rk_iterate(q, 1, resnorm, forces).
Inputs are seeded and synthetic and resident in HBM before timing starts.

Prints one JSON line: the FP32-bulk batched rate (value), the plain FP64
per-block rate beside it, the live roofline of the fused stage kernel
(HIP events around each stage launch on the launch stream), the HBM traffic
of that kernel from the committed rocprofv3 counter summary (when it was
taken on the current kernel source), the same kernel's ALU roofline on the
method's operation count per unit (counted on the oracle's own evaluation
in the CPU leg), and the FP64 CPU oracle timed on a bounded sample on the
host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# FP32 vector peak (packed FP32 counted; packed FP32 instructions are not
# used by this library, so half of it is the reachable vector rate)
PEAK_FP32_TFLOPS = 157.3
# VALU issue capacity: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a 64-wide
# wave's non-packed FP32 instruction occupies its SIMD for 4 cycles)
PEAK_VALU_LANE_INSTR = 256 * 4 * 16 * 2.4e9
METRIC = ("cell-snapshot RK-stage updates/s (FP32+batched vs FP64 plain); "
          "adjoint/primal time")
TUNE_CACHE = os.path.join(ROOT, "paper_1304_7654_amd", "tune_cache.json")
KERNEL_SOURCES = ["paper_1304_7654_amd/csrc/hb_fused_kernel.hpp", "paper_1304_7654_amd/csrc/hb_device.hpp"]


def code_text(src: str) -> str:
    """Source text without comments and blank-space differences, so that a
    comment edit does not count as a kernel change."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_hash() -> str:
    """Hash of the stage kernel's code (comments excluded), recorded in the
    counter summaries taken on it."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def read_profile_value(path, key, tuning, workload):
    """A per-launch figure of the fused stage kernel from a committed counter
    summary, or None when it is missing or was taken on another workload,
    kernel source or launch configuration."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("workload") != workload or kv.get("kernel_source_hash") != kernel_hash():
        return None
    t = "%d,%d,%d,%d" % (tuning["tile_i"], tuning["wg_per_cu"], tuning["xcd_order"],
                         tuning["tile_order"])
    if kv.get("tuning") != t:
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def profile_file(workload, what):
    """Committed counter summary of the fused stage kernel on a workload."""
    return os.path.join(ROOT, "profiles", "fused_stage_%s_%s.txt" % (workload, what))


def read_traffic(tuning, workload):
    """HBM bytes per fused stage launch (FETCH_SIZE / WRITE_SIZE summary)."""
    return read_profile_value(profile_file(workload, "traffic"), "bytes_per_launch", tuning, workload)


def algorithmic_bytes_per_iteration(problem) -> float:
    """Bytes the method must move per FP32-bulk iteration (4 stages), the
    FP32-stage-shadow variant of the algorithmic count: stage 1 reads Q (FP64,
    32 B per cell-snapshot) and writes the FP32 stage state (16); stages 2-3
    read the stage state (16) and Q (32) and write (16); stage 4 reads the
    stage state (16) and Q (32) and writes Q (32): 64 B per cell-snapshot
    and stage on average.  Metrics: 5 FP32 words per cell and stage (two face
    normals and the area; the face normals of the far sides belong to the
    neighbours), so 64 + 20/N_s B per unit."""
    cs = problem.cell_snapshots
    cells = sum(b.ni * b.nj for b in problem.blocks)
    return cs * (48 + 64 + 64 + 80) + 4 * 20 * cells


def design_bytes_per_iteration(problem) -> float:
    """The same with the 9 FP32 metric words per cell that the fused kernel
    reads (it also reads the two centre offsets of the viscous diamonds
    instead of forming them from the nodes): 64 + 36/N_s B per unit."""
    cs = problem.cell_snapshots
    cells = sum(b.ni * b.nj for b in problem.blocks)
    return cs * (48 + 64 + 64 + 80) + 4 * 36 * cells


def plain_algorithmic_stage_bytes(problem) -> float:
    """Bytes one FP64 stage must move by the method (FP64 stage states): read
    the stage input (32 B per cell-snapshot), read Q(0) (32, stages 2-4) and
    write the new state (32): (64 + 3 x 96)/4 = 88 B per cell-snapshot and
    stage on average, plus 5 FP64 metric words per cell (40 B), so
    88 + 40/N_s B per unit."""
    cs = problem.cell_snapshots
    cells = sum(b.ni * b.nj for b in problem.blocks)
    return 88.0 * cs + 40.0 * cells


# rigid motion of the moving-grid leg: 0.3 rad of pitch about the quarter
# chord, leading a heave of 1.5 length units by 0.5 rad
MOTION = dict(pitch_amp=0.3, pitch_phase=0.5, heave_amp=1.5, x_pivot=0.25, y_pivot=0.0)


def plain_stage_bytes(problem, moving) -> float:
    """Bytes one stage of the plain FP64 path's own design moves (every
    intermediate in HBM; not the method's algorithmic bytes): the ghost fill reads Q and writes the ghost-extended
    primitives E; each face family (one kernel for both) reads E and its face
    metrics (S, d) and writes its face fluxes; the update reads both flux
    arrays, the stage input, the base state, the face normals and the cell
    area, and writes the new state.  A moving grid adds the node coordinates
    (both face kernels) and the cell centres (update).  FP64 words."""
    tot = 0
    for b in problem.blocks:
        ni, nj, ns = b.ni, b.nj, b.ns
        q = 4 * ni * nj * ns
        ext = 4 * (ni + 4) * (nj + 4) * ns
        fi, fj = 4 * (ni + 1) * nj * ns, 4 * ni * (nj + 1) * ns
        mi, mj = 4 * (ni + 1) * nj, 4 * ni * (nj + 1)
        words = ((q + ext) + (ext + mi + fi) + (ext + mj + fj)
                 + (fi + fj + 3 * q + mi // 2 + mj // 2 + ni * nj))
        if moving:
            words += 4 * (ni + 1) * (nj + 1) + 2 * ni * nj
        tot += 8 * words
    return float(tot)


def plain_leg(torch, hb, problem, q0, steps, motion=None):
    """Plain FP64 per-block path: throughput with loads every iteration, and
    its stage time from HIP events around every stage (on the launch
    stream) for the roofline over the method's algorithmic bytes
    (plain_algorithmic_stage_bytes; the design's own traffic beside it)."""
    cs = problem.cell_snapshots
    stages = len(problem.solver.rk_alpha)
    g = hb.Grid(problem.blocks, problem.flow, problem.solver, precision=0, batched=0)
    if motion:
        g.set_motion(**motion)
    q = q0.clone()
    time_steps(torch, g, q, 1)
    q = q0.clone()
    t, _ = time_steps(torch, g, q, steps)
    assert g.status() == hb.HB_OK, "non-finite state in the plain FP64 run"
    q = q0.clone()
    g.profile_stages(True)
    time_steps(torch, g, q, steps, forces=False)
    ms, n = g.stage_stats()
    g.profile_stages(False)
    g.close()
    stage_s = ms / 1000.0 / n
    abytes = plain_algorithmic_stage_bytes(problem)
    dbytes = plain_stage_bytes(problem, bool(motion))
    return {"value": cs * stages * steps / t, "ms_per_step": 1000.0 * t / steps,
            "roofline": {"bound": "hbm", "achieved": abytes / stage_s / 1e9, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": abytes / stage_s / 1e9 / PEAK_HBM_GBS,
                         "kernels": "per block: k_ghost, k_flux (i- and j-faces), k_update",
                         "avg_stage_ms": 1000.0 * stage_s, "algorithmic_bytes_per_stage": abytes,
                         # the plain design's own HBM intermediates (ghost-extended
                         # primitives, face fluxes) on top of the method's bytes
                         "design_bytes_per_stage": dbytes,
                         "design_gbs": dbytes / stage_s / 1e9}}


def moving_leg(torch, hb, problem, q0, steps, tuning, motion):
    """The product path (FP32 bulk, batched fused kernel) on the rigidly
    heaving and pitching grid, with the fixed-grid run's tuning: throughput
    with loads every iteration, and the mean stage launch time from HIP
    events around every stage (on the launch stream)."""
    cs = problem.cell_snapshots
    stages = len(problem.solver.rk_alpha)
    g = hb.Grid(problem.blocks, problem.flow, problem.solver, precision=1, batched=1)
    g.set_tuning(tuning["tile_i"], tuning["wg_per_cu"], tuning["xcd_order"], tuning["tile_order"])
    g.set_motion(**motion)
    q = q0.clone()
    time_steps(torch, g, q, 1)
    q = q0.clone()
    t, _ = time_steps(torch, g, q, steps)
    assert g.status() == hb.HB_OK, "non-finite state in the moving-grid run"
    q = q0.clone()
    g.profile_stages(True)
    time_steps(torch, g, q, steps, forces=False)
    ms, n = g.stage_stats()
    g.profile_stages(False)
    g.close()
    return {"value": cs * stages * steps / t, "ms_per_step": 1000.0 * t / steps,
            "avg_stage_ms": ms / n, "path": "fused FP32 bulk, batched", "motion": motion}


def stream_probe(torch, mib=1024, reps=10):
    """Device copy bandwidth (read + write bytes per second) of a plain
    torch copy of `mib` MiB, the practical HBM peak the traffic is also set
    against."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def time_steps(torch, g, q, steps, forces=True):
    cf = torch.empty(g.n_forces, dtype=torch.float64, device=q.device) if forces else None
    norms = torch.empty(steps, dtype=torch.float64, device=q.device)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        g.rk_iterate(q, 1, norms[k:k + 1], cf)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1000.0, norms


def adjoint_over_primal(torch, hb, synth, name, reps):
    """t(hb_residual_adjoint with state, coordinate and incidence bars) over
    t(hb_residual), both FP64 on the same grid and state, HIP events (median
    of three interleaved trials each)."""
    p = synth.make_problem(name)
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=0, batched=1)
    dev = torch.device("cuda:0")
    q = torch.as_tensor(synth.initial_state(p)).to(dev)
    gen = torch.Generator().manual_seed(1307)
    rbar = torch.randn(q.shape, generator=gen, dtype=torch.float64).to(dev)
    r, qb = torch.empty_like(q), torch.empty_like(q)
    xyb = torch.empty(g.n_xy, dtype=torch.float64, device=dev)
    ab = torch.empty(1, dtype=torch.float64, device=dev)

    def timed(fn):
        fn()
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # three interleaved trials of each, medians
    tps, tas = [], []
    for _ in range(3):
        tps.append(timed(lambda: g.residual(q, r)))
        tas.append(timed(lambda: g.residual_adjoint(q, rbar, qb, xyb, ab)))
    tp, ta = sorted(tps)[1], sorted(tas)[1]
    g.close()
    return {"primal_ms": tp, "adjoint_ms": ta, "ratio": ta / tp,
            "cell_snapshots": p.cell_snapshots}


def cpu_baseline(problem, q_host, target_s=12.0):
    """FP64 oracle (as is) on a bounded sample of the workload's blocks."""
    import torch
    from oracle import hb_oracle as O
    blocks, flow, solver = O.from_synth(problem)
    qs = O.split(blocks, torch.as_tensor(q_host))
    # sample: blocks in order until ~1.2M cell-snapshots, one iteration first
    sel, cs = [], 0
    for k, b in enumerate(blocks):
        sel.append(k)
        cs += b.ns * b.ni * b.nj
        if cs >= 1_200_000:
            break
    sb = [blocks[k] for k in sel]
    sq = O.join([qs[k] for k in sel])
    t0 = time.perf_counter()
    O.rk_iterate(sb, sq, flow, solver, 1)
    dt = time.perf_counter() - t0
    iters = 1
    if dt < target_s / 2:
        extra = max(1, int(target_s / dt) - 1)
        t0 = time.perf_counter()
        O.rk_iterate(sb, sq, flow, solver, extra)
        dt = time.perf_counter() - t0
        iters = extra
    units = cs * len(solver.rk_alpha) * iters
    out = {"value": units / dt, "unit": "cell-snapshot RK-stage updates/s",
           "cores": torch.get_num_threads(), "kind": "oracle",
           "sample": "%d of %d blocks (%d cell-snapshots), %d iteration(s), %.1f s"
                     % (len(sel), len(blocks), cs, iters, dt),
           "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count()}
    # the same oracle on one thread, first sampled block only, iterations
    # repeated for about 2 s
    nt = torch.get_num_threads()
    torch.set_num_threads(1)
    b1 = [blocks[sel[0]]]
    q1 = qs[sel[0]].reshape(-1)
    its, d1 = 0, 0.0
    while d1 < 2.0:
        t0 = time.perf_counter()
        O.rk_iterate(b1, q1, flow, solver, 1)
        d1 += time.perf_counter() - t0
        its += 1
    torch.set_num_threads(nt)
    c1 = b1[0].ns * b1[0].ni * b1[0].nj
    out["single_thread"] = {"value": c1 * len(solver.rk_alpha) * its / d1,
                            "sample": "block %d (%d cell-snapshots), %d iteration(s), %.1f s"
                                      % (sel[0], c1, its, d1)}
    # the method's floating-point operations per unit, counted on the
    # oracle's own evaluation of one iteration of the whole workload
    from oracle import hb_opcount
    out["oracle_ops"] = hb_opcount.ops_per_unit(blocks, torch.as_tensor(q_host), flow, solver)
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch32_mixed")
    ap.add_argument("--plain-steps", type=int, default=5,
                    help="iterations of the fixed-grid FP64 legs (0 skips them)")
    ap.add_argument("--moving-steps", type=int, default=5,
                    help="iterations of the moving-grid leg (0 skips it)")
    ap.add_argument("--moving-only", action="store_true",
                    help="run only the moving-grid leg (for a kernel profile of it; "
                         "needs --tuning)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/primal timing")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuner cache file (JSON); its entry for this device and workload "
                         "is applied, else the autotuner runs and adds one")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even if cached")
    ap.add_argument("--tuning", default=None,
                    help="tile_i,wg_per_cu,xcd_order,tile_order: set instead of autotuning")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only; --gpus %d is not supported "
              "(the block decomposition over several GPUs is not built)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1304_7654_amd import hb, synth

    dev = torch.device("cuda:0")
    problem = synth.make_problem(args.workload)
    q_host = synth.initial_state(problem)
    q0 = torch.as_tensor(q_host).to(dev)
    cs = problem.cell_snapshots
    stages = len(problem.solver.rk_alpha)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.moving_only:
        if not args.tuning:
            sys.exit("bench.py: --moving-only needs --tuning")
        tu = dict(zip(("tile_i", "wg_per_cu", "xcd_order", "tile_order"),
                      (int(x) for x in args.tuning.split(","))))
        print(json.dumps({"moving_grid": moving_leg(torch, hb, problem, q0, args.moving_steps, tu,
                                                    MOTION)}))
        return

    # ---- FP32-bulk batched (the product path) ------------------------------
    g = hb.Grid(problem.blocks, problem.flow, problem.solver, precision=1, batched=1)
    if args.tuning:
        g.set_tuning(*[int(x) for x in args.tuning.split(",")])
        tuning = g.get_tuning()
    else:
        tuning = g.autotune(q0, args.tune_cache, force=args.retune)
    q = q0.clone()
    time_steps(torch, g, q, args.warmup)
    q = q0.clone()
    t, norms = time_steps(torch, g, q, args.steps)
    assert g.status() == hb.HB_OK, "non-finite state in the FP32 run"
    value = cs * stages * args.steps / t
    # live roofline of the fused stage kernel: events around each stage launch
    q = q0.clone()
    g.profile_stages(True)
    time_steps(torch, g, q, args.steps, forces=False)
    st_ms, st_n = g.stage_stats()
    g.profile_stages(False)
    stage_s = st_ms / 1000.0 / st_n
    bytes_launch = algorithmic_bytes_per_iteration(problem) / stages
    achieved = bytes_launch / stage_s / 1e9
    traffic = read_traffic(tuning, args.workload)
    valu = read_profile_value(profile_file(args.workload, "sq_counters"),
                              "valu_wave_instructions_per_launch", tuning, args.workload)
    g.close()
    probe = stream_probe(torch)

    # ---- plain FP64, per-block launches (baseline on the same GPU) ---------
    plain = fused = None
    if args.plain_steps > 0:
        plain = plain_leg(torch, hb, problem, q0, args.plain_steps)
        plain["speedup_of_value"] = value / plain["value"]
        # ---- fused FP64 (same kernel design, FP64 arithmetic) --------------
        gf = hb.Grid(problem.blocks, problem.flow, problem.solver, precision=0, batched=1)
        q = q0.clone()
        time_steps(torch, gf, q, 1)
        q = q0.clone()
        tf, _ = time_steps(torch, gf, q, args.plain_steps)
        fused = {"value": cs * stages * args.plain_steps / tf,
                 "ms_per_step": 1000.0 * tf / args.plain_steps}
        gf.close()
    # ---- the product path on the rigidly heaving and pitching grid --------
    moving = None
    if args.moving_steps > 0:
        moving = moving_leg(torch, hb, problem, q0, args.moving_steps, tuning, MOTION)
        moving["vs_fixed_grid"] = moving["value"] / value

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-snapshot RK-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * t / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 flux/source, f64 state/update/norms/forces",
        "data": "synthetic (seeded O-grid blocks, free stream + 1e-3 Gaussian perturbation)",
        "config": {"workload": args.workload, "blocks": len(problem.blocks),
                   "cell_snapshots": cs, "stages_per_step": stages,
                   "parallelism": "single GPU, one persistent launch per stage",
                   "tuning": tuning},
        "fp64_plain_per_block": plain,
        "fp64_fused_batched": fused,
        "moving_grid": moving,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "k_fused (FP32 bulk stage)", "avg_launch_ms": 1000.0 * stage_s,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     # the 9 metric words per cell the kernel reads (5 by the method)
                     "design_bytes_per_launch": design_bytes_per_iteration(problem) / stages,
                     # measured HBM traffic (counters) over the live launch time, against
                     # the 8 TB/s peak and against a 1 GiB device copy measured here
                     "traffic_gbs": None if traffic is None else traffic / stage_s / 1e9,
                     "traffic_frac": None if traffic is None else traffic / stage_s / 1e9 / PEAK_HBM_GBS,
                     "stream_probe_gbs": probe,
                     "frac_of_stream_probe": achieved / probe,
                     "traffic_frac_of_stream_probe": None if traffic is None else traffic / stage_s / 1e9 / probe},
        # VALU issue (64 lanes per wave-instruction, from the committed shader
        # counters) over the same live launch time: a utilisation figure
        "valu_issue": None if valu is None else {
            "achieved": 64.0 * valu / stage_s, "peak": PEAK_VALU_LANE_INSTR,
            "unit": "VALU lane-instructions/s", "frac": 64.0 * valu / stage_s / PEAK_VALU_LANE_INSTR,
            "valu_wave_instructions_per_launch": valu},
        "adjoint_over_primal": None if args.no_adjoint else {
            name: adjoint_over_primal(torch, hb, synth, name, reps)
            for name, reps in (("naca256x128_hh64", 50), ("naca1024x512_nh4", 10))},
        "resnorm_last": float(norms[-1].item()),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(problem, q_host)
        # ALU roofline of the same kernel: the method's operations per unit
        # (counted on the oracle) times the units of one launch, over the
        # live launch time, against the FP32 vector peak
        opu = out["cpu_baseline"]["oracle_ops"]["per_unit"]
        flops = opu * cs / stage_s
        out["roofline_alu"] = {"bound": "alu", "achieved": flops / 1e12, "peak": PEAK_FP32_TFLOPS,
                               "unit": "TFLOP/s", "frac": flops / 1e12 / PEAK_FP32_TFLOPS,
                               "ops_per_unit": opu,
                               "frac_of_unpacked_fp32": flops / 1e12 / (PEAK_FP32_TFLOPS / 2)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
