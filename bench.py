"""Benchmark of the GRMHD hot path on one MI355X.

One step = one SSPRK3 step (3 RK stages: con2prim, fused reconstruction +
HLLE + divergence + sources + stage update) over the whole grid of the
workload, inputs resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload curved256|flat64|curved384-mixed|batched400]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 64 FP64 lanes x 2 (FMA = 2 flops)

# Arithmetic of one stage-kernel launch per interior cell (3 faces + the cell's
# metric, sources, divergence and stage combine; +, -, *, /, sqrt = 1 flop each),
# counted by running the method's routines on an op-counting scalar.  The
# con2prim Newton iterations the stage kernel also runs are data-dependent and
# not counted, so the ALU fraction is a lower bound.
FLOPS_PER_CELL = {0: 2364, 1: 5292, 2: 5484}   # minmod, WENO5, WENO5-Z

# The headline metric: the plain-FP64 zone rate of the workload (value) and, in the
# same line, the adjoint/forward time ratio of the 128^3 WENO5-Z adjoint workload.
METRIC = "GRMHD zone-updates/s per RK stage vs FP64 plain; adjoint/forward time ratio"

WORKLOADS = {
    # name: (builder kwargs, description)
    "curved256": dict(kind="config1", n=256, desc="static curved metric 256^3, WENO5, HLLE, FP64, SSPRK3"),
    "flat64": dict(kind="config0", n=64, desc="flat 64^3 with jump, minmod, HLLE, FP64, SSPRK3"),
    "curved384-mixed": dict(kind="config3", n=384, desc="static curved metric 384^3, WENO5, FP32 recon+HLLE"),
    "curved256-mixed": dict(kind="config3", n=256, desc="static curved metric 256^3, WENO5, FP32 recon+HLLE"),
    "curved384-fp64": dict(kind="config3-fp64", n=384,
                           desc="static curved metric 384^3 (mixed-precision recipe and seed), WENO5, HLLE, FP64"),
    "batched400": dict(kind="config2", n=0, desc="400 uneven boxes (edges 16..64, flat/curved), WENO5, FP64"),
    # stand-ins for the paper's setupA (static spacetime, ideal gas, RK2), its own
    # single-GPU comparison point: the curved recipe with periodic faces, SSPRK2
    "setupA152": dict(kind="setupA", n=152, scheme=1, paper_v100=0.44e8,
                      desc="setupA stand-in: static curved metric 152^3, Gamma-law, WENO5, HLLE, RK2 (SSPRK2), "
                           "periodic, FP64"),
    # classic RK4 (stages fused like the SSPRK ones: L, accumulation, next stage state, con2prim)
    "curved256-rk4": dict(kind="config1", n=256, scheme=2,
                          desc="static curved metric 256^3, WENO5, HLLE, FP64, classic RK4"),
    "setupA240": dict(kind="setupA", n=240, scheme=1, paper_v100=0.47e8,
                      desc="setupA stand-in: static curved metric 240^3, Gamma-law, WENO5, HLLE, RK2 (SSPRK2), "
                           "periodic, FP64"),
}


def make_problem(w):
    from paper_2210_17509_amd import inputs as I
    spec = WORKLOADS[w]
    if spec["kind"] == "config1":
        return I.config1(n=spec["n"])
    if spec["kind"] == "config0":
        return I.config0(n=spec["n"])
    if spec["kind"] == "config3":
        return I.config3(n=spec["n"], steps=1)
    if spec["kind"] == "config3-fp64":
        return I.config3(n=spec["n"], steps=1, precision=I.PREC_FP64)
    if spec["kind"] == "config2":
        return I.config2()
    if spec["kind"] == "setupA":
        return I.config1(n=spec["n"], bc=I.BC_PERIODIC)
    raise ValueError(w)


def stage_bytes_per_cell(nstage=3):
    """Algorithmic HBM bytes of one stage-kernel launch per interior cell, averaged over
    the stages of a step (3 for SSPRK3, 2 for SSPRK2): P read 64, U_s read 64, U^n read
    64 (all stages but the first), vertex metric alpha + 6 gamma_ij ~ 1 vertex per cell
    56, U_{s+1} write 64, and the primitives of U_{s+1} (con2prim runs inside the stage
    kernel) write 64."""
    return 64 + 64 + 64 * (nstage - 1.0) / nstage + 56 + 64 + 64


def cpu_baseline(w, budget_s=12.0):
    """The FP64 oracle on the host cores on a bounded sample of the same workload recipe:
    one SSPRK3 step of the same recipe on a smaller cube sized to ~budget_s of wall time."""
    import numpy as np
    import oracle
    from paper_2210_17509_amd import inputs as I
    oracle.build(force=False)
    threads = min(16, os.cpu_count() or 1)
    oracle.set_threads(threads)
    kind = WORKLOADS[w]["kind"]
    kind = "config1" if kind == "setupA" else kind
    # probe the rate on a small cube, then size the sample
    def run(n):
        p = I.config1(n=n) if kind in ("config1", "config3", "config3-fp64", "config2") else I.config0(n=n)
        U, P = oracle.prim2con(p), p.P.copy()
        t = time.perf_counter()
        oracle.rk_step(p, U, P)
        return time.perf_counter() - t, n ** 3 * 3
    t, z = run(24)
    rate = z / t
    n = int(round((rate * budget_s / 3.0) ** (1.0 / 3.0)))
    n = max(24, min(n, 192))
    t, z = run(n)
    return {"value": z / t, "unit": "zone-updates/s per RK stage", "cores": threads, "kind": "oracle",
            "sample": f"one SSPRK3 step of the same recipe on {n}^3 cells ({t:.1f} s wall, {threads} threads)"}


def kernel_sources():
    """Every source the HIP library is built from (csrc/*.hip, csrc/*.h, the C header)."""
    import glob
    csrc = sorted(glob.glob(os.path.join(ROOT, "paper_2210_17509_amd", "csrc", "*.hip")) +
                  glob.glob(os.path.join(ROOT, "paper_2210_17509_amd", "csrc", "*.h")))
    return [os.path.relpath(f, ROOT) for f in csrc] + ["include/grmhd.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in kernel_sources():
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def hbm_summary_path(workload):
    return os.path.join(ROOT, "profiles", f"k_stage_{workload}_hbm.txt")


def committed_traffic(workload):
    """HBM bytes per stage-kernel launch from the committed counter summary of this
    workload, or None if there is none or the kernel sources changed since it was taken."""
    path = hbm_summary_path(workload)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return float(kv["traffic_bytes_per_launch"])


def _counter_rows(d, counter, name_part):
    import csv
    import glob
    vals = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]:
                    vals.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not vals:
        raise SystemExit(f"no {counter} rows for '{name_part}' under {d}")
    return vals


def hbm_summary(args):
    """Write the HBM-traffic summary of the stage kernel from four rocprofv3 --pmc runs
    (FETCH_SIZE and WRITE_SIZE of the workload, the same two of the 1 GiB copy)."""
    fdir, wdir, cfdir, cwdir = args.hbm_summary
    fetch = _counter_rows(fdir, "FETCH_SIZE", "k_stage")
    write = _counter_rows(wdir, "WRITE_SIZE", "k_stage")
    cf = [v for _, v in _counter_rows(cfdir, "FETCH_SIZE", "copyBuffer")]
    cw = [v for _, v in _counter_rows(cwdir, "WRITE_SIZE", "copyBuffer")]
    copy_kib = (1 << 30) / 1024.0
    ff, fw = copy_kib / (sum(cf) / len(cf)), copy_kib / (sum(cw) / len(cw))
    fk = sum(v for _, v in fetch) / len(fetch)
    wk = sum(v for _, v in write) / len(write)
    from paper_2210_17509_amd import inputs as I
    spec = WORKLOADS[args.workload]
    ncell = (spec["n"] ** 3) if spec["n"] else None
    traffic = (fk * ff + wk * fw) * 1024.0
    alg = stage_bytes_per_cell() * ncell if ncell else None
    lines = [
        f"# HBM traffic of the stage kernel, workload: {spec['desc']}",
        "# FETCH_SIZE / WRITE_SIZE are KiB per dispatch; each is scaled by what the same counter",
        "# reads for a plain 1 GiB device copy (bench.py --calibrate-copy).",
        "# Commands (repository root, one MI355X):",
        f"#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d F -o bench -- python bench.py --workload {args.workload} --steps 1 --warmup 0 --no-cpu-baseline --no-adjoint --no-extras",
        f"#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d W -o bench -- python bench.py --workload {args.workload} --steps 1 --warmup 0 --no-cpu-baseline --no-adjoint --no-extras",
        "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d CF -o copy -- python bench.py --calibrate-copy",
        "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d CW -o copy -- python bench.py --calibrate-copy",
        f"#   python bench.py --workload {args.workload} --hbm-summary F W CF CW",
        f"kernel_source_sha256: {kernel_source_hash()}",
        f"kernel: {fetch[0][0]}",
        f"dispatches: {len(fetch)} (FETCH) {len(write)} (WRITE)",
        f"fetch_kib_per_dispatch: {fk:.1f}",
        f"write_kib_per_dispatch: {wk:.1f}",
        f"copy_fetch_factor: {ff:.4f}",
        f"copy_write_factor: {fw:.4f}",
        f"traffic_bytes_per_launch: {traffic:.6e}",
    ]
    if alg:
        lines += [f"algorithmic_bytes_per_launch: {alg:.6e} ({stage_bytes_per_cell():.1f} B x {ncell} cells)",
                  f"traffic_over_algorithmic: {traffic / alg:.3f}"]
    os.makedirs(os.path.dirname(hbm_summary_path(args.workload)), exist_ok=True)
    with open(hbm_summary_path(args.workload), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


SQ_PASSES = (
    "SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVE_CYCLES SQ_WAIT_INST_ANY SQ_BUSY_CYCLES SQ_WAIT_ANY "
    "SQ_ACTIVE_INST_ANY",
    "SQ_INSTS_VMEM_RD SQ_INST_LEVEL_VMEM SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_INSTS_SALU SQ_INSTS_VALU_CVT "
    "SQ_INSTS_VALU_TRANS_F32 SQ_INSTS_VALU_TRANS_F64",
    # optional third pass: the FP64 instruction mix
    "SQ_WAVES SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64",
)


def _stats_avg_ms(name_part):
    """Mean duration of a kernel in the committed kernel-statistics summary, or None."""
    path = os.path.join(ROOT, "profiles", "kernels_curved256_stats.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if len(f) > 5 and name_part in line and f[0].isdigit():
                return float(f[1])
    return None


def sq_summary(args):
    """Write profiles/k_stage_<workload>_sq.txt from the two rocprofv3 --pmc runs of SQ_PASSES."""
    dirs = args.sq_summary
    if len(dirs) not in (2, 3):
        raise SystemExit("--sq-summary takes the two (or three) SQ pass folders")
    means, kernel, ndisp = {}, None, None
    for d, names in zip(dirs, SQ_PASSES):
        for c in names.split():
            rows = _counter_rows(d, c, "k_stage")
            kernel = kernel or rows[0][0]
            ndisp = len(rows)
            means[c] = sum(v for _, v in rows) / len(rows)
    waves = means["SQ_WAVES"]
    run = (f"--output-format csv -d {{}} -o bench -- python bench.py --workload {args.workload} --steps 1 "
           "--warmup 0 --no-cpu-baseline --no-adjoint --no-extras")
    lines = [f"# SQ counters of the stage kernel (con2prim included), workload: {WORKLOADS[args.workload]['desc']}",
             f"# (mean over the {ndisp} stage dispatches of one step; *_CYCLES and ACTIVE/WAIT counters in "
             "quad-cycles, summed over SEs)",
             "# Commands (repository root, one MI355X):",
             f"#   rocprofv3 --pmc {SQ_PASSES[0]} " + run.format("S1"),
             f"#   rocprofv3 --pmc {SQ_PASSES[1]} " + run.format("S2")]
    if len(dirs) == 3:
        lines.append(f"#   rocprofv3 --pmc {SQ_PASSES[2]} " + run.format("S3"))
    lines += [f"#   python bench.py --workload {args.workload} --sq-summary S1 S2" + (" S3" if len(dirs) == 3 else ""),
             f"kernel_source_sha256: {kernel_source_hash()}",
             f"kernel: {kernel}"]
    for c in sorted(means):
        lines.append(f"{c}: {means[c]:.4e}  ({means[c] / waves:.1f} per wave)")
    if "SQ_INSTS_VALU_FMA_F64" in means:
        # each FP64 VALU instruction of a wave covers 64 lanes (inactive ones included)
        lane_flops = 64.0 * (means["SQ_INSTS_VALU_ADD_F64"] + means["SQ_INSTS_VALU_MUL_F64"] +
                             means["SQ_INSTS_VALU_TRANS_F64"] + 2.0 * means["SQ_INSTS_VALU_FMA_F64"])
        ncell = WORKLOADS[args.workload]["n"] ** 3
        alg = FLOPS_PER_CELL[1] * ncell
        lines.append(f"issued FP64 lane-flops per launch (64 x (ADD + MUL + TRANS + 2 FMA)): {lane_flops:.4e}"
                     f" = {lane_flops / alg:.2f} x the counted right-hand side ({alg:.4e}; con2prim and"
                     " masked lanes account for the rest)")
        ms = _stats_avg_ms("k_stage<1, double, false, 3, false>")
        if ms:
            lines.append(f"issued FP64 rate at the kernel-trace mean {ms:.4f} ms: {lane_flops / ms / 1e9:.1f} TFLOP/s"
                         f" = {lane_flops / ms / 1e9 / FP64_VECTOR_PEAK_TFLOPS:.3f} of the FP64 vector peak")
    lines.append("waiting share of wave cycles (SQ_WAIT_ANY / SQ_WAVE_CYCLES): "
                 f"{means['SQ_WAIT_ANY'] / means['SQ_WAVE_CYCLES']:.3f}")
    path = os.path.join(ROOT, "profiles", f"k_stage_{args.workload}_sq.txt")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def stats_summary(args):
    """Write profiles/kernels_<workload>_stats.txt from a rocprofv3 --kernel-trace --stats folder."""
    import csv
    import glob
    d, cmd = args.stats_summary
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_stats.csv under {d}")
    with open(files[0]) as fh:
        rows = list(csv.DictReader(fh))
    if args.adjoint:
        name, desc = "adjoint128", ("adjoint, flat 128^3 smooth, WENO5-Z, 10 SSPRK3 steps with stage checkpoints, "
                                    "then 10 adjoint steps (FP64)")
    else:
        name, desc = args.workload, WORKLOADS[args.workload]["desc"]
    lines = [f"# rocprofv3 kernel statistics, workload: {desc}",
             "# Command (repository root, one MI355X):",
             f"#   {cmd}",
             f"kernel_source_sha256: {kernel_source_hash()}",
             f"{'calls':>6} {'avg_ms':>10} {'min_ms':>10} {'max_ms':>10} {'share%':>7}  kernel"]
    for r in rows[:12]:
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e6:10.4f} {float(r['MinNs']) / 1e6:10.4f} "
                     f"{float(r['MaxNs']) / 1e6:10.4f} {float(r['Percentage']):7.2f}  {r['Name'][:150]}")
    path = os.path.join(ROOT, "profiles", f"kernels_{name}_stats.txt")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def calibrate_copy(nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size: what FETCH_SIZE / WRITE_SIZE read for
    exactly nbytes read and nbytes written per launch."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": reps,
                      "GBs_read_plus_write": 2 * nbytes / dt / 1e9}), flush=True)


def adjoint_bench(args):
    """Forward (10 SSPRK3 steps writing stage checkpoints) and reverse pass (10 adjoint
    steps) of the 128^3 WENO5-Z workload; reports the time ratio."""
    import torch
    from paper_2210_17509_amd import grmhd as G
    from paper_2210_17509_amd import inputs as I
    prob = I.config4()
    dom = G.Domain.from_problem(prob)
    met = G.Metric.from_problem(prob)
    # steps start from the primitives the previous step left (P0 for the first:
    # the primitives U0 is built from)
    par = G.make_params(prob.params, tile=args.tile, p_current=1)
    P0 = torch.as_tensor(prob.P, device="cuda").contiguous()
    U0 = torch.zeros_like(P0)
    G.grmhd_prim2con(dom, par, met, P0, U0)
    steps = prob.steps
    ck = torch.empty((steps, 3) + tuple(U0.shape), dtype=torch.float64, device="cuda")
    ws = torch.empty(G.grmhd_workspace_bytes(dom, par) // 8, dtype=torch.float64, device="cuda")
    wsa = torch.empty(G.grmhd_workspace_bytes(dom, par, 0, 1) // 8, dtype=torch.float64, device="cuda")
    g_out = torch.randn(U0.shape, dtype=torch.float64, device="cuda")
    g_in = torch.zeros_like(g_out)

    def fwd():
        U, P = U0.clone(), P0.clone()
        for k in range(steps):
            G.grmhd_rk_step(dom, par, met, U, P, prob.dt, 0, ck[k], ws=ws)
        return P

    def bwd(P):
        a, b = g_out.clone(), g_in
        for k in reversed(range(steps)):
            G.grmhd_rk_step_adjoint(dom, par, met, ck[k], P, prob.dt, a, b, 0, ws=wsa)
            a, b = b, a

    P = fwd()
    bwd(P)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 10)
    t0 = time.perf_counter()
    for _ in range(reps):
        P = fwd()
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        bwd(P)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    ncell = prob.ninterior
    return {"metric": "adjoint/forward time ratio", "value": tb / tf, "unit": "ratio",
            "higher_is_better": False, "forward_ms": tf * 1e3, "backward_ms": tb * 1e3,
            "forward_zone_updates_per_s": ncell * 3 * steps / tf,
            "config": {"workload": "flat 128^3 smooth, WENO5-Z, 10 SSPRK3 steps with stage checkpoints, FP64",
                       "cells": ncell}}


def run_workload(name, args, steps=None, warmup=None):
    """Warm up, then time `steps` SSPRK3 steps of workload `name` (HIP events on every
    stage and con2prim launch, wall clock around the whole timed region)."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    import torch
    from paper_2210_17509_amd import grmhd as G
    prob = make_problem(name)
    dom = G.Domain.from_problem(prob)
    met = G.Metric.from_problem(prob)
    # A run of steps recovers the primitives once per RK stage (inside the stage
    # kernel); each step starts from the primitives the previous one left, the
    # first from those U was built from.
    par = G.make_params(prob.params, tile=args.tile, schedule=args.schedule, p_current=1)
    P = torch.as_tensor(prob.P, device="cuda").contiguous()
    U = torch.zeros_like(P)
    nfail = torch.zeros(1, dtype=torch.int64, device="cuda")
    rate = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.grmhd_prim2con(dom, par, met, P, U)
    if args.autotune:
        from paper_2210_17509_amd.autotune import autotune
        par, _ = autotune(dom, par, met, U, P, prob.dt, reps=2)
    scheme = WORKLOADS[name].get("scheme", G.GRMHD_SSPRK3)
    ws = torch.empty(G.grmhd_workspace_bytes(dom, par, scheme) // 8, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        G.grmhd_rk_step(dom, par, met, U, P, prob.dt, scheme, max_rate=rate, n_fail=nfail, ws=ws)
    torch.cuda.synchronize()
    G.grmhd_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        G.grmhd_rk_step(dom, par, met, U, P, prob.dt, scheme, max_rate=rate, n_fail=nfail, ws=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = G.grmhd_timing_read()
    G.grmhd_timing_enable(False)
    return {"prob": prob, "ncell": prob.ninterior, "wall": wall, "times": times, "nfail": int(nfail.item()),
            "par": par, "U": U, "P": P, "stages": {G.GRMHD_SSPRK3: 3, G.GRMHD_SSPRK2: 2, G.GRMHD_RK4: 4}[scheme]}


def batched_bench(args, single_value):
    """The 400-box batch stepped as a captured graph of one SSPRK3 step (tile shape and
    schedule autotuned), timed over `steps` replays; its zone rate against the single
    256^3 box of the headline."""
    import torch
    from paper_2210_17509_amd import grmhd as G
    from paper_2210_17509_amd.autotune import StepGraph, autotune
    prob = make_problem("batched400")
    dom = G.Domain.from_problem(prob)
    met = G.Metric.from_problem(prob)
    par = G.make_params(prob.params, p_current=1)
    P = torch.as_tensor(prob.P, device="cuda").contiguous()
    U = torch.zeros_like(P)
    nfail = torch.zeros(1, dtype=torch.int64, device="cuda")
    rate = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.grmhd_prim2con(dom, par, met, P, U)
    par, _ = autotune(dom, par, met, U, P, prob.dt, reps=2)
    graph = StepGraph(dom, par, met, U, P, prob.dt, max_rate=rate, n_fail=nfail)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = prob.ninterior * 3 * args.steps / wall
    return {"workload": WORKLOADS["batched400"]["desc"] + ", one captured graph per step", "value": value,
            "unit": "zone-updates/s per RK stage", "ratio_to_single_box": value / single_value,
            "cells": prob.ninterior, "boxes": len(prob.boxes), "tile": par.tile, "schedule": par.schedule,
            "ms_per_step": wall * 1e3 / args.steps, "n_fail": int(nfail.item())}


def mixed_bench(args, steps=50):
    """The mixed-precision workload (384^3, FP32 reconstruction + HLLE) and the same
    recipe in FP64, `steps` SSPRK3 steps each from the same initial data: both zone
    rates, their ratio, and the per-field error of the mixed run against the FP64 run."""
    fp = run_workload("curved384-fp64", args, steps=steps, warmup=0)
    mx = run_workload("curved384-mixed", args, steps=steps, warmup=0)
    vf = fp["ncell"] * 3 * steps / fp["wall"]
    vm = mx["ncell"] * 3 * steps / mx["wall"]
    out = {"workload": WORKLOADS["curved384-mixed"]["desc"] + f", {steps} SSPRK3 steps", "value": vm,
           "fp64_value": vf, "ratio_mixed_over_fp64": vm / vf, "unit": "zone-updates/s per RK stage",
           "n_fail": [fp["nfail"], mx["nfail"]],
           "stage_ms_avg": {"fp64": fp["times"]["stage"][0] / max(fp["times"]["stage"][1], 1),
                            "mixed": mx["times"]["stage"][0] / max(mx["times"]["stage"][1], 1)},
           "U_error_vs_fp64": field_errors(mx["prob"], mx["U"], fp["U"]),
           "P_error_vs_fp64": field_errors(mx["prob"], mx["P"], fp["P"])}
    del fp, mx
    return out


def setupA_bench(args, name="setupA240", steps=10):
    """The stand-in for the paper's setupA (its own single-GPU comparison: static
    spacetime, ideal gas, RK2): the curved recipe with periodic faces at 240^3,
    SSPRK2, in the paper's unit of zone-cycles/s (full steps of every cell)."""
    r = run_workload(name, args, steps=steps, warmup=2)
    spec = WORKLOADS[name]
    out = {"workload": spec["desc"], "zone_cycles_per_s": r["ncell"] * steps / r["wall"],
           "zone_updates_per_s_per_stage": r["ncell"] * r["stages"] * steps / r["wall"], "steps": steps,
           "n_fail": r["nfail"],
           "paper_context": {"zone_cycles_per_s": spec["paper_v100"],
                             "machine": "one Summit V100 (the paper's setupA, another machine: context only)"}}
    del r
    return out


def field_errors(prob, a, b):
    """Per-field relative L-inf and L2 of a against b over interior cells (both (8, cells))."""
    import numpy as np
    from paper_2210_17509_amd import inputs as I
    import torch
    mask = torch.as_tensor(np.concatenate([I.interior_mask(bx).ravel() for bx in prob.boxes]), device=a.device)
    d = (a - b)[:, mask]
    r = b[:, mask]
    linf = (d.abs().amax(dim=1) / r.abs().amax(dim=1).clamp_min(1e-300)).tolist()
    l2 = (d.norm(dim=1) / r.norm(dim=1).clamp_min(1e-300)).tolist()
    return {"rel_linf": linf, "rel_l2": l2}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="curved256", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--autotune", action="store_true", help="pick tile shape and schedule by timing")
    ap.add_argument("--compare", default=None, help="also time this workload and report the rate ratio")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint", action="store_true",
                    help="adjoint workload: 128^3 WENO5-Z, 10 steps with checkpoints, then the reverse pass")
    ap.add_argument("--no-adjoint", action="store_true", help="leave the adjoint/forward ratio out of the line")
    ap.add_argument("--no-extras", action="store_true",
                    help="leave the batched (400 boxes, graph) and mixed-precision (384^3, 50 steps) figures out")
    ap.add_argument("--hbm-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write profiles/k_stage_<workload>_hbm.txt from rocprofv3 --pmc output folders")
    ap.add_argument("--stats-summary", nargs=2, metavar=("STATS_DIR", "COMMAND"),
                    help="write profiles/kernels_<workload>_stats.txt (with --adjoint: kernels_adjoint128_stats.txt) "
                         "from a rocprofv3 --stats folder")
    ap.add_argument("--sq-summary", nargs="+", metavar="SQ_PASS_DIR",
                    help="write profiles/k_stage_<workload>_sq.txt from the two (or three, with the FP64 "
                         "instruction mix) rocprofv3 --pmc SQ passes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.hbm_summary:
        return hbm_summary(args)
    if args.stats_summary:
        return stats_summary(args)
    if args.sq_summary:
        return sq_summary(args)
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2210_17509_amd import grmhd as G

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        return calibrate_copy()
    if args.adjoint:
        print(json.dumps(adjoint_bench(args)), flush=True)
        return
    res = run_workload(args.workload, args)
    prob, ncell, wall, times, nfail, par = res["prob"], res["ncell"], res["wall"], res["times"], res["nfail"], \
        res["par"]

    stages = res["stages"]
    value = ncell * stages * args.steps / wall
    st_ms, st_n = times["stage"]
    c2p_ms, c2p_n = times["con2prim"]
    avg_stage_s = st_ms / 1e3 / max(st_n, 1)
    flops_per_launch = FLOPS_PER_CELL[prob.params.recon] * ncell
    achieved = flops_per_launch / avg_stage_s / 1e12
    hbm_gbs = stage_bytes_per_cell(stages) * ncell / avg_stage_s / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "zone-updates/s per RK stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prob.params.precision == 0 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload]["desc"], "cells": ncell, "boxes": len(prob.boxes),
                   "stages_per_step": stages, "n_fail": nfail, "tile": par.tile, "schedule": par.schedule,
                   "con2prim": "once per RK stage, fused into the stage kernel"},
        "kernels": {"stage_ms_avg": st_ms / max(st_n, 1), "stage_launches": st_n,
                    "con2prim_ms_avg": c2p_ms / max(c2p_n, 1), "con2prim_launches": c2p_n},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": committed_traffic(args.workload),
                     "kernel": "k_stage", "flops_per_cell": FLOPS_PER_CELL[prob.params.recon],
                     "algorithmic_hbm_GBs": hbm_gbs, "algorithmic_hbm_frac": hbm_gbs / HBM_PEAK_GBS},
    }
    spec = WORKLOADS[args.workload]
    if "paper_v100" in spec:
        # the paper's own single-GPU unit: full steps (all RK stages) of every cell per second
        out["zone_cycles_per_s"] = ncell * args.steps / wall
        out["paper_context"] = {"zone_cycles_per_s": spec["paper_v100"],
                                "machine": "one Summit V100 (the paper's setupA, another machine: context only)"}
    if args.compare:
        ref = run_workload(args.compare, args)
        ref_value = ref["ncell"] * ref["stages"] * args.steps / ref["wall"]
        out["compare"] = {"workload": WORKLOADS[args.compare]["desc"], "value": ref_value,
                          "ratio": value / ref_value}
        if ref["U"].shape == res["U"].shape and ref["prob"].P.shape == prob.P.shape:
            # same grid and the same number of steps from the same initial data
            out["compare"]["U_error_vs_compare"] = field_errors(prob, res["U"], ref["U"])
            out["compare"]["P_error_vs_compare"] = field_errors(prob, res["P"], ref["P"])
        del ref
    del res
    if not args.no_extras and args.workload == "curved256":
        out["batched"] = batched_bench(args, value)
        out["mixed_precision"] = mixed_bench(args)
        out["setupA_standin"] = setupA_bench(args)
    if not args.no_adjoint:
        a = adjoint_bench(args)
        out["adjoint_forward_ratio"] = a["value"]
        out["adjoint"] = {k: a[k] for k in ("forward_ms", "backward_ms", "config")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
