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
# counted by running the method's routines on an op-counting scalar.
FLOPS_PER_CELL = {0: 2364, 1: 5292, 2: 5484}   # minmod, WENO5, WENO5-Z

WORKLOADS = {
    # name: (builder kwargs, description)
    "curved256": dict(kind="config1", n=256, desc="static curved metric 256^3, WENO5, HLLE, FP64, SSPRK3"),
    "flat64": dict(kind="config0", n=64, desc="flat 64^3 with jump, minmod, HLLE, FP64, SSPRK3"),
    "curved384-mixed": dict(kind="config3", n=384, desc="static curved metric 384^3, WENO5, FP32 recon+HLLE"),
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
    raise ValueError(w)


def stage_bytes_per_cell():
    """Algorithmic HBM bytes of one stage-kernel launch per interior cell, averaged over
    the 3 SSPRK3 stages: P read 64, U_s read 64, U^n read 64 (stages 2, 3 only), vertex
    metric alpha + 6 gamma_ij ~ 1 vertex per cell 56, U_{s+1} write 64."""
    return 64 + 64 + 64 * 2.0 / 3.0 + 56 + 64


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
    # probe the rate on a small cube, then size the sample
    def run(n):
        p = I.config1(n=n) if kind in ("config1", "config3") else I.config0(n=n)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="curved256", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2210_17509_amd import grmhd as G

    torch.cuda.set_device(0)
    prob = make_problem(args.workload)
    dom = G.Domain.from_problem(prob)
    met = G.Metric.from_problem(prob)
    par = G.make_params(prob.params, tile=args.tile)
    P = torch.as_tensor(prob.P, device="cuda").contiguous()
    U = torch.zeros_like(P)
    nfail = torch.zeros(1, dtype=torch.int64, device="cuda")
    rate = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(G.grmhd_workspace_bytes(dom, par) // 8, dtype=torch.float64, device="cuda")
    G.grmhd_prim2con(dom, par, met, P, U)
    ncell = prob.ninterior

    for _ in range(args.warmup):
        G.grmhd_rk_step(dom, par, met, U, P, prob.dt, max_rate=rate, n_fail=nfail, ws=ws)
    torch.cuda.synchronize()

    G.grmhd_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G.grmhd_rk_step(dom, par, met, U, P, prob.dt, max_rate=rate, n_fail=nfail, ws=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = G.grmhd_timing_read()
    G.grmhd_timing_enable(False)

    stages = 3
    value = ncell * stages * args.steps / wall
    st_ms, st_n = times["stage"]
    c2p_ms, c2p_n = times["con2prim"]
    avg_stage_s = st_ms / 1e3 / max(st_n, 1)
    flops_per_launch = FLOPS_PER_CELL[prob.params.recon] * ncell
    achieved = flops_per_launch / avg_stage_s / 1e12
    hbm_gbs = stage_bytes_per_cell() * ncell / avg_stage_s / 1e9
    out = {
        "metric": "GRMHD zone-updates/s per RK stage",
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
        "config": {"workload": WORKLOADS[args.workload]["desc"], "cells": ncell, "stages_per_step": stages,
                   "n_fail": int(nfail.item())},
        "kernels": {"stage_ms_avg": st_ms / max(st_n, 1), "stage_launches": st_n,
                    "con2prim_ms_avg": c2p_ms / max(c2p_n, 1), "con2prim_launches": c2p_n},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_stage", "flops_per_cell": FLOPS_PER_CELL[prob.params.recon],
                     "algorithmic_hbm_GBs": hbm_gbs, "algorithmic_hbm_frac": hbm_gbs / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
