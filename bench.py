#!/usr/bin/env python3
"""Benchmark of the incompressible-DUGKS step on one MI355X.

Workload (default): D3Q19 cubic lid-driven cavity, 128^3 cells, lid U = 0.1
along x, NEQ velocity walls on all six sides, rho0 = 1, RT = 1/3, dx = 1,
Re = 100 (tau = U N / (Re RT)), CFL 0.5, FP64, started from rest.  One
"step" is one full time step (Appendix steps 1-9) over every cell and every
discrete velocity.  Prints one JSON line:

  value      MLUPS = cells * steps / seconds / 1e6 (inputs resident in HBM)
  roofline   dominant kernel's algorithmic HBM bytes (read f~ once, write f~
             once: 2 Q s bytes per cell) / its average launch time, against
             the 8 TB/s HBM peak; `traffic` = HBM bytes per launch measured
             with rocprofv3 counters (profiles/), null when stale
  cpu_baseline  the FP64 CPU oracle timed on this host on a bounded sample
             of the same workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f64|f32]
       [--mesh uniform|tanh] [--re 100] [--n 128] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DUGKS MLUPS + %HBM roofline (D3Q19 128^3); batched & adjoint vs plain, same err"


def cavity_cfg(n, dtype, mesh, re, lattice=19):
    import paper_1411_6121_amd as M

    U, RT = 0.1, 1.0 / 3.0
    nu = U * n / re
    uw = [[0.0] * 3 for _ in range(6)]
    uw[3] = [U, 0.0, 0.0]                       # lid: +y wall moving along +x
    tanh = 1 if mesh == "tanh" else 0
    d = dict(lattice=lattice, dtype=dtype, n=(n, n, n if lattice == 19 else 1),
             L=(float(n), float(n), float(n) if lattice == 19 else 1.0),
             mesh=(tanh, tanh, tanh if lattice == 19 else 0), k_stretch=1.5, rho0=1.0, RT=RT, tau=nu / RT,
             dt=1.0, bc=(1, 1, 1, 1, 1, 1) if lattice == 19 else (1, 1, 1, 1, 0, 0), uw=uw)
    d["dt"] = M.dugks_dt_from_cfl(d, 0.5)
    return d


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1411_6121_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as fh:
            h.update(fn.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p)).get(workload)
    except Exception:
        return None
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(cfg, budget_s=20.0, max_steps=8):
    """The oracle as it stands, on the full workload, for a bounded number of
    steps (stops after the step that crosses budget_s)."""
    import numpy as np

    import oracle as O

    ocfg = {k: v for k, v in cfg.items() if k != "dtype"}
    f = O.init(ocfg)
    cells = int(np.prod(cfg["n"]))
    steps, t0 = 0, time.perf_counter()
    while steps < max_steps:
        f = O.step(ocfg, f, None, steps * cfg["dt"])
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": round(cells * steps / el / 1e6, 4), "unit": "MLUPS", "cores": O.threads(), "kind": "oracle",
            "sample": f"{steps} FP64 steps of the same {'x'.join(str(v) for v in cfg['n'])} cavity from rest "
                      f"({el:.1f} s wall, OpenMP over cells)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--mesh", default="uniform", choices=["uniform", "tanh"])
    ap.add_argument("--re", type=float, default=100.0)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the step is measured on one MI355X); "
              "multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1411_6121_amd as M

    torch.cuda.init()
    cfg = cavity_cfg(args.n, args.dtype, args.mesh, args.re)
    Q, D, shp = M.shape_of(cfg)
    cells = int(shp[0] * shp[1] * shp[2])
    esize = 8 if args.dtype == "f64" else 4
    f = torch.empty((Q,) + shp, dtype=M.torch_dtype(cfg), device="cuda")
    g = torch.empty_like(f)
    ctx = M.dugks_init(cfg, f)
    cur, nxt = f, g
    for k in range(args.warmup):
        M.dugks_step(ctx, cur, nxt, None, k * cfg["dt"])
        cur, nxt = nxt, cur
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        M.dugks_step(ctx, cur, nxt, None, (args.warmup + k) * cfg["dt"])
        cur, nxt = nxt, cur
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1) / args.steps

    # state must stay finite (the step ran for real)
    tot = M.dugks_moments(ctx, cur)
    variant = M.dugks_kernel_variant(ctx)
    M.dugks_destroy(ctx)

    if args.copy_probe:
        buf = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")  # 256 MiB
        out = torch.empty_like(buf)
        for _ in range(3):
            out.copy_(buf)
        torch.cuda.synchronize()

    workload = f"D3Q19 {args.n}^3 lid-driven cavity, {args.mesh}, Re {args.re:g}, NEQ walls, {args.dtype}"
    bytes_per_step = 2.0 * Q * esize * cells
    achieved = bytes_per_step / (ms * 1e-3) / 1e9
    traffic = measured_traffic(workload)
    res = {
        "metric": METRIC,
        "value": round(cells / (ms * 1e-3) / 1e6, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (cavity from rest, no external data)",
        "config": {"workload": workload, "cells": cells, "Q": Q, "global_batch": 1, "seq_len": args.n,
                   "parallelism": "single GPU", "dt": cfg["dt"], "tau": cfg["tau"],
                   "kernel": {0: "general", 1: "fused-twice", 2: "fused"}.get(variant, str(variant))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_step},
        "wall_s_timed": round(wall, 3),
        "mass_total": tot[0],
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
