#!/usr/bin/env python3
"""Benchmark of the incompressible-DUGKS step on one MI355X.

Workload (headline): D3Q19 cubic lid-driven cavity, 128^3 cells, lid U = 0.1
along x, NEQ velocity walls on all six sides, rho0 = 1, RT = 1/3, dx = 1,
Re = 100 (tau = U N / (Re RT)), CFL 0.5, FP64, started from rest.  One
"step" is one full time step (Sec. II.B) over every cell and every
discrete velocity: one launch of the fused step kernel.  Prints one JSON
line:

  value      MLUPS = cells * steps / seconds / 1e6 (inputs resident in HBM)
  roofline   the step kernel's algorithmic HBM bytes (read f~ once, write f~
             once: 2 Q s bytes per cell) / its average launch time (HIP
             events on the launch stream over the timed steps), against the
             8 TB/s HBM peak; `traffic` = HBM bytes per launch measured with
             rocprofv3 counters (profiles/traffic.json), null when the kernel
             sources changed since
  also       the same workload in FP32, with the original-DUGKS
             equilibrium and on D3Q27; 64 uneven D2Q9 instances advanced by one batched
             launch per step (graph replay) vs 64 plain launches per step;
             the adjoint step vs the forward step (D2Q9 256^2 periodic, FP64)
  cpu_baseline  the FP64 CPU oracle timed on this host on a bounded sample
             of the same workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f64|f32]
       [--mesh uniform|tanh] [--re 100] [--n 128] [--no-cpu-baseline]
       [--no-extras]
       python bench.py --cavity-re12000   (the unsteady 2-D cavity of Sec. III)
       python bench.py --adjoint-only     (adjoint vs forward step, periodic and walled 256^2, periodic 1024^2)
       python bench.py --summarize-counters FETCH_DIR WRITE_DIR
         (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE output of
          `bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-extras
          --copy-probe`: writes profiles/traffic.json)
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
    three = lattice != 9
    d = dict(lattice=lattice, dtype=dtype, n=(n, n, n if three else 1),
             L=(float(n), float(n), float(n) if three else 1.0),
             mesh=(tanh, tanh, tanh if three else 0), k_stretch=1.5, rho0=1.0, RT=RT, tau=nu / RT,
             dt=1.0, bc=(1, 1, 1, 1, 1, 1) if three else (1, 1, 1, 1, 0, 0), uw=uw)
    d["dt"] = M.dugks_dt_from_cfl(d, 0.5)
    return d


# the sources the timed step kernels are compiled from, plus their launch
# policy (tile, chunk and kernel choice) and the ABI header: the counters are
# stale once any of these changes
KERNEL_SOURCES = ("kernels_split.hip", "kernels_fused.hip", "march.hpp", "kernels_general.hpp", "inst.hpp",
                  "lattice.hpp", "ctx.hpp", "../../include/dugks.h")


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1411_6121_amd", "csrc")
    for fn in KERNEL_SOURCES:
        with open(os.path.join(csrc, fn), "rb") as fh:
            h.update(os.path.basename(fn).encode())
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


def cpu_baseline(cfg, budget_s=15.0, max_steps=1000):
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


def _events():
    import torch

    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_steps(ctx, cfg, cur, nxt, steps, warmup, force=None):
    """ms per dugks_step (HIP events on the launch stream)"""
    import torch

    import paper_1411_6121_amd as M

    for k in range(warmup):
        M.dugks_step(ctx, cur, nxt, force, k * cfg["dt"])
        cur, nxt = nxt, cur
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for k in range(steps):
        M.dugks_step(ctx, cur, nxt, force, (warmup + k) * cfg["dt"])
        cur, nxt = nxt, cur
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, cur


def batch_cfg(spec, dtype):
    """one instance of the uneven D2Q9 set: cavity (lid U) or periodic-x
    channel driven by a uniform body force"""
    nx, ny, U, RT = spec["nx"], spec["ny"], spec["U"], 1.0 / 3.0
    nu = U * ny / spec["Re"]
    if spec["kind"] == "cavity":
        bc = (1, 1, 1, 1, 0, 0)
        uw = [[0, 0, 0], [0, 0, 0], [0, 0, 0], [U, 0, 0], [0, 0, 0], [0, 0, 0]]
    else:
        bc = (0, 0, 1, 1, 0, 0)
        uw = [[0, 0, 0]] * 6
    return dict(lattice=9, dtype=dtype, n=(nx, ny, 1), L=(float(nx), float(ny), 1.0), rho0=1.0, RT=RT,
                tau=nu / RT, dt=0.5, bc=bc, uw=uw, G=(spec["force"], 0.0, 0.0))


def bench_batched(dtype="f64", count=64, steps=5000, warmup=5):
    """one batched launch per step (graph replay) vs one plain launch per
    instance per step; both give bitwise-identical states"""
    import torch

    import paper_1411_6121_amd as M
    from synthetic import batch_instances

    cfgs = [batch_cfg(s, dtype) for s in batch_instances(seed=3, count=count)]
    cells = sum(c["n"][0] * c["n"][1] for c in cfgs)
    B = M.BatchSolver(cfgs)
    try:
        tile, chunk = B.tune(nsteps=3)
        B.run(warmup, use_graph=True)
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        B.run(steps, use_graph=True)
        e1.record()
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / steps
    finally:
        B.close()
    ctxs, bufs = [], []
    try:
        for c in cfgs:
            Q, D, shp = M.shape_of(c)
            f = torch.empty((Q,) + shp, dtype=M.torch_dtype(c), device="cuda")
            bufs.append([f, torch.empty_like(f)])
            ctxs.append(M.dugks_init(c, f))
        for k in range(warmup):
            for i, c in enumerate(cfgs):
                M.dugks_step(ctxs[i], bufs[i][0], bufs[i][1], None, k * c["dt"])
                bufs[i].reverse()
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        for k in range(steps):
            for i, c in enumerate(cfgs):
                M.dugks_step(ctxs[i], bufs[i][0], bufs[i][1], None, (warmup + k) * c["dt"])
                bufs[i].reverse()
        e1.record()
        torch.cuda.synchronize()
        ms_s = e0.elapsed_time(e1) / steps
    finally:
        for x in ctxs:
            M.dugks_destroy(x)
    return {"workload": f"{count} D2Q9 instances, sides 64..512, Re 100..1000, {dtype}", "cells": cells,
            "steps": steps, "ms_per_step_batched_graph": round(ms_b, 4), "ms_per_step_sequential": round(ms_s, 4),
            "speedup": round(ms_s / ms_b, 3), "mlups_batched": round(cells / ms_b / 1e3, 1),
            "tuned": {"tile_variant": tile, "chunk": chunk},
            "accuracy": "bitwise identical to the plain launches"}


def bench_adjoint(n=256, steps=50, warmup=5, walls=False, full_steps=2000):
    """adjoint step vs forward step, D2Q9 n^2, FP64, tau = 1, with a
    body-force field (the gradient workload): periodic, or (walls) a
    lid-driven cavity with NEQ walls on a tanh mesh (k = 1.5)"""
    import torch

    import paper_1411_6121_amd as M
    from synthetic import gaussian_bumps

    cfg = dict(lattice=9, dtype="f64", n=(n, n, 1), L=(float(n), float(n), 1.0), rho0=1.0, RT=1 / 3, tau=1.0,
               dt=0.5, bc=(0,) * 6)
    if walls:
        uw = [[0.0] * 3 for _ in range(6)]
        uw[3] = [0.05, 0.0, 0.0]
        cfg.update(bc=(1, 1, 1, 1, 0, 0), uw=uw, mesh=(1, 1, 0), k_stretch=1.5)
        cfg["dt"] = M.dugks_dt_from_cfl(cfg, 0.5)
    Q, D, shp = M.shape_of(cfg)
    Gf = torch.from_numpy(gaussian_bumps(7, n)).to("cuda")
    f = torch.empty((Q,) + shp, dtype=torch.float64, device="cuda")
    g = torch.empty_like(f)
    ctx = M.dugks_init(cfg, f, force=Gf)
    try:
        ms_f, f = time_steps(ctx, cfg, f, g, steps, warmup, force=Gf)
        lam = torch.ones_like(f)
        lam2 = torch.empty_like(f)
        gG = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda")
        for k in range(warmup):
            M.dugks_step_adjoint(ctx, f, lam, lam2, Gf, 0.0, gG)
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        for k in range(steps):
            M.dugks_step_adjoint(ctx, f, lam, lam2, Gf, k * cfg["dt"], gG)
            lam, lam2 = lam2, lam
        e1.record()
        torch.cuda.synchronize()
        ms_a = e0.elapsed_time(e1) / steps
    finally:
        M.dugks_destroy(ctx)
    kind = "lid-driven cavity, NEQ walls, tanh mesh" if walls else "periodic"
    out = {"workload": f"D2Q9 {n}^2 {kind}, force field, f64", "ms_forward_step": round(ms_f, 4),
           "ms_adjoint_step": round(ms_a, 4), "ratio": round(ms_a / ms_f, 3)}
    if not walls and full_steps > 0:
        out["full_gradient"] = full_gradient_time(cfg, Gf, full_steps, ms_f)
    return out


def device_context(step_gbs):
    """HIP version torch was built with, the GPU architecture and the
    bandwidth of a plain 512 MiB device-to-device copy (bytes read + written
    / time), the practically reachable HBM rate that the step's algorithmic
    rate compares with"""
    import torch

    src = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = _events()
    reps = 10
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * src.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return {"torch_hip": torch.version.hip, "arch": torch.cuda.get_device_properties(0).gcnArchName,
            "copy_512MiB_GBps": round(gbs, 1), "step_vs_copy": round(step_gbs / gbs, 4)}


def full_gradient_time(cfg, Gtar, nsteps, ms_forward):
    """Wall time of one whole gradient (checkpointed forward, recompute and
    adjoint steps, initial-state and read-out VJPs, host calls included) of
    the MSE between the final velocity at zero force and at Gtar, in units
    of plain forward steps"""
    import math
    import time

    import torch

    import paper_1411_6121_amd as M
    from paper_1411_6121_amd.autograd import rollout

    Q, D, shp = M.shape_of(cfg)
    zero_u = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda")
    with torch.no_grad():
        u_tar = rollout(cfg, Gtar, zero_u, nsteps)

    def grad_once():
        G = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda", requires_grad=True)
        ((rollout(cfg, G, zero_u, nsteps) - u_tar) ** 2).mean().backward()
        return G.grad

    grad_once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = grad_once()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    if not bool(torch.isfinite(g).all()):
        raise SystemExit("non-finite gradient")
    return {"steps": nsteps, "checkpoints": math.ceil(math.sqrt(nsteps)), "ms": round(ms, 2),
            "forward_step_units": round(ms / (nsteps * ms_forward), 2)}


def summarize_counters(fetch_dir, write_dir, workload):
    """HBM bytes per launch of the step kernel from rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs, each scaled by what the counter reads for the plain
    256 MiB device copy in the same run; writes profiles/traffic.json"""
    import csv
    import statistics

    def rows(d):
        return list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))

    def per_dispatch(rs, name):
        step = [float(r["Counter_Value"]) for r in rs if r["Counter_Name"] == name and
                ("k_fused2<" in r["Kernel_Name"] or "k_split<" in r["Kernel_Name"])]
        copy = [float(r["Counter_Value"]) for r in rs if r["Counter_Name"] == name and "copyBuffer" in r["Kernel_Name"]
                and int(r["Grid_Size"]) >= 65536]
        return step, copy

    probe_kib = 256 * 1024.0
    fs, fc = per_dispatch(rows(fetch_dir), "FETCH_SIZE")
    ws, wc = per_dispatch(rows(write_dir), "WRITE_SIZE")
    if not (fs and fc and ws and wc):
        raise SystemExit("counter files lack the step kernel or the 256 MiB copy probe")
    kf = probe_kib / statistics.median(fc)
    kw = probe_kib / statistics.median(wc)
    fetch = statistics.mean(fs) * kf * 1024
    write = statistics.mean(ws) * kw * 1024
    p = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(p)) if os.path.exists(p) else {}
    data[workload] = {"source_hash": source_hash(), "bytes_per_launch": round(fetch + write),
                      "fetch_bytes": round(fetch), "write_bytes": round(write),
                      "fetch_scale": round(kf, 4), "write_scale": round(kw, 4),
                      "raw_fetch_kib": round(statistics.mean(fs), 1), "raw_write_kib": round(statistics.mean(ws), 1),
                      "dispatches": len(fs)}
    os.makedirs(os.path.dirname(p), exist_ok=True)
    with open(p, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(data[workload]))


def cavity12000_cfg(n, dtype="f64"):
    """Sec. III 2-D cavity at Re = 12000: L = 1, lid U = 1, RT = 100/3,
    bounce-back walls, tanh mesh with k = 2.5, CFL 0.5, from rest"""
    import paper_1411_6121_amd as M

    U, RT, nu = 1.0, 100.0 / 3.0, 1.0 / 12000.0
    uw = [[0.0] * 3 for _ in range(6)]
    uw[3] = [U, 0.0, 0.0]
    d = dict(lattice=9, dtype=dtype, n=(n, n, 1), L=(1.0, 1.0, 1.0), mesh=(1, 1, 0), k_stretch=2.5, rho0=1.0, RT=RT,
             tau=nu / RT, dt=1.0, bc=(3, 3, 3, 3, 0, 0), uw=uw)
    d["dt"] = M.dugks_dt_from_cfl(d, 0.5)
    return d


def bench_wall_subsets(args):
    """ms per step of the timed cavity (same mesh, lattice, precision and
    time step) with walls on all axes, on none, and on each axis or pair
    alone, the other axes periodic; the wall kinds stay those of the cavity
    (NEQ, lid on the +y side)"""
    import torch

    import paper_1411_6121_amd as M

    subsets = {"all": "xyz", "none": "", "x": "x", "y": "y", "z": "z", "xy": "xy"}
    out = {}
    for name, axes in subsets.items():
        cfg = cavity_cfg(args.n, args.dtype, args.mesh, args.re, lattice=args.lattice)
        cfg["bc"] = tuple(1 if "xyz"[a // 2] in axes else 0 for a in range(6))
        Q, D, shp = M.shape_of(cfg)
        f = torch.empty((Q,) + shp, dtype=M.torch_dtype(cfg), device="cuda")
        g = torch.empty_like(f)
        ctx = M.dugks_init(cfg, f)
        try:
            ms, cur = time_steps(ctx, cfg, f, g, args.steps, args.warmup)
            M.dugks_moments(ctx, cur)  # the state stays finite
        finally:
            M.dugks_destroy(ctx)
        del f, g, cur
        out[name] = round(ms, 5)
        print(f"walls on {name or 'none'}: {ms:.4f} ms", file=sys.stderr, flush=True)
    return {"workload": workload_name(args.n, args.mesh, args.re, args.dtype, args.lattice),
            "ms_per_step_by_wall_axes": out, "steps": args.steps, "warmup": args.warmup}


def main_frequency(t, ek):
    """frequency of the largest spectral peak of E_k(t) above 0.05 (E_k
    detrended by a quadratic fit, Hann window), and the resolution 1/T"""
    import numpy as np

    tc = t - t.mean()
    e = ek - np.polyval(np.polyfit(tc, ek, 2), tc)
    F = np.abs(np.fft.rfft(e * np.hanning(len(e)))) ** 2
    fr = np.fft.rfftfreq(len(e), d=t[1] - t[0])
    sel = fr > 0.05
    return float(fr[sel][np.argmax(F[sel])]), float(1.0 / (t[-1] - t[0])), float(e.std() / ek.mean())


def run_cavity12000(n, t_end, sample_dt=0.02):
    """advance the Re = 12000 cavity from rest to t_end, E_k recorded on the
    device every sample_dt (dugks_totals_async); reports the main frequency
    of E_k over the second half and the steady criterion of Sec. III (relative
    velocity change over the last 1000 steps)"""
    import numpy as np
    import torch

    import paper_1411_6121_amd as M

    d = cavity12000_cfg(n)
    dt = d["dt"]
    every = max(1, int(round(sample_dt / dt)))
    nsamp = int(t_end / (every * dt))
    fa = torch.empty((9, 1, n, n), dtype=torch.float64, device="cuda")
    fb = torch.empty_like(fa)
    hist = torch.zeros((nsamp, 6), dtype=torch.float64, device="cuda")
    ctx = M.dugks_init(d, fa)
    try:
        cur, nxt = fa, fb
        e0, e1 = _events()
        e0.record()
        last = time.time()
        for s in range(nsamp):
            if M.dugks_run(ctx, cur, nxt, every):
                cur, nxt = nxt, cur
            M.dugks_totals_async(ctx, cur, hist[s])
            if time.time() - last > 20:
                last = time.time()
                print(f"[re12000 {n}^2] t = {(s + 1) * every * dt:.0f} of {t_end:g}", file=sys.stderr, flush=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        prev = cur.clone()
        if M.dugks_run(ctx, cur, nxt, 1000):
            cur, nxt = nxt, cur
        dn, bn = M.dugks_velocity_change(ctx, prev, cur)
    finally:
        M.dugks_destroy(ctx)
    h = hist.cpu().numpy()
    if h[:, 5].any():
        raise RuntimeError("non-finite values during the Re = 12000 run")
    t = (np.arange(nsamp) + 1) * every * dt
    late = t > t_end / 2
    f, res, osc = main_frequency(t[late], h[late, 4])
    steps = nsamp * every
    return {"n": n, "t_end": round(float(t[-1]), 2), "steps": steps, "dt": dt,
            "ms_per_step": round(ms / steps, 5), "mlups": round(n * n * steps / (ms * 1e3), 1),
            "ek_final": round(float(h[-1, 4]), 6), "ek_oscillation_rel": float(f"{osc:.3g}"),
            "main_frequency": round(f, 4), "frequency_resolution": round(res, 4),
            "velocity_change_1000_steps": float(f"{dn / bn:.3g}")}


def bench_cavity12000(sizes=(128, 96, 80)):
    """128^2 and 96^2 to t = 3000, 80^2 (steady early) to t = 1500"""
    out = {"workload": "D2Q9 cavity Re 12000, tanh mesh k = 2.5, bounce-back walls, f64, from rest",
           "paper": {"128": "periodic, main frequency 0.6144", "80, 96": "steady"}}
    ends = {128: 3000.0, 96: 3000.0, 80: 1500.0}
    for n in sizes:
        te = ends.get(n, 3000.0)
        out[str(n)] = run_cavity12000(n, te)
        print(f"[re12000 {n}^2] {json.dumps(out[str(n)])}", file=sys.stderr, flush=True)
    return out


def workload_name(n, mesh, re, dtype, lattice=19):
    dims = f"{n}^2" if lattice == 9 else f"{n}^3"
    return f"D{2 if lattice == 9 else 3}Q{lattice} {dims} lid-driven cavity, {mesh}, Re {re:g}, NEQ walls, {dtype}"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--mesh", default="uniform", choices=["uniform", "tanh"])
    ap.add_argument("--re", type=float, default=100.0)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--lattice", type=int, default=19, choices=[9, 19, 27],
                    help="velocity set of the timed cavity (the headline is D3Q19)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32 / batched / adjoint figures")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter scaling)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--adjoint-only", action="store_true",
                    help="print only the adjoint figures (periodic and walled D2Q9 256^2) as one JSON line")
    ap.add_argument("--profile-case", choices=["adjoint1024", "batch64"],
                    help="a few steps of one extra workload for the profiler (D2Q9 1024^2 periodic adjoint "
                         "with its forward steps, or the 64-instance FP64 batch), one JSON line")
    ap.add_argument("--cavity-re12000", action="store_true",
                    help="run the Re = 12000 2-D cavity (128^2 and 96^2 to t = 3000, 80^2 to t = 1500; "
                         "about six minutes) and print its JSON line instead of the benchmark")
    ap.add_argument("--re12000-sizes", type=int, nargs="+", default=[128, 96, 80],
                    help="meshes of the Re = 12000 run")
    ap.add_argument("--wall-subsets", action="store_true",
                    help="time the timed cavity's step with walls on subsets of the axes (the others "
                         "periodic) and print one JSON line: what the walls cost")
    args = ap.parse_args()

    workload = workload_name(args.n, args.mesh, args.re, args.dtype, args.lattice)
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, workload)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only (the step is measured on one MI355X); "
              "multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1411_6121_amd as M

    torch.cuda.init()
    if args.cavity_re12000:
        print(json.dumps(bench_cavity12000(tuple(args.re12000_sizes))))
        return
    if args.wall_subsets:
        print(json.dumps(bench_wall_subsets(args)))
        return
    if args.profile_case == "adjoint1024":
        print(json.dumps({"adjoint_1024": bench_adjoint(1024, steps=args.steps, warmup=args.warmup,
                                                         full_steps=0)}))
        return
    if args.profile_case == "batch64":
        print(json.dumps({"batched": bench_batched("f64", steps=args.steps, warmup=args.warmup)}))
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": bench_adjoint(), "adjoint_walls": bench_adjoint(walls=True),
                          "adjoint_1024": bench_adjoint(1024, steps=20, full_steps=0)}))
        return
    cfg = cavity_cfg(args.n, args.dtype, args.mesh, args.re, lattice=args.lattice)
    Q, D, shp = M.shape_of(cfg)
    cells = int(shp[0] * shp[1] * shp[2])
    esize = 8 if args.dtype == "f64" else 4
    f = torch.empty((Q,) + shp, dtype=M.torch_dtype(cfg), device="cuda")
    g = torch.empty_like(f)
    ctx = M.dugks_init(cfg, f)
    t_wall = time.perf_counter()
    ms, cur = time_steps(ctx, cfg, f, g, args.steps, args.warmup)
    wall = time.perf_counter() - t_wall
    # state must stay finite (the step ran for real)
    tot = M.dugks_moments(ctx, cur)
    variant = M.dugks_kernel_variant(ctx)
    M.dugks_destroy(ctx)
    del f, g, cur

    if args.copy_probe:
        buf = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")  # 256 MiB
        out = torch.empty_like(buf)
        for _ in range(3):
            out.copy_(buf)
        torch.cuda.synchronize()
        del buf, out

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
                   "kernel": {0: "general", 1: "fused-twice", 2: "fused", 3: "fused-split"}.get(variant, str(variant))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_step},
        "wall_s_timed": round(wall, 3),
        "mass_total": tot[0],
    }
    if not args.no_extras and args.lattice == 19:
        also = {}
        if args.dtype == "f64":
            c32 = cavity_cfg(args.n, "f32", args.mesh, args.re)
            f = torch.empty((Q,) + shp, dtype=torch.float32, device="cuda")
            g = torch.empty_like(f)
            ctx = M.dugks_init(c32, f)
            ms32, _ = time_steps(ctx, c32, f, g, args.steps, args.warmup)
            M.dugks_destroy(ctx)
            del f, g
            b32 = 2.0 * Q * 4 * cells
            also["f32"] = {"ms_per_step": round(ms32, 5), "mlups": round(cells / ms32 / 1e3, 2),
                           "hbm_frac": round(b32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        # the original-DUGKS equilibrium variant (same workload)
        corig = dict(cfg, model=1)
        f = torch.empty((Q,) + shp, dtype=M.torch_dtype(cfg), device="cuda")
        g = torch.empty_like(f)
        ctx = M.dugks_init(corig, f)
        kvo = M.dugks_kernel_variant(ctx)
        mso, _ = time_steps(ctx, corig, f, g, max(args.steps // 4, 10), max(args.warmup // 4, 2))
        M.dugks_destroy(ctx)
        del f, g
        also["original_model"] = {"ms_per_step": round(mso, 5), "mlups": round(cells / mso / 1e3, 2),
                                  "hbm_frac": round(bytes_per_step / (mso * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "kernel": "fused-split" if kvo == 3 else "general (two launches)"}
        # the paper's own 3-D velocity set on the same cavity
        c27 = cavity_cfg(args.n, args.dtype, args.mesh, args.re, lattice=27)
        f = torch.empty((27,) + shp, dtype=M.torch_dtype(c27), device="cuda")
        g = torch.empty_like(f)
        ctx = M.dugks_init(c27, f)
        ms27, _ = time_steps(ctx, c27, f, g, max(args.steps // 4, 10), max(args.warmup // 4, 2))
        M.dugks_destroy(ctx)
        del f, g
        b27 = 2.0 * 27 * esize * cells
        also["d3q27"] = {"ms_per_step": round(ms27, 5), "mlups": round(cells / ms27 / 1e3, 2),
                         "hbm_frac": round(b27 / (ms27 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        # the 128^3 cavity on the stretched mesh (tanh k = 1.5, Re 1000), both precisions
        for dt_name in ("f64", "f32"):
            ct = cavity_cfg(args.n, dt_name, "tanh", 1000.0)
            f = torch.empty((Q,) + shp, dtype=M.torch_dtype(ct), device="cuda")
            g = torch.empty_like(f)
            ctx = M.dugks_init(ct, f)
            kvt = M.dugks_kernel_variant(ctx)
            mst, _ = time_steps(ctx, ct, f, g, max(args.steps // 2, 10), max(args.warmup // 2, 2))
            M.dugks_destroy(ctx)
            del f, g
            bt = 2.0 * Q * (8 if dt_name == "f64" else 4) * cells
            also[f"tanh_re1000_{dt_name}"] = {
                "ms_per_step": round(mst, 5), "mlups": round(cells / mst / 1e3, 2),
                "hbm_frac": round(bt / (mst * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "kernel": {0: "general", 1: "fused-twice", 2: "fused", 3: "fused-split"}.get(kvt, str(kvt))}
        also["batched"] = bench_batched()
        also["batched_f32"] = bench_batched("f32")
        also["adjoint"] = bench_adjoint()
        also["adjoint_walls"] = bench_adjoint(walls=True)
        also["adjoint_1024"] = bench_adjoint(1024, steps=20, full_steps=0)
        res["also"] = also
        res["context"] = device_context(achieved)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
