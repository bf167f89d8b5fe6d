#!/usr/bin/env python3
"""Throughput of the leap-format dynamical-core step on one MI355X.

Workload: the 0.25-degree grid (1440 x 720 intervals x 30 sigma levels, dt = 120 s,
M = 4 adaptation sub-steps) on a seeded synthetic atmosphere (solid-body wind plus a
degree <= 40 random streamfunction of peak 8 m/s, 6 km terrain, balanced p_s with 1%
noise, 3 K temperature noise).  One bench step = one forward outer step (12
adaptation + 3 advection stage launches) followed by one adjoint outer step
(forward recompute + reverse sweep) in FP32 storage with FP64 accumulation.
The metric is grid-point updates per second: nx * ny * nz per bench step.

Printed: one JSON line with the value, the FP64 repeat and FP32/FP64 speedup, the
HBM roofline of the dominant kernel (adaptation stage) measured live with HIP
events on the launch stream, and the FP64 CPU oracle timed on the host.
"""
from __future__ import annotations

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


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fwd.hip", "adj.hip", "dycore_internal.h"):
        p = os.path.join(ROOT, "paper_2103_10114_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def state_bytes(nx, ny, nz, elem):
    return elem * ((ny + 1) * nz * nx * 2 + ny * nz * nx + (ny + 1) * nx)


def time_gpu(fn, reps):
    import torch
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3


def adapt_pipelined(nx):
    """The FP32 adaptation stage runs in its pipelined form when its 27 LDS rows fit in 160 KB."""
    return ((27 * nx * 4 + 15) // 16) * 16 + 2 * 128 * 8 <= 160 * 1024


def run_prec(cfg, st, prec, steps, warmup, adjoint, seed_lam=7):
    import torch
    from paper_2103_10114_amd import Dycore, synth
    core = Dycore(cfg.nx, cfg.ny, cfg.nz, cfg.dt, prec=prec, phis=st["phis"], forward_only=not adjoint)
    d = core.to_device(st)
    lam = core.to_device(synth.random_like(st, seed_lam)) if adjoint else None

    def one():
        core.step(d, 1)
        if adjoint:
            core.step_adjoint(d, lam)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nonfinite = core.count_nonfinite(d)
    return core, d, el, nonfinite


def roofline(core, d, cfg, elem, reps=10):
    """Average launch duration of the adaptation and advection stage kernels, timed with HIP
    events on the launch stream over reps RK3 steps of each process alone."""
    ms = {}
    for proc in ("A", "L"):
        h = cfg.dt / core.substeps if proc == "A" else cfg.dt
        core.process_run(d, proc, 1, h)     # warm
        el = time_gpu(lambda: core.process_run(d, proc, reps, h), 1)
        ms[proc] = el / (3 * reps) * 1e3
    # algorithmic bytes per launch: an RK3 step moves 8 states (stage 1 r+w, stages 2-3 r+r+w)
    alg = 8.0 / 3.0 * state_bytes(cfg.nx, cfg.ny, cfg.nz, elem)
    ach = alg / (ms["A"] * 1e-3) / 1e9
    return ms, alg, ach


def traffic_from_profiles(kernel_hash):
    p = os.path.join(ROOT, "profiles", "traffic_adapt_stage_c4_fp32.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except Exception:
        return None
    if t.get("kernel_hash") != kernel_hash:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline():
    """The FP64 oracle as it stands, on the host: one forward and one adjoint outer step with the
    0.25-degree step structure (dt = 120 s, M = 4: 15 stages each way) on the 256 x 128 x 30 grid."""
    import dataclasses
    import oracle
    from paper_2103_10114_amd import synth
    cfg = dataclasses.replace(synth.CONFIGS["c2"], dt=120.0)
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    lam = synth.random_like(st, 7)
    t0 = time.perf_counter()
    s1 = o.step(st, 1, cfg.dt, msub=4)
    t1 = time.perf_counter()
    o.adj_step(s1, lam, cfg.dt, msub=4)
    t2 = time.perf_counter()
    pts = cfg.nx * cfg.ny * cfg.nz
    return {"value": pts / (t2 - t0), "unit": "grid-pt updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"1 forward + 1 adjoint outer step, 15 stages each (dt 120 s, M 4), FP64, on the "
                       f"256x128x30 grid ({pts} points); forward {t1 - t0:.2f} s with OpenMP over rows, "
                       f"adjoint {t2 - t1:.2f} s serial"),
            "forward_updates_per_s": pts / (t1 - t0)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the whole global grid is resident on one MI355X; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_10114_amd import lib, synth
    lib()  # fail loudly if the HIP library is missing
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calib_copy:
        src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = synth.CONFIGS[args.config]
    print(f"[bench] building synthetic state {cfg.nx}x{cfg.ny}x{cfg.nz}", file=sys.stderr, flush=True)
    st = synth.make_state(cfg)
    adjoint = not args.no_adjoint
    pts = cfg.nx * cfg.ny * cfg.nz

    print(f"[bench] fp32 steps={args.steps} warmup={args.warmup} adjoint={adjoint}", file=sys.stderr, flush=True)
    core, d, el, nonfin = run_prec(cfg, st, "fp32", args.steps, args.warmup, adjoint)
    value = pts * args.steps / el
    msub = core.substeps
    out = {
        "metric": "grid-pt updates/s fwd+adjoint FP32 vs FP64 at 0.25°; % HBM roofline",
        "value": value,
        "unit": "grid-pt updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"leap-format dycore step, {cfg.nx}x{cfg.ny}x{cfg.nz} (0.25 deg), dt {cfg.dt:g} s, "
                               f"M {msub}, forward{' + adjoint' if adjoint else ''} per step",
                   "nx": cfg.nx, "ny": cfg.ny, "nz": cfg.nz, "dt": cfg.dt, "adapt_substeps": msub,
                   "adjoint": adjoint, "block": core.block, "seed": cfg.seed},
        "nonfinite_after": nonfin,
    }
    if not args.no_roofline:
        print("[bench] roofline timing", file=sys.stderr, flush=True)
        ms, alg, ach = roofline(core, d, cfg, 4)
        kh = kernel_source_hash()
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": traffic_from_profiles(kh),
                           "kernel": f"k_stage<float,{-(-cfg.nx // core.block)},{2 if adapt_pipelined(cfg.nx) else 0}> "
                                     "(adaptation stage)",
                           "avg_launch_ms": ms["A"], "advection_launch_ms": ms["L"],
                           "alg_bytes_per_launch": alg, "kernel_hash": kh}
    del core, d
    torch.cuda.empty_cache()
    if not args.no_fp64:
        s64 = max(2, args.steps // 2)
        print(f"[bench] fp64 steps={s64}", file=sys.stderr, flush=True)
        core64, d64, el64, nonfin64 = run_prec(cfg, st, "fp64", s64, 1, adjoint)
        v64 = pts * s64 / el64
        out["fp64"] = {"value": v64, "ms_per_step": el64 / s64 * 1e3, "steps": s64, "nonfinite_after": nonfin64}
        out["speedup_fp32_over_fp64"] = value / v64
        if not args.no_roofline:
            ms64, alg64, ach64 = roofline(core64, d64, cfg, 8, reps=5)
            out["fp64"]["roofline"] = {"achieved": ach64, "frac": ach64 / HBM_PEAK_GBS, "avg_launch_ms": ms64["A"]}
        del core64, d64
    if not args.no_cpu:
        print("[bench] cpu oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
