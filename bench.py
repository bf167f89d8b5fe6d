#!/usr/bin/env python3
"""Throughput of the leap-format dynamical-core step on one MI355X.

Workload: the 0.25-degree grid (1440 x 720 intervals x 30 sigma levels, dt = 120 s,
M = 4 adaptation sub-steps) on a seeded synthetic atmosphere (solid-body wind plus a
degree <= 40 random streamfunction of peak 8 m/s, 6 km terrain, balanced p_s with 1%
noise, 3 K temperature noise).  One bench step = one forward outer step (12
adaptation + 3 advection stage launches) that keeps its stage inputs, followed by
the adjoint of that step (reverse sweep over them) in FP32 storage with FP64
accumulation.  The adjoint that recomputes its stage inputs is timed separately.
The metric is grid-point updates per second: nx * ny * nz per bench step.

Printed: one JSON line with the value, forward-only and adjoint-only rates, a
48-step adjoint window with checkpoints every 8 steps (time and checkpoint bytes),
the FP64 repeat and FP32/FP64 speedup, the HBM roofline of the dominant kernel
(the row-fused adaptation-stage adjoint, timed live with HIP events that the library records
on its launch stream around each of its launches in the timed steps; the forward adaptation
and advection stages beside it), the
24-member mixed ensemble (one persistent launch per stage, hipGraph replay), and
the FP64 CPU oracle timed on the host on a bounded sample of the same workload.
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
    """Hash of the sources every kernel is built from (stage kernels, adjoint kernels, shared header)."""
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


def run_prec(cfg, st, prec, steps, warmup, adjoint, seed_lam=7):
    import torch
    from paper_2103_10114_amd import Dycore, synth
    core = Dycore(cfg.nx, cfg.ny, cfg.nz, cfg.dt, prec=prec, phis=st["phis"], forward_only=not adjoint)
    d = core.to_device(st)
    lam = core.to_device(synth.random_like(st, seed_lam)) if adjoint else None

    def one():
        if adjoint:
            # the forward step keeps its stage inputs; the adjoint of that step sweeps back over them
            core.step_record(d)
            core.step_adjoint_recorded(lam)
        else:
            core.step(d, 1)

    for _ in range(warmup):
        one()
    if adjoint:
        # events around each launch of the row-fused adaptation-stage adjoint in the timed steps
        core.kernel_timer_start(3 * core.substeps * steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    core.kernel_timing = core.kernel_timer_stop() if adjoint else (0.0, 0)
    nonfinite = core.count_nonfinite(d)
    return core, d, el, nonfinite


def roofline(core, d, cfg, elem, reps=10):
    """Average duration of an adaptation and of an advection stage (the tile kernel and its pole
    cap-sum pre-kernel), timed with HIP events on the launch stream over reps RK3 steps of each
    process alone."""
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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c4_fp32.json")
# the two launches of a forward advection stage: band tiles and, beside them, the polar tiles
ADVECTION_LAUNCHES = ("k_stage_atile<float,256,false>", "k_stage_atile<float,256,true>")


def traffic_from_profiles(kernel_hash, key):
    """HBM bytes per launch of kernel `key` (a name, or a tuple of the launches that together make
    one stage, summed) from the committed PMC summary, while it was taken from the kernels built now
    (same source hash); None otherwise."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        t = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if t.get("kernel_hash") != kernel_hash:
        return None
    ks = t.get("kernels", {})
    keys = key if isinstance(key, tuple) else (key,)
    if any(k not in ks for k in keys):
        return None
    return sum(ks[k]["fetch_bytes"] + ks[k]["write_bytes"] for k in keys)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(msub):
    """The FP64 oracle as it stands, on the host, on a bounded sample of the 0.25-degree workload:
    one adaptation stage and one advection stage, each forward and adjoint, on the full
    1440x720x30 grid with all OpenMP threads (the forward stages run their rows in parallel, the
    adjoint sweep is serial).  The rate of a whole bench step (one forward outer step + one adjoint
    outer step, whose forward recompute repeats the forward stages) is scaled from these four
    timings: 2 (3M t_A + 3 t_L) + 3M t_A' + 3 t_L'.  Also: the adaptation stage forward at 1 thread
    on the same grid, and one forward outer step of the 128x64x9 grid at 1 thread and at all
    threads."""
    import oracle
    from paper_2103_10114_amd import synth
    cfg = synth.CONFIGS["c4"]
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    lam = synth.random_like(st, 7)
    threads = oracle.num_threads()
    h = cfg.dt / msub
    t = {}
    for which, ch in (("A", h), ("L", cfg.dt)):
        t0 = time.perf_counter()
        o.stage(st, st, ch, which)
        t1 = time.perf_counter()
        o.adj_stage(st, lam, ch, which)
        t2 = time.perf_counter()
        t[which] = (t1 - t0, t2 - t1)
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    o.stage(st, st, h, "A")
    t_a1 = time.perf_counter() - t0
    oracle.set_num_threads(threads)
    del o, st, lam
    fwd = 3 * msub * t["A"][0] + 3 * t["L"][0]
    step = 2 * fwd + 3 * msub * t["A"][1] + 3 * t["L"][1]
    pts = cfg.nx * cfg.ny * cfg.nz
    # thread scaling on a small grid
    c1 = synth.CONFIGS["c1"]
    s1 = synth.make_state(c1)
    o1 = oracle.Oracle(c1.nx, c1.ny, c1.nz, phis=s1["phis"])
    rates = {}
    for n in (1, threads):
        oracle.set_num_threads(n)
        t0 = time.perf_counter()
        o1.step(s1, 1, c1.dt)
        rates[n] = c1.nx * c1.ny * c1.nz / (time.perf_counter() - t0)
    oracle.set_num_threads(threads)
    return {"value": pts / step, "unit": "grid-pt updates/s", "cores": threads, "kind": "oracle",
            "sample": (f"1440x720x30 grid, FP64: one adaptation stage forward {t['A'][0]:.2f} s and adjoint "
                       f"{t['A'][1]:.2f} s, one advection stage forward {t['L'][0]:.2f} s and adjoint "
                       f"{t['L'][1]:.2f} s ({threads} OpenMP threads over rows for the forward; the "
                       f"adjoint sweep is serial); scaled to one forward + one adjoint outer step "
                       f"(M {msub}: {3 * msub} + 3 stages each way, forward stages twice)"),
            "forward_updates_per_s": pts / fwd, "adjoint_sweep": "serial", "cpu_model": cpu_model(),
            "c4_adaptation_stage_s": {"threads_1": t_a1, f"threads_{threads}": t["A"][0]},
            "c1_forward_updates_per_s": {"threads_1": rates[1], f"threads_{threads}": rates[threads]}}


def ensemble_c5(steps):
    """The 24-member mixed ensemble (8 each of 128x64x9, 256x128x30, 720x360x30): one persistent
    launch per stage at the autotuned workgroup size, the batched step captured once in a hipGraph
    and replayed; then the one-step adjoint of every member (dycore_step_adjoint, member after
    member, from its state after the replays, with a seeded output adjoint)."""
    import torch
    from paper_2103_10114_amd import Batch, Dycore, synth
    cfgs = [synth.ensemble_member(m) for m in range(24)]
    cores, states = [], []
    for cfg in cfgs:
        st = synth.make_state(cfg)
        c = Dycore(cfg.nx, cfg.ny, cfg.nz, cfg.dt, prec="fp32", phis=st["phis"])
        cores.append(c)
        states.append(c.to_device(st))
    b, table = Batch.autotune(cores, states)
    b.step(1)
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        b.step(1)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pts = sum(c.nx * c.ny * c.nz for c in cfgs)
    bad = sum(core.count_nonfinite(st) for core, st in zip(cores, states))
    lams = [core.to_device(synth.random_like(st, 900 + m)) for m, (core, st) in enumerate(zip(cores, states))]
    for core, st, lam in zip(cores, states, lams):     # warm
        core.step_adjoint(st, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for core, st, lam in zip(cores, states, lams):
        core.step_adjoint(st, lam)
    torch.cuda.synchronize()
    ela = time.perf_counter() - t0
    bad_adj = sum(core.count_nonfinite(lam) for core, lam in zip(cores, lams))
    return {"value": pts * steps / el, "unit": "grid-pt updates/s", "members": len(cfgs), "points_per_step": pts,
            "steps": steps, "ms_per_step": el / steps * 1e3, "graph_replay": True, "nonfinite_after": bad,
            "block": min(table, key=table.get), "autotune_ms_per_step": {str(k): v for k, v in table.items()},
            "adjoint_one_step": {"ms_all_members": ela * 1e3, "updates_per_s": pts / ela,
                                 "nonfinite_after": bad_adj}}


def window_adjoint(core, d, lam, nsteps, ckpt):
    """nsteps forward outer steps, then the adjoint over all of them with recompute from checkpoints
    taken every ckpt steps (the window's step-start states recomputed from its checkpoint)."""
    import torch
    from paper_2103_10114_amd import adjoint_window
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, mem = adjoint_window(core, d, nsteps, lam, ckpt_every=ckpt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pts = core.nx * core.ny * core.nz
    return {"steps": nsteps, "ckpt_every": ckpt, "seconds": el, "updates_per_s": pts * nsteps / el,
            "checkpoint_bytes": mem["checkpoint_bytes"], "window_bytes": mem["window_bytes"],
            "checkpoints": mem["checkpoints"]}


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
    ap.add_argument("--no-c5", action="store_true", help="skip the 24-member ensemble")
    ap.add_argument("--window", type=int, default=48, help="steps of the checkpointed adjoint window (0: skip)")
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
                               f"M {msub}, forward{' + adjoint of that step (stage inputs kept by the forward)' if adjoint else ''} per step",
                   "nx": cfg.nx, "ny": cfg.ny, "nz": cfg.nz, "dt": cfg.dt, "adapt_substeps": msub,
                   "adjoint": adjoint, "block": core.block, "seed": cfg.seed},
        "nonfinite_after": nonfin,
    }
    if adjoint:
        import torch
        from paper_2103_10114_amd import synth as _s
        lam = core.to_device(_s.random_like(st, 7))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            core.step(d, 1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            core.step_adjoint(d, lam)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out["forward_updates_per_s"] = pts * args.steps / (t1 - t0)
        out["adjoint_updates_per_s"] = pts * args.steps / (t2 - t1)   # recomputing its stage inputs
        if args.window > 0:
            print(f"[bench] checkpointed adjoint window, {args.window} steps", file=sys.stderr, flush=True)
            out["adjoint_window"] = window_adjoint(core, d, lam, args.window, 8)
        del lam
    if not args.no_roofline:
        print("[bench] roofline timing", file=sys.stderr, flush=True)
        kh = kernel_source_hash()
        sb = state_bytes(cfg.nx, cfg.ny, cfg.nz, 4)
        ms, alg, ach = roofline(core, d, cfg, 4)
        stage_name = "k_stage_tile<float>"
        fwd = {"kernel": stage_name + " (adaptation stage)", "avg_launch_ms": ms["A"],
               "alg_bytes_per_launch": alg, "achieved": ach, "frac": ach / HBM_PEAK_GBS,
               "traffic": traffic_from_profiles(kh, stage_name),
               "advection": {"kernel": "k_stage_atile<float,256,false> (band tiles) beside "
                                       "k_stage_atile<float,256,true> (polar tiles)", "avg_launch_ms": ms["L"],
                             "achieved": alg / (ms["L"] * 1e-3) / 1e9,
                             "frac": alg / (ms["L"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "traffic": traffic_from_profiles(kh, ADVECTION_LAUNCHES)}}
        # the whole bench step: every forward stage moves 8/3 states, every stage adjoint 4
        nst = 3 * (msub + 1) if adjoint else 0
        step_states = 3 * (msub + 1) * 8.0 / 3.0 + 4.0 * nst
        step_ach = step_states * sb / (el / args.steps) / 1e9
        out["whole_step"] = {"alg_states": step_states, "alg_bytes": step_states * sb, "achieved": step_ach,
                             "unit": "GB/s", "frac": step_ach / HBM_PEAK_GBS}
        tot, n = core.kernel_timing
        if n > 0:
            # the dominant kernel of the bench step: over the three stages of an RK step the
            # adjoint reads the stage input and the output adjoint, writes the stage's input
            # adjoint and updates the step-input adjoint: 3 + 5 + 4 = 12 states, 4 per stage; the
            # timed launch covers rows 2..ny-2 of the ny+1 (rows 1 and ny-1 run in a launch of
            # their own after the pole rows' sums, the pole rows in the per-point kernels)
            ams = tot / n
            aalg = 4.0 * sb * (cfg.ny - 3) / (cfg.ny + 1)
            aach = aalg / (ams * 1e-3) / 1e9
            aname = "k_aat<float>"
            out["roofline"] = {"bound": "hbm", "achieved": aach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": aach / HBM_PEAK_GBS, "traffic": traffic_from_profiles(kh, aname),
                               "kernel": aname + " (tiled row-fused adaptation-stage adjoint, rows 2..ny-2)",
                               "avg_launch_ms": ams, "launches_timed": n, "alg_bytes_per_launch": aalg,
                               "kernel_hash": kh, "forward_stage": fwd}
        else:
            out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS, "traffic": fwd["traffic"],
                               "kernel": fwd["kernel"], "avg_launch_ms": ms["A"],
                               "advection_launch_ms": ms["L"], "alg_bytes_per_launch": alg, "kernel_hash": kh}
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
    if not args.no_c5:
        print("[bench] 24-member ensemble", file=sys.stderr, flush=True)
        out["ensemble_c5"] = ensemble_c5(5)
    if not args.no_cpu:
        print("[bench] cpu oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(msub)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
