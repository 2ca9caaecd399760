#!/usr/bin/env python3
"""Benchmark of the staggered CG hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--suite default|mixed32|batch24|serve|...]

Default workload (one JSON line): FP64 staggered CG solves of (m^2 - D^2) x = b
to relative true residual 1e-10 on a 32^4 lattice (links proj_SU3(exp(0.5 i
H)), seed 103; Gaussian source, seed 203; m = 0.01; both parities), the
largest single-GPU configuration of the metric.  One step is one complete
solve on the GPU (the fused CG kernels, the device-side scalars and stopping
test, and the FP64 true-residual check); the gauge field and the source are
resident in HBM before the timed region.  `value` is solves/s over the K
timed steps.

The same line reports:
  mixed         FP32 and FP16 reliable-update solves/s of the same system and
                their ratio to FP64;
  roofline      the FP64 D_slash kernel on the same 32^4 field (working set
                0.9 GB, far beyond the 256 MB Infinity Cache): 100
                full-lattice applications per run, HIP events on the library's
                stream; achieved = algorithmic bytes per output site (8 links
                + 1 gathered input vector + 1 output vector: 864 B with two
                stored link rows, 1248 B with three) x V / mean duration;
  cg_iteration  the solve's bytes per CG iteration over its time per iteration;
  c2_16         the 16^4 workload (eps 0.3, m 0.05): FP64 solves/s and the
                D_slash, cache-resident and cold (8 fields cycled);
  batch24       24^4, twelve sources: FP64 one by one against FP32 / FP16
                reliable-update batched solves, and the ratios;
  serve         four resident fields 8^4..32^4, a Poisson request stream at
                half the measured saturation rate: p50 / p99 latency overall
                and per lattice size;
  cpu_baseline  the FP64 CPU oracle solving the same 32^4 system once on the
                host cores (model, sockets and cores recorded).

Other suites (--suite) print their own JSON line: sweeps of the 32^4 mixed
solves, the 24^4 batch, the serving load, the device-copy calibration, the
CPU oracle on all workloads and the Wilson-fermion solver.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CG solves/s to 1e-10 (mixed vs FP64) + D_slash HBM GB/s % of peak; p99"
HBM_PEAK_GBS = 8000.0


def dslash_bytes_per_site(rows: int) -> int:
    """FP64 D_slash algorithmic bytes per output site: 8 links of 3 x rows
    complex entries, one gathered input vector and one output vector."""
    return 8 * 3 * rows * 16 + 48 + 48


def cg_bytes_per_half_site(rows: int) -> int:
    """FP64 CG iteration, algorithmic bytes per site of one parity system:
    K1 (links, r and p gathered, ap and p' stored) + K2 (links, ap gathered,
    p' read, x and r read and written)."""
    links = 8 * 3 * rows * 16
    return (links + 96 + 48 + 48) + (links + 48 + 48 + 96 + 96)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_f64_32x32x32x32_traffic.txt")
KERNEL_SOURCES = ["dslash.hip", "hop.hpp", "stag_types.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1311_2719_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(volume: int, path: str = TRAFFIC_FILE):
    """HBM bytes per D_slash launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    try:
        fields = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        if fields.get("kernel_source_hash") != kernel_hash() or int(fields.get("volume", -1)) != volume:
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--suite", default="default",
                    choices=["default", "mixed32", "batch24", "serve", "copy", "cpu_baseline", "wilson",
                             "kernels32", "md"])
    ap.add_argument("--oracle-threads-one", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--dslash-reps", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving point")
    ap.add_argument("--no-cold", action="store_true", help="skip the cold 16^4 D_slash")
    ap.add_argument("--cpu-seconds", type=float, default=25.0, help="bound on the CPU oracle baseline's time")
    ap.add_argument("--serve-requests", type=int, default=None,
                    help="requests per serving point (default 500; 2000 for --suite serve)")
    ap.add_argument("--serve-load", type=float, default=0.5, help="load of the default run's serving point")
    ap.add_argument("--serve-loads", type=float, nargs="*", default=[0.25, 0.5, 0.75, 0.9, 1.0, 1.2])
    args = ap.parse_args()
    if args.serve_requests is None:
        args.serve_requests = 2000 if args.suite == "serve" else 500
    return args


def timed_solves(ctx, f, b, x, steps, warmup, **kw):
    import torch

    for _ in range(warmup):
        ctx.cg_solve(f, b, x, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        infos.append(ctx.cg_solve(f, b, x, **kw))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, infos


def dslash_timing(ctx, f, b, reps, batches=5, **kw):
    """Per-launch durations (s) of the FP64 D_slash (full lattice unless kw
    names a parity and site range), from HIP events recorded on the stream
    the library launches on; and the mean per launch of `reps` launches back
    to back under one event pair, the median over `batches` such runs (a
    transient disturbance of one run does not set the figure)."""
    import torch

    out = ctx.new_fermion(f)
    s = ctx.stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for _ in range(10):
        ctx.dslash(f, b, out, **kw)
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(s)
        ctx.dslash(f, b, out, **kw)
        e1.record(s)
    torch.cuda.synchronize()
    per_launch = np.array([e0.elapsed_time(e1) * 1e-3 for e0, e1 in ev])
    means = []
    for _ in range(batches):
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record(s)
        for _ in range(reps):
            ctx.dslash(f, b, out, **kw)
        a1.record(s)
        torch.cuda.synchronize()
        means.append(a0.elapsed_time(a1) * 1e-3 / reps)
    return per_launch, float(np.median(means))


def _host_cpu():
    """The host CPU as lscpu reports it: model, sockets, cores, threads."""
    import subprocess

    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        info["physical_cores"] = int(info["Socket(s)"]) * int(info["Core(s) per socket"])
    except (KeyError, ValueError):
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return info


def cpu_baseline(dims, U, b, m, tol, gpu_iters, max_seconds=30.0):
    """The oracle's FP64 solve of the same system on the host cores: whole
    solves until max_seconds have passed (at least one)."""
    import oracle

    t0 = time.perf_counter()
    n = 0
    it = 0
    while True:
        x, _, info = oracle.cg_solve(dims, U, m, b, tol=tol)
        n += 1
        it = info["iters"]
        if time.perf_counter() - t0 > max_seconds or n >= 40:
            break
    dt = (time.perf_counter() - t0) / n
    host = _host_cpu()
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d complete FP64 solve(s) of the same %s system (oracle iterations %d, GPU %d), %.1f s"
                      % (n, "x".join(map(str, dims)), it, gpu_iters, dt * n),
            "host": host}


def _gen(kind, dims, eps, seed):
    from paper_1311_2719_amd import inputs

    if kind == "smooth":
        return inputs.smooth_su3(dims, eps, seed)
    return inputs.gaussian_source(dims, seed)


def generate(specs):
    """Host arrays for every workload, generated in parallel worker processes
    (each array from its own seeded generator, so the result is the same as a
    serial run).  Called before anything touches the GPU."""
    import concurrent.futures as cf
    import multiprocessing as mp

    workers = max(1, min(len(specs), 8, (os.cpu_count() or 2) - 1))
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        futs = {k: ex.submit(_gen, *v) for k, v in specs.items()}
        return {k: f.result() for k, f in futs.items()}


def serve_stream(ctx, fields, kinds, masses, bs, xs, rate, n, rng, precision, tol=1e-10):
    """Submit n requests (request i on fields[kinds[i]]) at Poisson times of
    the given rate (inf: all at once); latency = completion - scheduled
    arrival.  Returns (latencies, ok count, wall seconds)."""
    arr = np.cumsum(rng.exponential(1.0 / rate, n)) if np.isfinite(rate) else np.zeros(n)
    t0 = time.perf_counter()
    tickets = []
    for i in range(n):
        while time.perf_counter() - t0 < arr[i]:
            time.sleep(min(1e-4, max(0.0, arr[i] - (time.perf_counter() - t0))))
        sub = time.perf_counter() - t0
        t = ctx.submit(fields[kinds[i]], bs[i], xs[i], mass=float(masses[i]), tol=tol, precision=precision)
        tickets.append((t, arr[i], sub))
    lat, ok = [], 0
    for t, a, sub in tickets:
        info = ctx.wait(t)
        ctx.release(t)
        lat.append(sub - a + info["seconds"])
        ok += info["status"] == 0 and info["true_rel_resid"] <= tol
    return np.array(lat), ok, time.perf_counter() - t0


def serving_sources(ctx, fields, kinds):
    """One Gaussian source per request, drawn on the device from a generator
    seeded 10000 + i, and a zero solution buffer."""
    import torch

    gen = torch.Generator(device="cuda")
    bs, xs = [], []
    for i, k in enumerate(kinds):
        f = fields[k]
        gen.manual_seed(10000 + i)
        shape = (2, 3, f.volume // 2)
        bs.append(torch.complex(torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64),
                                torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64)))
        xs.append(ctx.new_fermion(f))
    torch.cuda.synchronize()
    return bs, xs


def stage(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def run_default(args):
    from paper_1311_2719_amd import inputs

    c3_dims, c3_m, tol = (32, 32, 32, 32), 0.01, 1e-10
    c2_dims, c2_m = (16, 16, 16, 16), 0.05
    c4_dims, n4 = (24, 24, 24, 24), 12
    serve_specs = [((8, 8, 8, 8), 105), ((16, 16, 16, 16), 106), ((24, 24, 24, 24), 107), ((32, 32, 32, 32), 108)]
    stage("generating inputs")
    specs = {"c3": ("smooth", c3_dims, 0.5, 103), "c3_b": ("source", c3_dims, 0.0, 203),
             "c2": ("smooth", c2_dims, 0.3, 102), "c2_b": ("source", c2_dims, 0.0, 202),
             "c4": ("smooth", c4_dims, 0.5, 104)}
    for i in range(n4):
        specs["c4_b%d" % i] = ("source", c4_dims, 0.0, 2040 + i)
    if not args.no_serve:
        for dims, seed in serve_specs:
            specs["s%d" % dims[0]] = ("smooth", dims, 0.5, seed)
    if not args.no_cold:
        for i in range(8):
            specs["cold%d" % i] = ("smooth", c2_dims, 0.3, 500 + i)
            specs["cold_b%d" % i] = ("source", c2_dims, 0.0, 600 + i)
    t_gen = time.perf_counter()
    host = generate(specs)
    t_gen = time.perf_counter() - t_gen

    import torch

    from paper_1311_2719_amd import binding

    ctx = binding.Context(device=0, arena_bytes=40 << 30)
    V3 = int(np.prod(c3_dims))
    f3 = ctx.set_gauge(c3_dims, host["c3"])
    b3 = ctx.pack(f3, host["c3_b"])
    x3 = ctx.new_fermion(f3)
    torch.cuda.synchronize()

    # ---- the headline: FP64 solves of the 32^4 system -------------------------------
    stage("FP64 CG %s warmup %d steps %d" % (c3_dims, args.warmup, args.steps))
    secs, infos = timed_solves(ctx, f3, b3, x3, args.steps, args.warmup, mass=c3_m, tol=tol)
    fp64_rate = args.steps / secs
    info = infos[-1]
    if any(i["status"] != 0 or i["true_rel_resid"] > tol for i in infos):
        raise SystemExit("FP64 solve failed: %s" % infos)
    rows3 = ctx.link_rows(f3)
    iters = max(info["iters_parity"])
    cg_iter = {"bytes_per_iteration": cg_bytes_per_half_site(rows3) * V3, "iterations": info["iters_parity"],
               "us_per_iteration": secs / args.steps / iters * 1e6,
               "note": "both parity systems per iteration; whole solve time (incl. the FP64 residual checks and "
                       "epoch boundaries) over the larger parity's iteration count"}
    cg_iter["gbs"] = cg_iter["bytes_per_iteration"] / (cg_iter["us_per_iteration"] * 1e-6) / 1e9
    cg_iter["frac"] = cg_iter["gbs"] / HBM_PEAK_GBS

    mixed = {}
    if not args.no_mixed:
        for name, prec in (("fp32_ru", binding.FP32_RU), ("fp16_ru", binding.FP16_RU)):
            stage("%s CG %s" % (name, c3_dims))
            s2, inf2 = timed_solves(ctx, f3, b3, x3, max(3, args.steps // 2), 1, mass=c3_m, tol=tol, precision=prec)
            rate = len(inf2) / s2
            mixed[name] = {"solves_per_s": rate, "ratio_vs_fp64": rate / fp64_rate, "iters": inf2[-1]["iters_parity"],
                           "reliable_updates": inf2[-1]["reliable_updates"],
                           "true_rel_resid": inf2[-1]["true_rel_resid"],
                           "ok": all(i["status"] == 0 and i["true_rel_resid"] <= tol for i in inf2)}

    # the same FP64 solves with the source from and the solution to pinned host memory
    stage("FP64 CG with host transfers")
    b_host = torch.empty(b3.shape, dtype=b3.dtype, pin_memory=True)
    b_host.copy_(b3.cpu())
    x_host = torch.empty(x3.shape, dtype=x3.dtype, pin_memory=True)
    n_pcie = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_pcie):
        b3.copy_(b_host)
        torch.cuda.synchronize()
        ctx.cg_solve(f3, b3, x3, mass=c3_m, tol=tol)
        x_host.copy_(x3)
    torch.cuda.synchronize()
    pcie = {"solves_per_s": n_pcie / (time.perf_counter() - t0), "solves": n_pcie,
            "bytes_each_way": int(b3.numel() * b3.element_size()),
            "what": "source copied from pinned host memory, solve, solution copied back, per solve"}

    # ---- roofline: the FP64 D_slash on the same 32^4 field ---------------------------
    stage("D_slash 32^4 x%d" % args.dslash_reps)
    durs, mean = dslash_timing(ctx, f3, b3, args.dslash_reps)
    algo_bytes = dslash_bytes_per_site(rows3) * V3
    achieved = algo_bytes / mean / 1e9
    tune = ctx.tune_info(f3)
    stage("D_slash 32^4, one share of 16")
    n_share = V3 // 16
    d, smean = dslash_timing(ctx, f3, b3, 50, out_parity=binding.ODD, offset=0, count=n_share)
    shard = {"lattice": list(c3_dims), "out_parity": "odd", "sites": n_share, "mean_us": smean * 1e6,
             "p99_us": float(np.percentile(d, 99) * 1e6),
             "gbs": dslash_bytes_per_site(rows3) * n_share / smean / 1e9}

    cpu = None
    if not args.no_cpu:
        stage("CPU oracle baseline (one 32^4 solve)")
        cpu = cpu_baseline(c3_dims, host["c3"], host["c3_b"], c3_m, tol, iters, max_seconds=args.cpu_seconds)
    ctx.free_gauge(f3)
    del b3, x3, b_host, x_host

    # ---- the 16^4 workload: FP64 solves; D_slash in cache and cold ------------------
    stage("16^4 workload")
    V2 = int(np.prod(c2_dims))
    f2 = ctx.set_gauge(c2_dims, host["c2"])
    b2 = ctx.pack(f2, host["c2_b"])
    x2 = ctx.new_fermion(f2)
    s16, i16 = timed_solves(ctx, f2, b2, x2, max(5, args.steps), 2, mass=c2_m, tol=tol)
    rows2 = ctx.link_rows(f2)
    d16, m16 = dslash_timing(ctx, f2, b2, args.dslash_reps)
    c2 = {"fp64_solves_per_s": len(i16) / s16, "iters": i16[-1]["iters_parity"],
          "ok": all(i["status"] == 0 and i["true_rel_resid"] <= tol for i in i16),
          "dslash_cached": {"mean_us": m16 * 1e6, "p50_us": float(np.percentile(d16, 50) * 1e6),
                            "p99_us": float(np.percentile(d16, 99) * 1e6),
                            "gbs": dslash_bytes_per_site(rows2) * V2 / m16 / 1e9,
                            "frac": dslash_bytes_per_site(rows2) * V2 / m16 / 1e9 / HBM_PEAK_GBS,
                            "note": "working set (about 60 MB) resident in the 256 MB Infinity Cache: not HBM"}}
    ctx.free_gauge(f2)
    if not args.no_cold:
        fields, ins, outs = [], [], []
        for i in range(8):
            fc = ctx.set_gauge(c2_dims, host["cold%d" % i])
            fields.append(fc)
            ins.append(ctx.pack(fc, host["cold_b%d" % i]))
            outs.append(ctx.new_fermion(fc))
        cmean = dslash_cycle(ctx, fields, ins, outs, 80)
        c2["dslash_cold"] = {"fields": 8, "mean_us": cmean * 1e6, "gbs": dslash_bytes_per_site(rows2) * V2 / cmean / 1e9,
                             "frac": dslash_bytes_per_site(rows2) * V2 / cmean / 1e9 / HBM_PEAK_GBS}
        for fc in fields:
            ctx.free_gauge(fc)
        del ins, outs

    # ---- 24^4, twelve sources: FP64 one by one against the batched mixed solves ------
    stage("24^4 batch of %d" % n4)
    masses = inputs.masses_uniform(0.01, 0.2, n4)
    f4 = ctx.set_gauge(c4_dims, host["c4"])
    bs4 = [ctx.pack(f4, host["c4_b%d" % i]) for i in range(n4)]
    xs4 = [ctx.new_fermion(f4) for _ in range(n4)]
    torch.cuda.synchronize()
    ctx.cg_solve(f4, bs4[0], xs4[0], mass=float(masses[0]), tol=tol)  # tuning
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it64 = [ctx.cg_solve(f4, bs4[i], xs4[i], mass=float(masses[i]), tol=tol)["iters"] for i in range(n4)]
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    batch = {"fp64_one_by_one": {"solves_per_s": n4 / t64, "seconds": t64, "iters": it64}}
    for name, prec in (("fp32_ru_batched", binding.FP32_RU), ("fp16_ru_batched", binding.FP16_RU)):
        plist = [binding.params(float(mm), tol=tol, precision=prec) for mm in masses]
        ctx.cg_solve_batch(f4, bs4, xs4, plist)  # warm-up and tuning
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            binfos = ctx.cg_solve_batch(f4, bs4, xs4, plist)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        batch[name] = {"solves_per_s": n4 / tb, "seconds": tb, "ratio_vs_fp64_one_by_one": t64 / tb,
                       "iters": [i["iters"] for i in binfos],
                       "true_rel_resid_max": max(i["true_rel_resid"] for i in binfos),
                       "ok": all(i["status"] == 0 and i["true_rel_resid"] <= tol for i in binfos),
                       "cg_shape": ctx.cg_tune_info(f4, precision=prec, nrhs=n4)}
    ctx.free_gauge(f4)
    del bs4, xs4

    # ---- serving: four resident fields, Poisson arrivals at half the saturation rate --
    serve = None
    if not args.no_serve:
        stage("serving")
        nreq = args.serve_requests
        sctx = binding.Context(device=0, arena_bytes=32 << 30)
        sctx.serve_config(slots_per_field=16, epoch_iters=16, queue_capacity=max(4096, nreq))
        fields = [sctx.set_gauge(dims, host["s%d" % dims[0]]) for dims, _ in serve_specs]
        rng = np.random.default_rng(305)
        kinds = rng.integers(0, len(fields), nreq)
        smass = np.exp(rng.uniform(np.log(0.01), np.log(0.2), nreq))
        sb, sx = serving_sources(sctx, fields, kinds)
        serve_stream(sctx, fields, kinds, smass, sb, sx, np.inf, min(nreq, 32), rng, binding.FP32_RU)  # warm-up
        lat, ok, wall = serve_stream(sctx, fields, kinds, smass, sb, sx, np.inf, nreq, rng, binding.FP32_RU)
        sat = nreq / wall
        rate = args.serve_load * sat
        stage("serving at load %.2f" % args.serve_load)
        lat, ok2, wall2 = serve_stream(sctx, fields, kinds, smass, sb, sx, rate, nreq, rng, binding.FP32_RU)
        per = {}
        for k, (dims, _) in enumerate(serve_specs):
            lk = lat[kinds[:nreq] == k]
            if lk.size:
                per["%d^4" % dims[0]] = {"requests": int(lk.size), "p50_s": float(np.percentile(lk, 50)),
                                         "p99_s": float(np.percentile(lk, 99))}
        serve = {"requests": nreq, "precision": "fp32_ru", "saturation_solves_per_s": sat, "load": args.serve_load,
                 "arrival_rate_per_s": rate, "solves_per_s": nreq / wall2, "p50_s": float(np.percentile(lat, 50)),
                 "p99_s": float(np.percentile(lat, 99)), "per_lattice": per, "ok": int(ok2), "ok_saturation": int(ok),
                 "latency": "completion - scheduled Poisson arrival; sources pre-staged on the device"}
        sctx.close()

    line = {
        "metric": METRIC,
        "value": fp64_rate,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "staggered CG, 32^4, proj_SU3(exp(0.5iH)) links seed 103, Gaussian source seed 203, "
                               "m=0.01, FP64 to true residual 1e-10, both parities",
                   "lattice": list(c3_dims), "mass": c3_m, "tol": tol, "precision": "fp64", "parity": "all"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(V3),
                     "kernel": "k_dslash<PrecF64NT> (full lattice, FP64 with non-temporal link loads, 32^4 on the same field)",
                     "algorithmic_bytes_per_launch": algo_bytes, "bytes_per_site": dslash_bytes_per_site(rows3),
                     "link_rows": rows3, "mean_us": mean * 1e6, "p50_us": float(np.percentile(durs, 50) * 1e6),
                     "p99_us": float(np.percentile(durs, 99) * 1e6), "config": tune,
                     "timing": "mean_us: median over 5 runs of %d back-to-back launches under one event pair; "
                               "p50/p99: an event pair around each launch" % len(durs)},
        "solve": {"iters": info["iters_parity"], "reliable_updates": info["reliable_updates"],
                  "true_rel_resid": info["true_rel_resid"]},
        "mixed": mixed,
        "cg_iteration": cg_iter,
        "pcie_inclusive": pcie,
        "dslash_32_share": shard,
        "c2_16": c2,
        "batch24": batch,
        "serve": serve,
        "inputs_seconds": t_gen,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def dslash_cycle(ctx, fields, ins, outs, reps):
    """Mean duration (s) of a full-lattice FP64 D_slash when consecutive
    launches cycle over distinct fields and sources."""
    import torch

    n = len(fields)
    for i in range(2 * n):
        ctx.dslash(fields[i % n], ins[i % n], outs[i % n])
    torch.cuda.synchronize()
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record(ctx.stream)
    for i in range(reps):
        ctx.dslash(fields[i % n], ins[i % n], outs[i % n])
    a1.record(ctx.stream)
    torch.cuda.synchronize()
    return a0.elapsed_time(a1) * 1e-3 / reps


def run_copy(args):
    """Device bandwidth ceilings with torch's own kernels on 2 GiB buffers
    (8x the Infinity Cache): a copy (read + write), a sum (read only) and a
    fill (write only), each repeated.  The copy is also the reference kernel
    whose counter readings (FETCH_SIZE / WRITE_SIZE) calibrate the conversion
    of those counters to bytes."""
    import torch

    n = 2 << 30
    a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    reps = max(1, args.steps)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    t_copy = timed(lambda: b.copy_(a))
    t_read = timed(lambda: a.sum())
    t_write = timed(lambda: b.fill_(2.0))
    print(json.dumps({"suite": "copy", "bytes_read_per_launch": n, "bytes_written_per_launch": n, "launches": reps,
                      "mean_us": t_copy * 1e6, "gbs_read_plus_write": 2 * n / t_copy / 1e9,
                      "read_only_gbs": n / t_read / 1e9, "write_only_gbs": n / t_write / 1e9,
                      "kernels": "torch copy_, sum, fill_ on float64 buffers of 2 GiB"}), flush=True)


def run_md(args):
    """Molecular dynamics around the solve: one leapfrog trajectory on a 16^4
    field (links proj_SU3(exp(0.3 i H)) seed 102, momenta seed 702, Gaussian
    chi seed 703; beta 5.6, m 0.05, 10 steps of 0.02) with FP64 and with FP32
    reliable-update force solves; the fermion and gauge force kernels timed
    alone (accumulating into the momenta, as the trajectory uses them)."""
    import torch

    from paper_1311_2719_amd import binding, inputs

    dims, beta, m, eps, n = (16, 16, 16, 16), 5.6, 0.05, 0.02, 10
    V = int(np.prod(dims))
    U = inputs.smooth_su3(dims, 0.3, 102)
    Q = inputs.gaussian_momenta(dims, 702)
    ctx = binding.Context(device=0, arena_bytes=8 << 30)
    f = ctx.set_gauge(dims, U)
    phi = ctx.pseudofermion(f, ctx.pack(f, inputs.gaussian_source(dims, 703)), m)
    res = {}
    for name, prec in (("fp64", binding.FP64), ("fp32_ru", binding.FP32_RU)):
        Ud = torch.from_numpy(U).cuda()
        Qd = torch.from_numpy(Q).cuda()
        stage("md: trajectory %s" % name)
        info = ctx.md_trajectory(dims, Ud, Qd, phi, beta, m, eps, n, tol=1e-10, precision=prec)
        res[name] = {"seconds": info["seconds"], "delta_h": info["delta_h"], "cg_iters": info["cg_iters"],
                     "solves": info["solves"], "kinetic": info["kinetic"], "gauge_action": info["gauge_action"],
                     "fermion_action": info["fermion_action"]}
    # the force kernels alone
    x = ctx.new_fermion(f)
    y = ctx.new_fermion(f)
    ctx.cg_solve(f, phi, x, y=y, mass=m, parity=binding.EVEN)
    w = x.clone()
    w[1] = y[1]
    Ud = torch.from_numpy(U).cuda()
    Qd = torch.from_numpy(Q).cuda()

    def timed(fn, reps=50):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            fn()
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    tf = timed(lambda: ctx.fermion_force(f, w, force=Qd, coeff=1e-9, accumulate=True))
    tg = timed(lambda: ctx.gauge_force(dims, Ud, beta, force=Qd, coeff=1e-9, accumulate=True))
    rows = ctx.link_rows(f)
    fbytes = 4 * 3 * rows * 16 + 48 + 48 + 2 * 4 * 144  # links, W here and at the neighbours, momenta read + written
    res["fermion_force"] = {"mean_us": tf * 1e6, "bytes_per_site": fbytes, "gbs": fbytes * V / tf / 1e9,
                            "frac": fbytes * V / tf / 1e9 / HBM_PEAK_GBS,
                            "note": "working set about 0.2 GB at 16^4, partly Infinity-Cache resident"}
    res["gauge_force"] = {"mean_us": tg * 1e6, "links": 4 * V}
    ctx.free_gauge(f)
    # the fermion force on the 32^4 workload's field (off the Infinity Cache:
    # links 0.6 GB, momenta 0.6 GB); W a Gaussian field, the kernel's work
    # does not depend on the values
    dims3 = (32, 32, 32, 32)
    V3 = int(np.prod(dims3))
    stage("md: fermion force 32^4")
    f3 = ctx.set_gauge(dims3, inputs.smooth_su3(dims3, 0.5, 103))
    w3 = ctx.pack(f3, inputs.gaussian_source(dims3, 203))
    Q3 = torch.zeros((V3, 4, 3, 3), dtype=torch.complex128, device="cuda")
    tf3 = timed(lambda: ctx.fermion_force(f3, w3, force=Q3, coeff=1e-9, accumulate=True), reps=20)
    fbytes3 = 4 * 3 * ctx.link_rows(f3) * 16 + 48 + 48 + 2 * 4 * 144
    res["fermion_force_32"] = {"mean_us": tf3 * 1e6, "bytes_per_site": fbytes3, "gbs": fbytes3 * V3 / tf3 / 1e9,
                               "frac": fbytes3 * V3 / tf3 / 1e9 / HBM_PEAK_GBS}
    ctx.close()
    _emit({"suite": "md", "workload": "16^4 eps 0.3 links seed 102, momenta seed 702, chi seed 703, beta 5.6, "
                                      "m 0.05, leapfrog 10 x 0.02, CG 1e-10; force kernel also at 32^4 "
                                      "(eps 0.5 links seed 103)", "results": res})


def run_kernels32(args):
    """The 32^4 workload's kernels for profilers: the FP64 D_slash
    (args.dslash_reps launches) and one solve in each precision."""
    import torch

    from paper_1311_2719_amd import binding, inputs

    dims, m = (32, 32, 32, 32), 0.01
    stage("kernels32: links")
    U = inputs.smooth_su3(dims, 0.5, 103)
    ctx = binding.Context(device=0, arena_bytes=16 << 30)
    f = ctx.set_gauge(dims, U)
    del U
    b = ctx.pack(f, inputs.gaussian_source(dims, 203))
    x = ctx.new_fermion(f)
    out = ctx.new_fermion(f)
    ctx.dslash(f, b, out)  # tuning
    torch.cuda.synchronize()
    stage("kernels32: D_slash x%d" % args.dslash_reps)
    for _ in range(args.dslash_reps):
        ctx.dslash(f, b, out)
    torch.cuda.synchronize()
    res = {}
    for name, prec in (("fp64", binding.FP64), ("fp32_ru", binding.FP32_RU), ("fp16_ru", binding.FP16_RU)):
        stage("kernels32: %s solve" % name)
        ctx.cg_solve(f, b, x, mass=m, precision=prec)  # tuning
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.cg_solve(f, b, x, mass=m, precision=prec)
        res[name] = {"seconds": time.perf_counter() - t0, "iters": info["iters_parity"],
                     "cg_shape": ctx.cg_tune_info(f, precision=prec, nrhs=1)}
    res["dslash_config"] = ctx.tune_info(f)
    ctx.close()
    _emit({"suite": "kernels32", "results": res})


def _emit(d):
    print(json.dumps(d), flush=True)


def run_mixed32(args):
    """32^4 (proj_SU3(exp(0.5 i H)), seed 103; source seed 203; m = 0.01):
    FP64, FP32 and FP16 reliable-update solves to true residual 1e-10."""
    import torch

    from paper_1311_2719_amd import binding, inputs

    dims, m, tol = (32, 32, 32, 32), 0.01, 1e-10
    print("bench mixed32: generating links", file=sys.stderr, flush=True)
    U = inputs.smooth_su3(dims, 0.5, seed=103)
    ctx = binding.Context(device=0, arena_bytes=12 << 30)
    f = ctx.set_gauge(dims, U)
    del U
    b = ctx.pack(f, inputs.gaussian_source(dims, seed=203))
    x = ctx.new_fermion(f)
    torch.cuda.synchronize()
    res = {}
    for name, prec in (("fp64", binding.FP64), ("fp32_ru", binding.FP32_RU), ("fp16_ru", binding.FP16_RU)):
        print("bench mixed32: %s" % name, file=sys.stderr, flush=True)
        secs, infos = timed_solves(ctx, f, b, x, max(1, args.steps // 5), 1, mass=m, tol=tol, precision=prec)
        i = infos[-1]
        res[name] = {"solves_per_s": len(infos) / secs, "seconds_per_solve": secs / len(infos), "iters": i["iters"],
                     "reliable_updates": i["reliable_updates"], "true_rel_resid": i["true_rel_resid"],
                     "ok": all(v["status"] == 0 and v["true_rel_resid"] <= tol for v in infos)}
    for k in ("fp32_ru", "fp16_ru"):
        res[k]["ratio_vs_fp64"] = res[k]["solves_per_s"] / res["fp64"]["solves_per_s"]
    ctx.close()
    _emit({"suite": "mixed32", "workload": "staggered CG 32^4, eps=0.5 links seed 103, source seed 203, m=0.01, "
                                           "true residual 1e-10, both parities", "results": res})


def run_batch24(args):
    """24^4 (eps = 0.5, seed 104), 12 sources (seeds 2040..2051), masses
    evenly in [0.01, 0.2]: one batched FP32 reliable-update solve of all 12
    (links read once per sweep for the whole batch) against the same 12
    systems solved one at a time in plain FP64."""
    import torch

    from paper_1311_2719_amd import binding, inputs

    dims, tol, n = (24, 24, 24, 24), 1e-10, 12
    print("bench batch24: generating links", file=sys.stderr, flush=True)
    U = inputs.smooth_su3(dims, 0.5, seed=104)
    masses = inputs.masses_uniform(0.01, 0.2, n)
    ctx = binding.Context(device=0, arena_bytes=12 << 30)
    f = ctx.set_gauge(dims, U)
    del U
    bs = [ctx.pack(f, inputs.gaussian_source(dims, seed=2040 + i)) for i in range(n)]
    xs = [ctx.new_fermion(f) for _ in range(n)]
    torch.cuda.synchronize()
    out = {}
    # FP64 one by one
    print("bench batch24: fp64 one at a time", file=sys.stderr, flush=True)
    for i in range(n):  # warm-up and tuning
        ctx.cg_solve(f, bs[i], xs[i], mass=float(masses[i]), tol=tol)
        break
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it64 = []
    for i in range(n):
        info = ctx.cg_solve(f, bs[i], xs[i], mass=float(masses[i]), tol=tol)
        it64.append(info["iters"])
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    out["fp64_single"] = {"solves_per_s": n / t64, "seconds": t64, "iters": it64}
    for name, prec in (("fp32_ru_batched", binding.FP32_RU), ("fp16_ru_batched", binding.FP16_RU),
                       ("fp64_batched", binding.FP64)):
        print("bench batch24: %s" % name, file=sys.stderr, flush=True)
        plist = [binding.params(float(mm), tol=tol, precision=prec) for mm in masses]
        ctx.cg_solve_batch(f, bs, xs, plist)  # warm-up and tuning
        torch.cuda.synchronize()
        reps = max(1, args.steps // 5)
        t0 = time.perf_counter()
        for _ in range(reps):
            infos = ctx.cg_solve_batch(f, bs, xs, plist)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        out[name] = {"solves_per_s": n / tb, "seconds": tb, "ratio_vs_fp64_single": (n / tb) / (n / t64),
                     "iters": [i["iters"] for i in infos], "true_rel_resid_max": max(i["true_rel_resid"] for i in infos),
                     "ok": all(i["status"] == 0 and i["true_rel_resid"] <= tol for i in infos),
                     "cg_shape": ctx.cg_tune_info(f, precision=prec, nrhs=n)}
    ctx.close()
    _emit({"suite": "batch24", "workload": "24^4, eps=0.5 links seed 104, 12 sources seeds 2040-2051, "
                                           "m = linspace(0.01, 0.2, 12), true residual 1e-10", "results": out})


def run_serve(args):
    """Serving stream: 4 resident fields 8^4, 16^4, 24^4, 32^4 (eps = 0.5,
    seeds 105..108); requests with Poisson arrivals, lattice uniform over the
    four, mass log-uniform in [0.01, 0.2], Gaussian source, FP32 reliable
    updates to 1e-10.  The arrival rate is swept as a fraction of the measured
    saturation throughput; latency = completion - scheduled arrival."""
    import torch

    from paper_1311_2719_amd import binding, inputs

    specs = [((8, 8, 8, 8), 105), ((16, 16, 16, 16), 106), ((24, 24, 24, 24), 107), ((32, 32, 32, 32), 108)]
    nreq = args.serve_requests
    ctx = binding.Context(device=0, arena_bytes=64 << 30)
    ctx.serve_config(slots_per_field=16, epoch_iters=16, queue_capacity=max(4096, nreq))
    fields = []
    for dims, seed in specs:
        print("bench serve: field %s" % (dims,), file=sys.stderr, flush=True)
        U = inputs.smooth_su3(dims, 0.5, seed=seed)
        fields.append(ctx.set_gauge(dims, U))
        del U
    rng = np.random.default_rng(305)
    kinds = rng.integers(0, len(fields), nreq)
    masses = np.exp(rng.uniform(np.log(0.01), np.log(0.2), nreq))
    bs, xs = serving_sources(ctx, fields, kinds)

    def point(rate):
        lat, ok, wall = serve_stream(ctx, fields, kinds, masses, bs, xs, rate, nreq, rng, binding.FP32_RU)
        per = {}
        for k, (dims, _) in enumerate(specs):
            lk = lat[kinds == k]
            if lk.size:
                per["%d^4" % dims[0]] = {"requests": int(lk.size), "p50_s": float(np.percentile(lk, 50)),
                                         "p99_s": float(np.percentile(lk, 99))}
        return {"rate_per_s": None if not np.isfinite(rate) else rate, "solves_per_s": nreq / wall,
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)), "ok": int(ok),
                "per_lattice": per}

    # warm-up (tuning, workspaces) on a few requests of each field
    serve_stream(ctx, fields, kinds, masses, bs, xs, np.inf, min(nreq, 32), rng, binding.FP32_RU)
    print("bench serve: saturation", file=sys.stderr, flush=True)
    sat_point = point(np.inf)
    sat = sat_point["solves_per_s"]
    sat_point["load"] = "saturation (all submitted at t=0)"
    points = [sat_point]
    for frac in args.serve_loads:
        print("bench serve: load %.2f" % frac, file=sys.stderr, flush=True)
        pt = point(frac * sat)
        pt["load"] = frac
        points.append(pt)
    ctx.close()
    _emit({"suite": "serve", "requests_per_point": nreq, "precision": "fp32_ru", "tol": 1e-10,
           "fields": [list(d) for d, _ in specs], "points": points})


def wilson_bytes_per_site(rows: int) -> int:
    """Wilson hop algorithmic bytes per output site (FP64): 8 links of
    3 x rows complex entries, one gathered and one written spin-colour vector."""
    return 8 * 3 * rows * 16 + 192 + 192


def run_wilson(args):
    """Wilson fermions (the paper's second workload): FP64 solves of M x = b,
    M = 1 - kappa H, by CG on the even-odd normal equations, 16^4 lattice
    (links proj_SU3(exp(0.3 i H)) seed 102, Gaussian spin-colour source seed
    202, kappa = 0.12, true residual reported); the hop H timed alone at 16^4
    and 32^4 (unit links); the oracle's solve of the same system on the host."""
    import torch

    import oracle
    from paper_1311_2719_amd import binding, inputs

    dims, kappa, tol = (16, 16, 16, 16), 0.12, 1e-10
    V = int(np.prod(dims))
    U = inputs.smooth_su3(dims, 0.3, seed=102)
    b_lex = inputs.gaussian_spinor(dims, seed=202)
    ctx = binding.Context(device=0, arena_bytes=8 << 30)
    f = ctx.set_gauge_wilson(dims, U)
    b = ctx.pack_spinor(f, b_lex)
    x = ctx.new_spinor(f)
    torch.cuda.synchronize()
    for _ in range(max(1, args.warmup)):
        ctx.wilson_solve(f, b, x, kappa, tol=tol)
    torch.cuda.synchronize()
    steps = max(1, args.steps)
    t0 = time.perf_counter()
    infos = [ctx.wilson_solve(f, b, x, kappa, tol=tol) for _ in range(steps)]
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0

    def hop_mean(field, inp, reps):
        out = ctx.new_spinor(field)
        for _ in range(5):
            ctx.wilson_dslash(field, inp, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            ctx.wilson_dslash(field, inp, out)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    rows = ctx.link_rows(f)
    h16 = hop_mean(f, b, 100)
    dims32 = (32, 32, 32, 32)
    f32 = ctx.set_gauge_wilson(dims32, inputs.unit_links(dims32))
    b32 = ctx.pack_spinor(f32, inputs.gaussian_spinor(dims32, seed=203))
    h32 = hop_mean(f32, b32, 30)
    V32 = int(np.prod(dims32))
    rows32 = ctx.link_rows(f32)
    ctx.free_gauge(f32)
    del b32
    cpu = None
    if not args.no_cpu:
        t1 = time.perf_counter()
        _, oi = oracle.wilson_cg(dims, U, kappa, b_lex, tol=tol)
        tc = time.perf_counter() - t1
        cpu = {"value": 1.0 / tc, "unit": "solves/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": "1 complete FP64 solve of the same 16x16x16x16 system (oracle iterations %d)" % oi["iters"]}
    info = infos[-1]
    ctx.close()
    _emit({"suite": "wilson", "metric": "Wilson CG solves/s to 1e-10 (FP64, even-odd)",
           "workload": "Wilson M = 1 - kappa H, 16^4, proj_SU3(exp(0.3iH)) links seed 102, Gaussian spin-colour "
                       "source seed 202, kappa = 0.12, CG on the even-odd normal equations to 1e-10",
           "value": steps / secs, "unit": "solves/s", "ms_per_solve": secs / steps * 1e3,
           "iters": info["iters"], "true_rel_resid": info["true_rel_resid"],
           "ok": all(i["status"] == 0 for i in infos),
           "hop_16": {"mean_us": h16 * 1e6, "link_rows": rows, "bytes_per_site": wilson_bytes_per_site(rows),
                      "gbs": wilson_bytes_per_site(rows) * V / h16 / 1e9,
                      "frac": wilson_bytes_per_site(rows) * V / h16 / 1e9 / HBM_PEAK_GBS},
           "hop_32": {"mean_us": h32 * 1e6, "link_rows": rows32,
                      "gbs": wilson_bytes_per_site(rows32) * V32 / h32 / 1e9,
                      "frac": wilson_bytes_per_site(rows32) * V32 / h32 / 1e9 / HBM_PEAK_GBS},
           "cpu_baseline": cpu})


def run_cpu_baseline(args):
    """The CPU oracle timed on the host cores (the baseline beside the GPU
    numbers, never a target): FP64 D_slash GB/s (1248 B per site, the
    oracle stores full links) and FP64 CG solves/s on the four workloads --
    4^4 Haar, 16^4 eps 0.3, 32^4 eps 0.5, 24^4 eps 0.5 (one of its twelve
    sources, the lightest mass) -- with all OpenMP threads, and the 4^4 and
    16^4 ones again with one thread (a child process); plus a STREAM-style
    triad as the host's own bandwidth roofline.  No GPU is used."""
    import subprocess

    import oracle
    from paper_1311_2719_amd import inputs

    if args.oracle_threads_one:
        os.environ["OMP_NUM_THREADS"] = "1"
    work = [("4^4 Haar m=0.1", (4, 4, 4, 4), lambda d: inputs.haar_su3(d, 101), 201, 0.1),
            ("16^4 eps=0.3 m=0.05", (16, 16, 16, 16), lambda d: inputs.smooth_su3(d, 0.3, 102), 202, 0.05)]
    if not args.oracle_threads_one:
        work += [("32^4 eps=0.5 m=0.01", (32, 32, 32, 32), lambda d: inputs.smooth_su3(d, 0.5, 103), 203, 0.01),
                 ("24^4 eps=0.5 m=0.01 (source 2040)", (24, 24, 24, 24), lambda d: inputs.smooth_su3(d, 0.5, 104),
                  2040, 0.01)]
    results = []
    for name, dims, links, seed, m in work:
        print("bench cpu_baseline: %s" % name, file=sys.stderr, flush=True)
        U = links(dims)
        b = inputs.gaussian_source(dims, seed)
        V = int(np.prod(dims))
        oracle.dslash(dims, U, b)
        reps, t0 = 0, time.perf_counter()
        while reps < 3 or (time.perf_counter() - t0 < 1.0 and reps < 50):
            oracle.dslash(dims, U, b)
            reps += 1
        td = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        _, _, info = oracle.cg_solve(dims, U, m, b, tol=1e-10)
        tc = time.perf_counter() - t0
        results.append({"workload": name, "dslash_us": td * 1e6, "dslash_gbs": 1248 * V / td / 1e9,
                        "cg_seconds": tc, "cg_solves_per_s": 1.0 / tc, "cg_iters": info["iters"],
                        "true_rel_resid": info["true_rel"]})
        del U, b
    line = {"suite": "cpu_baseline", "kind": "oracle", "threads": oracle.max_threads(),
            "triad_gbs": oracle.stream_triad(1 << 26) / 1e9, "host": _host_cpu(), "results": results}
    if not args.oracle_threads_one:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--suite", "cpu_baseline",
                            "--oracle-threads-one"], capture_output=True, text=True,
                           env=dict(os.environ, OMP_NUM_THREADS="1"))
        one = [json.loads(x) for x in r.stdout.splitlines() if x.startswith("{")]
        line["one_thread"] = one[0] if one else {"error": r.stderr[-500:]}
    print(json.dumps(line), flush=True)


SUITES = {"mixed32": run_mixed32, "batch24": run_batch24, "serve": run_serve, "cpu_baseline": run_cpu_baseline,
          "wilson": run_wilson, "kernels32": run_kernels32, "md": run_md}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.suite == "default":
        run_default(args)
    elif args.suite == "copy":
        run_copy(args)
    else:
        SUITES[args.suite](args)


if __name__ == "__main__":
    main()
