#!/usr/bin/env python3
"""Benchmark of the staggered CG hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--suite default|mixed32|batch24|serve]

Default workload (one JSON line): FP64 staggered CG solves of (m^2 - D^2) x = b
to relative true residual 1e-10 on a 16^4 lattice (links proj_SU3(exp(0.3 i H)),
seed 102; Gaussian source, seed 202; m = 0.05; both parities).  One step is
one complete solve on the GPU (D_slash, the fused CG kernels, the device-side
scalars and stopping test, and the FP64 true-residual check); the gauge field
and the source are resident in HBM before the timed region.  `value` is
solves/s over the K timed steps.

The same line reports:
  roofline      the FP64 D_slash kernel: 100 full-lattice applications per
                run, each bracketed by HIP events on the library's stream;
                achieved = algorithmic bytes per output site (8 links + 1
                gathered input vector + 1 output vector: 864 B with two
                stored link rows, 1248 B with three) x V / mean duration;
  mixed         FP32 and FP16 (reliable-update) solves/s on the same system;
  cpu_baseline  the FP64 CPU oracle solving the same system on the host cores.

Other suites (--suite) print their own JSON line: the 32^4 mixed-precision
solve, the 24^4 twelve-right-hand-side batched solve, and the serving stream.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_f64_16x16x16x16_traffic.txt")
KERNEL_SOURCES = ["dslash.hip", "hop.hpp", "stag_types.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1311_2719_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(volume: int):
    """HBM bytes per D_slash launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    try:
        fields = {}
        with open(TRAFFIC_FILE) as fh:
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
                    choices=["default", "mixed32", "batch24", "serve", "copy", "cpu_baseline", "wilson"])
    ap.add_argument("--oracle-threads-one", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--dslash-reps", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-dslash32", action="store_true", help="skip the 32^4 D_slash bandwidth check")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-loads", type=float, nargs="*", default=[0.25, 0.5, 0.75, 0.9, 1.0, 1.2])
    return ap.parse_args()


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


def dslash_cold(ctx, dims, copies, reps):
    """Mean duration (s) of a full-lattice FP64 D_slash when consecutive
    launches cycle over `copies` distinct fields and sources of shape dims
    (their working set exceeds the 256 MB Infinity Cache)."""
    import torch

    from paper_1311_2719_amd import inputs

    fields, ins, outs = [], [], []
    for i in range(copies):
        f = ctx.set_gauge(dims, inputs.smooth_su3(dims, 0.3, seed=500 + i))
        fields.append(f)
        ins.append(ctx.pack(f, inputs.gaussian_source(dims, seed=600 + i)))
        outs.append(ctx.new_fermion(f))
    for i in range(2 * copies):
        ctx.dslash(fields[i % copies], ins[i % copies], outs[i % copies])
    torch.cuda.synchronize()
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record(ctx.stream)
    for i in range(reps):
        ctx.dslash(fields[i % copies], ins[i % copies], outs[i % copies])
    a1.record(ctx.stream)
    torch.cuda.synchronize()
    rows = ctx.link_rows(fields[0])
    for f in fields:
        ctx.free_gauge(f)
    return a0.elapsed_time(a1) * 1e-3 / reps, rows


def cpu_baseline(dims, U, b, m, tol, gpu_iters):
    import oracle

    t0 = time.perf_counter()
    n = 0
    it = 0
    while True:
        x, _, info = oracle.cg_solve(dims, U, m, b, tol=tol)
        n += 1
        it = info["iters"]
        if time.perf_counter() - t0 > 12.0 or n >= 40:
            break
    dt = (time.perf_counter() - t0) / n
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d complete FP64 solve(s) of the same %s system (oracle iterations %d, GPU %d)"
                      % (n, "x".join(map(str, dims)), it, gpu_iters)}


def run_default(args):
    import torch

    from paper_1311_2719_amd import binding, inputs

    dims, eps, m, tol = (16, 16, 16, 16), 0.3, 0.05, 1e-10
    V = int(np.prod(dims))
    U = inputs.smooth_su3(dims, eps, seed=102)
    b_lex = inputs.gaussian_source(dims, seed=202)
    ctx = binding.Context(device=0, arena_bytes=6 << 30)
    f = ctx.set_gauge(dims, U)
    b = ctx.pack(f, b_lex)
    x = ctx.new_fermion(f)
    torch.cuda.synchronize()
    print("bench: FP64 CG %s warmup %d steps %d" % (dims, args.warmup, args.steps), file=sys.stderr, flush=True)
    secs, infos = timed_solves(ctx, f, b, x, args.steps, args.warmup, mass=m, tol=tol)
    fp64_rate = args.steps / secs
    info = infos[-1]
    if any(i["status"] != 0 or i["true_rel_resid"] > tol for i in infos):
        raise SystemExit("FP64 solve failed: %s" % infos)

    # the same solves with the source coming from and the solution going to
    # pinned host memory (PCIe both ways inside the timed region); reported
    # beside the device-resident rate, never as the value
    print("bench: FP64 CG with host transfers", file=sys.stderr, flush=True)
    b_host = torch.empty(b.shape, dtype=b.dtype, pin_memory=True)
    b_host.copy_(b.cpu())
    x_host = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
    n_pcie = max(3, args.steps // 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_pcie):
        b.copy_(b_host)
        torch.cuda.synchronize()
        ctx.cg_solve(f, b, x, mass=m, tol=tol)
        x_host.copy_(x)
    torch.cuda.synchronize()
    pcie = {"solves_per_s": n_pcie / (time.perf_counter() - t0), "solves": n_pcie,
            "bytes_each_way": int(b.numel() * b.element_size()),
            "what": "source copied from pinned host memory, solve, solution copied back, per solve"}

    print("bench: D_slash x%d" % args.dslash_reps, file=sys.stderr, flush=True)
    durs, mean = dslash_timing(ctx, f, b, args.dslash_reps)
    rows = ctx.link_rows(f)
    algo_bytes = dslash_bytes_per_site(rows) * V
    achieved = algo_bytes / mean / 1e9
    traffic = read_traffic(V)
    tune = ctx.tune_info(f)

    mixed = {}
    if not args.no_mixed:
        for name, prec in (("fp32_ru", binding.FP32_RU), ("fp16_ru", binding.FP16_RU)):
            print("bench: %s CG" % name, file=sys.stderr, flush=True)
            s2, inf2 = timed_solves(ctx, f, b, x, max(3, args.steps // 2), 1, mass=m, tol=tol, precision=prec)
            ok = all(i["status"] == 0 and i["true_rel_resid"] <= tol for i in inf2)
            rate = len(inf2) / s2
            mixed[name] = {"solves_per_s": rate, "ratio_vs_fp64": rate / fp64_rate, "iters": inf2[-1]["iters"],
                           "reliable_updates": inf2[-1]["reliable_updates"],
                           "true_rel_resid": inf2[-1]["true_rel_resid"], "ok": ok}

    d32 = cold = shard = None
    if not args.no_dslash32:
        # cold: 8 distinct 16^4 fields cycled, so consecutive launches do not
        # find their links in the Infinity Cache
        print("bench: D_slash 16^4 cold (8 fields)", file=sys.stderr, flush=True)
        cmean, crows = dslash_cold(ctx, dims, 8, 80)
        cold = {"lattice": list(dims), "fields": 8, "mean_us": cmean * 1e6,
                "gbs": dslash_bytes_per_site(crows) * V / cmean / 1e9,
                "frac": dslash_bytes_per_site(crows) * V / cmean / 1e9 / HBM_PEAK_GBS, "link_rows": crows}
        # 32^4: a working set (0.9 GB per application with two link rows) far
        # beyond the Infinity Cache, so the bandwidth here is HBM bandwidth
        print("bench: D_slash 32^4", file=sys.stderr, flush=True)
        dims32 = (32, 32, 32, 32)
        U32 = inputs.unit_links(dims32)
        f32 = ctx.set_gauge(dims32, U32)
        del U32
        b32 = ctx.pack(f32, inputs.gaussian_source(dims32, seed=203))
        d, dmean = dslash_timing(ctx, f32, b32, 50)
        V32 = int(np.prod(dims32))
        r32 = ctx.link_rows(f32)
        d32 = {"lattice": list(dims32), "mean_us": dmean * 1e6, "p99_us": float(np.percentile(d, 99) * 1e6),
               "gbs": dslash_bytes_per_site(r32) * V32 / dmean / 1e9,
               "frac": dslash_bytes_per_site(r32) * V32 / dmean / 1e9 / HBM_PEAK_GBS,
               "link_rows": r32, "config": ctx.tune_info(f32)}
        # one GPU's share of a 16-GPU split of the 32^4 operator (the paper's
        # site-range decomposition): odd-parity sites [0, V/16), full input
        print("bench: D_slash 32^4 one share of 16", file=sys.stderr, flush=True)
        n_share = V32 // 16
        d, smean = dslash_timing(ctx, f32, b32, 50, out_parity=binding.ODD, offset=0, count=n_share)
        shard = {"lattice": list(dims32), "out_parity": "odd", "sites": n_share, "mean_us": smean * 1e6,
                 "p99_us": float(np.percentile(d, 99) * 1e6),
                 "gbs": dslash_bytes_per_site(r32) * n_share / smean / 1e9}
        ctx.free_gauge(f32)
        del b32

    cpu = None
    if not args.no_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(dims, U, b_lex, m, tol, info["iters"])

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
        "config": {"workload": "staggered CG, 16^4, proj_SU3(exp(0.3iH)) links seed 102, Gaussian source seed 202, "
                               "m=0.05, FP64 to true residual 1e-10, both parities",
                   "lattice": list(dims), "mass": m, "tol": tol, "precision": "fp64", "parity": "all"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_dslash64 (full lattice, FP64)", "algorithmic_bytes_per_launch": algo_bytes,
                     "bytes_per_site": dslash_bytes_per_site(rows), "link_rows": rows, "mean_us": mean * 1e6},
        "dslash": {"p50_us": float(np.percentile(durs, 50) * 1e6), "p99_us": float(np.percentile(durs, 99) * 1e6),
                   "mean_event_pair_us": float(durs.mean() * 1e6), "launches": int(len(durs)), "config": tune,
                   "timing": "mean_us: median over 5 runs of %d back-to-back launches under one event pair; p50/p99: "
                             "an event pair around each launch" % len(durs)},
        "solve": {"iters": info["iters"], "reliable_updates": info["reliable_updates"],
                  "true_rel_resid": info["true_rel_resid"]},
        "mixed": mixed,
        "pcie_inclusive": pcie,
        "dslash_16_cold": cold,
        "dslash_32": d32,
        "dslash_32_share": shard,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def run_copy(args):
    """A plain device-to-device copy of 512 MiB, repeated: the reference
    kernel whose counter readings (FETCH_SIZE / WRITE_SIZE) calibrate the
    conversion of those counters to HBM bytes."""
    import torch

    n = 512 << 20
    a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    print(json.dumps({"suite": "copy", "bytes_read_per_launch": n, "bytes_written_per_launch": n,
                      "launches": reps, "mean_us": sec * 1e6, "gbs_read_plus_write": 2 * n / sec / 1e9}), flush=True)


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
    # sources drawn on the device from a seeded generator, one per request
    gen = torch.Generator(device="cuda")
    bs, xs = [], []
    for i in range(nreq):
        f = fields[kinds[i]]
        gen.manual_seed(10000 + i)
        b = torch.complex(torch.randn((2, 3, f.volume // 2), generator=gen, device="cuda", dtype=torch.float64),
                          torch.randn((2, 3, f.volume // 2), generator=gen, device="cuda", dtype=torch.float64))
        bs.append(b)
        xs.append(ctx.new_fermion(f))
    torch.cuda.synchronize()

    def run_stream(rate, n):
        """Submit n requests at Poisson times (rate per s; inf = all at once)."""
        arr = np.cumsum(rng.exponential(1.0 / rate, n)) if np.isfinite(rate) else np.zeros(n)
        t0 = time.perf_counter()
        tickets = []
        for i in range(n):
            while time.perf_counter() - t0 < arr[i]:
                time.sleep(min(1e-4, max(0.0, arr[i] - (time.perf_counter() - t0))))
            sub = time.perf_counter() - t0
            t = ctx.submit(fields[kinds[i]], bs[i], xs[i], mass=float(masses[i]), tol=1e-10,
                           precision=binding.FP32_RU)
            tickets.append((t, arr[i], sub))
        lat, ok = [], 0
        for t, a, sub in tickets:
            info = ctx.wait(t)
            ctx.release(t)
            lat.append(sub - a + info["seconds"])
            ok += info["status"] == 0 and info["true_rel_resid"] <= 1e-10
        wall = time.perf_counter() - t0
        return np.array(lat), ok, wall

    # warm-up (tuning, workspaces) on a few requests of each field
    run_stream(np.inf, min(nreq, 32))
    print("bench serve: saturation", file=sys.stderr, flush=True)
    lat, ok, wall = run_stream(np.inf, nreq)
    sat = nreq / wall
    points = [{"load": "saturation (all submitted at t=0)", "rate_per_s": None, "solves_per_s": sat,
               "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)), "ok": int(ok)}]
    for frac in args.serve_loads:
        rate = frac * sat
        print("bench serve: load %.2f" % frac, file=sys.stderr, flush=True)
        lat, ok, wall = run_stream(rate, nreq)
        points.append({"load": frac, "rate_per_s": rate, "solves_per_s": nreq / wall,
                       "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                       "ok": int(ok)})
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


def _host_cpu():
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
    return info


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
          "wilson": run_wilson}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
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
