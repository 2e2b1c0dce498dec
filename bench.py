#!/usr/bin/env python3
"""Injection throughput of the batched incremental path versus the plain
one-render-per-injection path, on one GPU.

Workload: the scaling-sweep scene at its large size (N = 134,826 Gaussians,
SH degree 3, 800 x 800, 16 x 16 tiles), parameters stored as fp32 (or
--fmt f16/bf16), 5,000 single-bit sites per field (bit j mod width, every
field), B = 32 variants per launch.  A step is four B-variant batches on
every campaign stream (global_batch = 4 x B x streams injections): each batch
stages its corrupted variants, projects their corrupted primitives, lists and
re-composites their dirty tiles and reduces their PSNR/footprint records.
The K timed steps run as one sg_campaign call.  The clean scene, its tile
lists and its clean frame are resident (prepared once, outside the timed
region).

Prints one JSON line.  `value` is batched injections/s; `plain` holds the
plain path (sg_inject + sg_render + sg_restore + metric readback per
injection) on the same GPU; `roofline` is the compositing launches' fp32
arithmetic rate (20 flops per pixel-primitive evaluation) against the fp32
vector peak; `cpu_baseline` is the FP64 oracle's plain path on the host.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

# Hardware queues the HIP runtime spreads streams over (read once, when the
# runtime starts).  Batches of a campaign are chains of short launches whose
# throughput comes from running many of them concurrently; HIP's default of 4
# queues caps that at four chains.  Each queue runs its launches one after
# another, so the campaign rate rises with the queue count (2.2 M injections/s
# at 8 queues, 3.1 M at 16, 3.3 M at 18) up to 23 queues and collapses at 24
# (1.6 M).  18 keeps a margin below that edge.
HW_QUEUES = 18
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < HW_QUEUES:
    os.environ["GPU_MAX_HW_QUEUES"] = str(HW_QUEUES)

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_HI = 134_826
FLOPS_PER_EVAL = 20            # q-form and alpha test of one pixel-primitive evaluation
FP32_PEAK_TFLOPS = 157.3       # MI355X fp32 vector peak
PERSIST_RESUME = 16            # checkpoint spacing of the persistent engine's prepared view
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "campaign_step_w2hi_f32_b32_hbm_traffic.txt")
# the sources the campaign step kernel is compiled from
STEP_SOURCES = ("k_composite.hip", "sg_batch.h", "sg_device.h", "sg_kernels.h", "sg_types.h")
DIRTY_BINS = [0, 1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096]
PAPER_CONTEXT = {"inj_per_s": 2515, "hardware": "Blackwell-generation GPU (model not named), B=32, resolution not stated",
                 "l40s_inj_per_s": 1522}


def step_sources_sha():
    """sha256 over the campaign step kernel's sources, in STEP_SOURCES order."""
    import hashlib
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2606_21791_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def _measured_traffic(resume=None):
    """HBM bytes per campaign step launch from the committed counter summary,
    valid only while the kernel's sources are the ones that were measured.
    The summary holds one figure per checkpoint spacing it was measured at
    (lines "traffic_bytes_per_launch[resume=G]: bytes"); resume=None returns
    all of them as {G: bytes}, an int returns that spacing's figure or None."""
    try:
        txt = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    sha = None
    figs = {}
    for line in txt.splitlines():
        line = line.strip()
        if line.startswith("sources sha256 at measurement:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes_per_launch[resume="):
            key, val = line.split(":", 1)
            figs[int(key[len("traffic_bytes_per_launch[resume="):-1])] = int(val)
    if sha != step_sources_sha() or not figs:
        return None
    return figs if resume is None else figs.get(int(resume))


def _workload(fmt):
    from paper_2606_21791_amd import synth
    sc = synth.make_scene(N_HI, seed=3, sh_degree=3)
    cam = synth.make_camera(800, 800)
    W = 32 if fmt == "f32" else 16
    sites = synth.make_sites_stratified(N_HI, 3, 5000, seed=12 + {"f32": 0, "f16": 1, "bf16": 2}[fmt], width_bits=W)
    order = np.random.default_rng(99).permutation(len(sites))
    return sc, cam, sites.take(order)


_CPU = {}   # inputs of the oracle baseline, shared with forked workers


def _cpu_one(k):
    """One oracle injection of the plain path on the whole frame: FP64
    projection of every primitive, compositing of all 800 x 800 pixels and
    the metrics against the clean frame.  Returns (projection seconds,
    compositing and metrics seconds)."""
    from threadpoolctl import threadpool_limits
    from oracle import formats, metrics as om, render as orender
    d = _CPU
    with threadpool_limits(limits=1):
        w = [x.copy() for x in d["words"]]
        st = d["sites"]
        f, c, p, b = int(st.field[k]), int(st.comp[k]), int(st.prim[k]), int(st.bit[k])
        w[f][c, p] = formats.flip(w[f][c, p:p + 1], b)[0]
        t0 = time.perf_counter()
        pr = orender.project(orender.decode_scene(w, d["fmt"]), 3, d["cam"])
        t1 = time.perf_counter()
        out = orender.render(pr, d["cam"])
        om.frame_metrics(out["image"], d["clean"], out["nonfinite"])
        t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def cpu_baseline(sc, cam, sites, fmt, procs):
    """The oracle's plain path timed on the host on a bounded sample: `procs`
    single-bit injections of the headline workload, each a full-frame FP64
    render of the corrupted scene with its metrics, run at once in forked
    worker processes of one thread each (the clean frame is rendered once
    beforehand).  The value is the all-process rate; the single-thread rate
    is the mean time of one injection.  Runs before the GPU is touched, so the
    workers fork from a process without a device context."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import formats, render as orender
    with threadpool_limits(limits=1):
        words = [formats.store(f, fmt) for f in sc.fields]
        t0 = time.perf_counter()
        clean = orender.render(orender.project(orender.decode_scene(words, fmt), 3, cam), cam)["image"]
        t_clean = time.perf_counter() - t0
    _CPU.update(words=words, sites=sites, fmt=fmt, cam=cam, clean=clean)
    with mp.get_context("fork").Pool(procs) as pool:
        t0 = time.perf_counter()
        many = pool.map(_cpu_one, range(procs), chunksize=1)
        wall = time.perf_counter() - t0
    per = [a + b for a, b in many]
    mean_one = float(np.mean(per))
    res = {"unit": "injections/s", "kind": "oracle", "value": procs / wall, "cores": procs,
           "single_thread_value": 1.0 / mean_one,
           "sample": f"{procs} single-bit injections of the headline workload (sites 0..{procs - 1} of the "
                     f"campaign), each an FP64 plain-path render of the whole {cam.width}x{cam.height} frame of "
                     f"the {sc.n}-primitive scene (projection {np.mean([a for a, _ in many]):.1f} s, compositing "
                     f"and metrics {np.mean([b for _, b in many]):.1f} s per injection), run at once in {procs} "
                     f"forked processes of one thread each: {wall:.1f} s wall; the clean frame took "
                     f"{t_clean:.1f} s beforehand and is not counted"}
    _CPU.clear()
    return res


def make_parser():
    """The command line of bench.py."""
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60,
                    help="timed steps; a step is --batches-per-stream batches of --batch variants on every stream")
    ap.add_argument("--batches-per-stream", type=int, default=4,
                    help="batches of --batch variants each stream runs per step")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--fmt", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-tune", action="store_true",
                    help="use --tile/--streams/--threads/--wgs-per-cu/--resume/--graphs as given instead of the "
                         "autotuner's choice at the fixed --batch")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--streams", type=int, default=64, help="HIP streams the batches rotate over")
    ap.add_argument("--threads", type=int, default=2,
                    help="host threads of the native campaign call (0: a Python loop of sg_render_batch calls)")
    ap.add_argument("--wgs-per-cu", type=int, default=2, help="persistent compositing workgroups per CU (0: default)")
    ap.add_argument("--grid", type=int, default=0,
                    help="total persistent compositing workgroups, overriding --wgs-per-cu (0: per CU)")
    ap.add_argument("--resume", type=int, default=64,
                    help="checkpoint spacing of prepared scenes (0: walk every merged list from its start)")
    ap.add_argument("--graphs", action="store_true", help="replay each batch as a captured graph")
    ap.add_argument("--free-batch", type=int, default=512,
                    help="also tune B up to this bound and time that configuration (0: skip)")
    ap.add_argument("--plain", type=int, default=100, help="injections timed on the plain path")
    ap.add_argument("--no-persistent", dest="persistent", action="store_false",
                    help="skip the persistent campaign engine's rate on the same injections")
    ap.add_argument("--storm-n", type=int, default=32 * 2_056_645, help="primitives of the fault-storm scene")
    ap.add_argument("--storm-k", type=int, default=1000, help="upsets written per storm frame")
    ap.add_argument("--storm-frames", type=int, default=300, help="frames of the fault storm")
    ap.add_argument("--no-formats", dest="formats", action="store_false",
                    help="skip the fp16/bf16 (or fp32) rates at the headline configuration")
    ap.add_argument("--cpu-inj", type=int, default=1, help="time the oracle baseline (0: skip)")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes run at once for the all-core baseline (0: the host's cores, at most 16)")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="seconds of Poisson arrivals for the serving measurement (0: skip)")
    ap.add_argument("--workload", default="w2", choices=["w2", "guard", "large", "stress", "serve", "copy", "views", "storm",
                                                         "scenes"],
                    help="w2: the headline; guard: support guard and accumulated dose on the N=134,826 scene; "
                         "large: the 2,056,645-primitive bf16 scene at 1600x900; stress: one guarded render at "
                         "65,812,640 primitives")
    return ap


def main():
    ap = make_parser()
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every run here uses a single MI355X (--gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.workload != "w2":
        {"guard": run_guard, "large": run_large, "stress": run_stress, "serve": run_serve,
         "copy": run_copy, "views": run_views, "storm": run_storm, "scenes": run_scenes}[args.workload](args)
        return

    sc, cam, sites = _workload(args.fmt)
    cpu = None
    if args.cpu_inj > 0:   # before the GPU is touched (the workers fork)
        procs = args.cpu_procs if args.cpu_procs > 0 else min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(sc, cam, sites, args.fmt, procs)

    import torch
    from paper_2606_21791_amd import binding as sgb

    ctx = sgb.Context(0)
    ds = sgb.DeviceScene.upload(ctx, sc, args.fmt)
    tune_sample = sgb.sites_array(sites.field[:4096], sites.comp[:4096], sites.prim[:4096], sites.bit[:4096])
    tuned = None
    if not args.no_tune:
        t0 = time.perf_counter()
        tuned = ctx.autotune(ds, cam, tune_sample, fixed_batch=args.batch)
        tuned["seconds"] = round(time.perf_counter() - t0, 2)
        args.tile, args.streams, args.threads = tuned["tile"], tuned["streams"], tuned["threads"]
        args.wgs_per_cu, args.resume, args.graphs = tuned["wgs_per_cu"], tuned["resume"], bool(tuned["graphs"])
        args.grid = tuned["grid"]
    ctx.set_persistent(args.wgs_per_cu)
    ctx.set_persistent_grid(args.grid)
    ctx.set_resume(args.resume)
    ctx.set_graphs(args.graphs)
    NS = max(1, args.streams)
    streams = [torch.cuda.Stream() for _ in range(NS)]
    prep = ctx.prepare(ds, cam, sgb.raster_struct(tile=args.tile))
    torch.cuda.synchronize()
    B = args.batch
    # A step is --batches-per-stream B-variant batches on every stream: GB
    # injections, each of them the whole hot path (staging, projection of the
    # corrupted primitives, dirty tiles, compositing, metrics).
    GB = B * NS * args.batches_per_stream
    n_sites = len(sites)
    steps_total = args.warmup + args.steps
    n_all = steps_total * GB
    all_idx = np.arange(n_all) % n_sites
    sa_all = sgb.sites_array(sites.field[all_idx], sites.comp[all_idx], sites.prim[all_idx], sites.bit[all_idx])
    va_all = sgb.variants_array(np.arange(n_all), np.ones(n_all, np.uint32))
    va_b = sgb.variants_array(np.arange(B), np.ones(B, np.uint32))
    rec_bytes = sgb.METRICS_DTYPE.itemsize
    mt_all = sgb.metrics_tensor(n_all)
    w_end = args.warmup * GB

    def run_steps(first, last):
        """Steps [first, last): one campaign call (batches round-robin over the
        streams, enqueued by `threads` host threads), or a Python loop of
        sg_render_batch calls."""
        if args.threads > 0:
            ctx.campaign(prep, sa_all, va_all[first * GB:last * GB], mt_all[first * GB * rec_bytes:last * GB * rec_bytes],
                         batch=B, streams=NS, threads=args.threads)
        else:
            for j in range(first * GB // B, last * GB // B):
                with torch.cuda.stream(streams[j % NS]):
                    ctx.render_batch(prep, sa_all[j * B:(j + 1) * B], va_b,
                                     metrics=mt_all[j * B * rec_bytes:(j + 1) * B * rec_bytes])

    run_steps(0, args.warmup)
    torch.cuda.synchronize()
    # the K timed steps: one campaign, bracketed by synchronisations
    with _no_gc():
        t_start = time.perf_counter()
        run_steps(args.warmup, steps_total)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
    recs = sgb.read_metrics(mt_all)[w_end:]
    inj_per_s = args.steps * GB / elapsed
    # the same campaign REPS more times, for the spread of the rate
    REPS = 3
    rep_rates = []
    for r in range(REPS):
        with _no_gc():
            t0 = time.perf_counter()
            run_steps(args.warmup, steps_total)
            torch.cuda.synchronize()
            rep_rates.append(args.steps * GB / (time.perf_counter() - t0))
    rep_rates = np.array(rep_rates)

    # the same steps again with per-launch HIP events (recorded by each step
    # launch at its own start and end), for the per-pass breakdown and the
    # duration of the compositing launches
    ctx.timing(True)
    ctx.pass_times()
    with _no_gc():
        run_steps(args.warmup, steps_total)
        torch.cuda.synchronize()
    passes = ctx.pass_times()
    ctx.timing(False)
    recs_timed = sgb.read_metrics(mt_all)[w_end:]

    # dominant kernel: the campaign step launches that composite a batch (the
    # pipeline's fill and drain launches are timed apart, under "reduce")
    comp_ms, comp_n = passes["composite_items"]
    comp_avg_s = comp_ms / max(comp_n, 1) / 1e3
    evals_per_launch = float(recs["evals"].sum()) / max(comp_n, 1)
    achieved = evals_per_launch * FLOPS_PER_EVAL / comp_avg_s / 1e12 if comp_avg_s > 0 else 0.0

    def campaign_rate(c, pr, sa, n_inj, batch, nstreams, threads):
        """Injections/s of one campaign over the first n_inj variants of sa
        (after a warm-up campaign of a few steps), and its records."""
        va = sgb.variants_array(np.arange(n_inj), np.ones(n_inj, np.uint32))
        mt = sgb.metrics_tensor(n_inj)
        kw = dict(batch=batch, streams=nstreams, threads=threads)
        c.campaign(pr, sa, va[:min(n_inj, max(1, args.warmup) * batch * nstreams)], mt, **kw)
        torch.cuda.synchronize()
        with _no_gc():
            t0 = time.perf_counter()
            c.campaign(pr, sa, va, mt, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        return n_inj / dt, sgb.read_metrics(mt)

    # the other storage formats at the same launch configuration and step count
    per_format = {}
    for fmt in ("f32", "f16", "bf16"):
        if fmt == args.fmt or not args.formats:
            continue
        sc_f, _, sites_f = _workload(fmt)
        ds_f = sgb.DeviceScene.upload(ctx, sc_f, fmt)
        prep_fm = ctx.prepare(ds_f, cam, sgb.raster_struct(tile=args.tile))
        n_f = args.steps * GB
        idx_f = np.arange(n_f) % len(sites_f)
        sa_f = sgb.sites_array(sites_f.field[idx_f], sites_f.comp[idx_f], sites_f.prim[idx_f], sites_f.bit[idx_f])
        rate_f, r_f = campaign_rate(ctx, prep_fm, sa_f, n_f, B, NS, max(1, args.threads))
        per_format[fmt] = {"value": round(rate_f, 1), "injections": n_f, "steps": args.steps,
                           "dirty_tiles_per_injection": round(float(r_f["dirty_tiles"].mean()), 2),
                           "catastrophic_fraction": round(float(r_f["catastrophic"].mean()), 4)}
        del prep_fm, ds_f

    # the same injections with B tuned too (many variants per launch)
    free = None
    if args.free_batch > 0:
        t0 = time.perf_counter()
        tf = ctx.autotune(ds, cam, tune_sample, max_batch=args.free_batch)
        tf["seconds"] = round(time.perf_counter() - t0, 2)
        ctx_f = sgb.Context(0)
        ctx_f.apply_tune(tf)
        prep_f = ctx_f.prepare(ds, cam, sgb.raster_struct(tile=tf["tile"]))
        n_inj = args.steps * GB
        rate_tf, rf = campaign_rate(ctx_f, prep_f, sa_all[w_end:], n_inj, tf["batch"], tf["streams"], tf["threads"])
        same = all(np.array_equal(rf[k], recs[k]) for k in ("changed_px", "max_abs", "nonfinite")) and \
            bool(np.allclose(rf["sse"], recs["sse"], rtol=1e-12, atol=0.0))
        free = {"value": round(rate_tf, 1), "unit": "injections/s", "injections": n_inj,
                "config": {k: tf[k] for k in ("tile", "batch", "streams", "threads", "wgs_per_cu", "grid", "resume",
                                              "graphs")},
                "tune_seconds": tf["seconds"], "records_identical_to_headline": same}
        del prep_f, ctx_f

    # the same injections through the persistent engine: chunks of as many
    # variants as its buffers hold, each listed, composited by one persistent
    # launch and reduced (no per-batch launches, two streams)
    persist = None
    if args.persistent:
        # its own context and prepared view, with checkpoints every 16 list
        # entries (the persistent launch gains from the finer resume state)
        ctx_p = sgb.Context(0)
        ctx_p.set_resume(PERSIST_RESUME)
        prep_p = ctx_p.prepare(ds, cam, sgb.raster_struct(tile=args.tile))
        n_inj = args.steps * GB
        va_p = sgb.variants_array(np.arange(n_inj), np.ones(n_inj, np.uint32))
        mt_p = sgb.metrics_tensor(n_inj)
        sa_p = sa_all[w_end:]
        ctx_p.campaign(prep_p, sa_p, va_p, mt_p, engine=sgb.SG_ENGINE_PERSISTENT)   # warm-up, buffers sized
        torch.cuda.synchronize()
        p_rates = []
        for r in range(1 + REPS):
            with _no_gc():
                t0 = time.perf_counter()
                ctx_p.campaign(prep_p, sa_p, va_p, mt_p, engine=sgb.SG_ENGINE_PERSISTENT)
                torch.cuda.synchronize()
                p_rates.append(n_inj / (time.perf_counter() - t0))
        rp = sgb.read_metrics(mt_p)
        ctx_p.timing(True)
        ctx_p.pass_times()
        ctx_p.campaign(prep_p, sa_p, va_p, mt_p, engine=sgb.SG_ENGINE_PERSISTENT)
        torch.cuda.synchronize()
        pp = ctx_p.pass_times()
        ctx_p.timing(False)
        del prep_p, ctx_p
        pc_ms, pc_n = pp["composite_items"]
        pc_avg_s = pc_ms / max(pc_n, 1) / 1e3
        p_evals = float(rp["evals"].sum()) / max(pc_n, 1)
        p_ach = p_evals * FLOPS_PER_EVAL / pc_avg_s / 1e12 if pc_avg_s > 0 else 0.0
        persist = {"value": round(p_rates[0], 1), "unit": "injections/s", "injections": n_inj,
                   "repetitions": {"n": REPS, "median": round(float(np.median(p_rates[1:])), 1)},
                   "variants_per_launch": int(-(-n_inj // max(pc_n, 1))), "resume_spacing": PERSIST_RESUME,
                   # every field but the evaluation count, which the checkpoint spacing changes
                   "records_identical_to_headline": bool(all(np.array_equal(rp[k], recs[k]) for k in rp.dtype.names
                                                             if k != "evals")),
                   "pass_ms": {k: round(v[0], 3) for k, v in pp.items() if v[1]},
                   "roofline": {"bound": "alu", "kernel": "k_persist_composite", "achieved": round(p_ach, 3),
                                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(p_ach / FP32_PEAK_TFLOPS, 4),
                                "avg_launch_ms": round(pc_avg_s * 1e3, 4), "launches": pc_n,
                                "evals_per_launch": round(p_evals), "flops_per_eval": FLOPS_PER_EVAL}}

    # plain path: inject, full render with metrics against the clean frame, restore, read back
    frame = prep.frame()
    mt1 = sgb.metrics_tensor(1)
    P = args.plain
    for k in range(min(5, P)):
        sa = sa_all[k:k + 1]
        ctx.inject(ds, sa)
        ctx.render(ds, cam, sgb.raster_struct(tile=args.tile), clean=frame, metrics=mt1)
        ctx.restore(ds, sa)
        sgb.read_metrics(mt1)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.pass_times()
    t0 = time.perf_counter()
    plain_recs = []
    for k in range(P):
        sa = sa_all[w_end + k:w_end + k + 1]
        ctx.inject(ds, sa)
        ctx.render(ds, cam, sgb.raster_struct(tile=args.tile), clean=frame, metrics=mt1)
        ctx.restore(ds, sa)
        plain_recs.append(sgb.read_metrics(mt1)[0])
    torch.cuda.synchronize()
    plain_dt = time.perf_counter() - t0
    plain_passes = ctx.pass_times()
    ctx.timing(False)
    plain_recs = np.array(plain_recs)
    # the same injections on both paths give the same records
    same = recs[:P]
    agree = bool(np.array_equal(same["changed_px"], plain_recs["changed_px"]) and
                 np.array_equal(same["nonfinite"], plain_recs["nonfinite"]))

    out = {
        "metric": "injections/s at N=135k 800x800 batched vs plain; p50/p99 request latency",
        "value": round(inj_per_s, 1),
        "unit": "injections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.fmt == "f32" else f"{args.fmt} storage, f32/f64 arithmetic",
        "data": "synthetic (seeded scene and sites standing in for the paper's trained scenes)",
        "config": {"workload": f"scaling-sweep large scene: N=134,826 Gaussians, SH degree 3, {args.fmt} storage, "
                               f"800x800, {args.tile}x{args.tile} tiles, B={B} single-bit variants per launch, "
                               f"incremental dirty-tile re-composite; a step is {args.batches_per_stream} batches on "
                               f"each of the {NS} streams",
                   "global_batch": GB, "batch_per_launch": B, "n_sites": n_sites,
                   "instances_clean": prep.instances(), "streams": NS, "host_threads": args.threads, "wgs_per_cu": args.wgs_per_cu,
                   "grid": args.grid,
                   "graphs": args.graphs, "resume_spacing": args.resume,
                   "tuned": tuned is not None, "gpu_max_hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"])},
        "repeat_records_identical": bool(all(np.array_equal(recs[k], recs_timed[k])
                                             for k in ("sse", "changed_px", "max_abs", "nonfinite", "evals"))),
        "plain": {"value": round(P / plain_dt, 1), "unit": "injections/s", "injections": P,
                  "ms_per_injection": round(plain_dt / P * 1e3, 4),
                  "pass_ms_per_injection": {k: round(v[0] / max(P, 1), 4) for k, v in plain_passes.items() if v[1]},
                  "pass_gbps": _plain_pass_gbps(sc.n, prep.instances(), cam, args.fmt, plain_passes, P),
                  "records_agree_with_batched": agree},
        "speedup_vs_plain": round(inj_per_s / (P / plain_dt), 2),
        "tuned_any_batch": free,
        "persistent": persist,
        "pass_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in passes.items() if v[1]},
        "repetitions": {"n": REPS, "median": round(float(np.median(rep_rates)), 1),
                        "p10": round(float(np.percentile(rep_rates, 10)), 1),
                        "p90": round(float(np.percentile(rep_rates, 90)), 1)},
        "dirty_tile_histogram": {"bin_edges": DIRTY_BINS,
                                 "counts": np.histogram(recs["dirty_tiles"], bins=DIRTY_BINS)[0].tolist()},
        "per_format": per_format,
        "dirty_tiles_per_injection": round(float(recs["dirty_tiles"].mean()), 2),
        "catastrophic_fraction": round(float(recs["catastrophic"].mean()), 4),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": (_measured_traffic(args.resume)
                                 if (args.fmt == "f32" and B == 32 and args.tile == 16) else None),
                     "aggregate_achieved": round(float(recs["evals"].sum()) * FLOPS_PER_EVAL / elapsed / 1e12, 3),
                     "kernel": "k_campaign_step", "avg_launch_ms": round(comp_avg_s * 1e3, 4),
                     "evals_per_launch": round(evals_per_launch), "flops_per_eval": FLOPS_PER_EVAL},
        "paper_context": PAPER_CONTEXT,
    }
    if args.serve_seconds > 0:
        del prep, ds
        torch.cuda.synchronize()
        out["serving"] = serve_workload(args.serve_seconds)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def _plain_pass_gbps(n, inst, cam, fmt, passes, P):
    """Achieved GB/s of the plain path's passes from their algorithmic bytes:
    project reads 59 stored words and writes a 48-B record, depth and
    rectangle per primitive; binning reads depth and rectangle and writes an
    8-B key per instance; the per-tile sort reads and writes each key once;
    compositing reads each instance's key and record and the clean frame."""
    w = 4 if fmt == "f32" else 2
    px = cam.width * cam.height
    alg = {"project": n * (59 * w + 48 + 4 + 8), "bin": n * 12 + inst * 8, "sort": inst * 16,
           "composite_full": inst * (8 + 48) + px * 12}
    out = {}
    for k, b in alg.items():
        ms, cnt = passes.get(k, (0.0, 0))
        if cnt and ms > 0:
            gbps = b / (ms / P / 1e3) / 1e9
            out[k] = {"bytes": int(b), "GB_s": round(gbps, 1), "frac_of_8TB_s": round(gbps / 8000.0, 4)}
    return out


class _no_gc:
    """Keeps Python's cyclic collector out of a timed submission loop (a full
    collection in a process holding torch stalls the host for tens of ms)."""

    def __enter__(self):
        gc.collect()
        gc.disable()

    def __exit__(self, *exc):
        gc.enable()


def _batched_rate(ctx, prep, sites, B, streams, threads, steps, warmup, guard=0, box=None, box_mask=0x1F, protect=0):
    """Batched incremental injections/s of one campaign call over `steps`
    batches of B (after `warmup` batches), and the per-variant records."""
    import torch
    from paper_2606_21791_amd import binding as sgb
    n = len(sites)
    total = (warmup + steps) * B
    idx = np.arange(total) % n
    sa = sgb.sites_array(sites.field[idx], sites.comp[idx], sites.prim[idx], sites.bit[idx])
    va = sgb.variants_array(np.arange(total), np.ones(total, np.uint32), guard, protect)
    mt = sgb.metrics_tensor(total)
    rb = sgb.METRICS_DTYPE.itemsize
    kw = dict(box=box, box_mask=box_mask, batch=B, streams=streams, threads=threads)
    ctx.campaign(prep, sa, va[:warmup * B], mt[:warmup * B * rb], **kw)
    torch.cuda.synchronize()
    with _no_gc():
        t0 = time.perf_counter()
        ctx.campaign(prep, sa, va[warmup * B:], mt[warmup * B * rb:], **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    recs = sgb.read_metrics(mt)[warmup * B:]
    return steps * B / dt, recs


def _side_batches(args, cap):
    """Batches timed by the workloads other than the headline: as many as the
    headline's steps hold (steps x batches per stream x streams), at most cap."""
    return max(1, min(cap, args.steps * args.batches_per_stream * max(1, args.streams)))


def _tune_into(ctx, args, ds, cam, sites):
    """Autotune at the fixed --batch (unless --no-tune) and apply the result to
    ctx and args; returns the tuner's record or None."""
    from paper_2606_21791_amd import binding as sgb
    if args.no_tune:
        ctx.set_persistent(args.wgs_per_cu)
        ctx.set_persistent_grid(args.grid)
        ctx.set_resume(args.resume)
        ctx.set_graphs(args.graphs)
        return None
    k = min(4096, len(sites))
    sample = sgb.sites_array(sites.field[:k], sites.comp[:k], sites.prim[:k], sites.bit[:k])
    t = ctx.autotune(ds, cam, sample, fixed_batch=args.batch)
    args.tile, args.streams, args.threads = t["tile"], t["streams"], t["threads"]
    args.wgs_per_cu, args.resume, args.graphs = t["wgs_per_cu"], t["resume"], bool(t["graphs"])
    args.grid = t["grid"]
    ctx.apply_tune(t)
    return t


def _coarsen(mask, s):
    """Region mask of the 8 x 8 grid coarsened to (8/s) x (8/s) regions."""
    out = 0
    for b in range(64):
        if (mask >> b) & 1:
            ry, rx = divmod(b, 8)
            out |= 1 << ((ry // s) * (8 // s) + rx // s)
    return out


def _contamination(recs, sel=None):
    """Sort-first contamination (Sec. 5.10) per partition of 4, 16 and 64
    regions: mean fraction of regions whose pixels change (rendered) and
    whose primitive sets change (predicted), and the mean intersection over
    union of the two region sets (variants with a non-empty union)."""
    pred = [int(x) for x in recs["predicted_regions"]]
    rend = [int(x) for x in recs["rendered_regions"]]
    if sel is not None:
        pred = [pred[i] for i in sel]
        rend = [rend[i] for i in sel]
    out = {"variants": len(pred)}
    for s, R in ((4, 4), (2, 16), (1, 64)):
        p = [_coarsen(m, s) if s > 1 else m for m in pred]
        r = [_coarsen(m, s) if s > 1 else m for m in rend]
        ious = [bin(a & b).count("1") / bin(a | b).count("1") for a, b in zip(p, r) if a | b]
        out[f"R{R}"] = {"rendered_frac": round(float(np.mean([bin(x).count("1") / R for x in r])) if r else 0.0, 4),
                        "predicted_frac": round(float(np.mean([bin(x).count("1") / R for x in p])) if p else 0.0, 4),
                        "iou": round(float(np.mean(ious)), 4) if ious else None}
    return out


def _summ(recs):
    ps = recs["psnr"][np.isfinite(recs["psnr"])]
    return {"mean_psnr_db": round(float(ps.mean()), 3) if ps.size else None,
            "worst_footprint": round(float(recs["footprint"].max()), 5),
            "mean_footprint": round(float(recs["footprint"].mean()), 6),
            "catastrophic_fraction": round(float(recs["catastrophic"].mean()), 5),
            "nonfinite": int(recs["nonfinite"].sum()), "clamps": int(recs["clamps"].sum())}


def run_guard(args):
    """Support guard on the N=134,826 scene (fp32, 800x800) with a
    per-primitive box: guard cost per frame (scrub pass and clamp-on-load),
    guarded vs unguarded single flips, and accumulated-dose frames."""
    import torch
    from paper_2606_21791_amd import binding as sgb, synth
    sc, cam, sites = _workload("f32")
    ctx = sgb.Context(0)
    lo32, hi32 = synth.make_box_jitter(sc, seed=4)
    ds = sgb.DeviceScene.upload(ctx, sc, "f32")
    box = sgb.Box.per_prim(ctx, lo32, hi32, "f32")
    tuned = _tune_into(ctx, args, ds, cam, sites)
    prep = ctx.prepare(ds, cam, sgb.raster_struct(tile=args.tile))
    torch.cuda.synchronize()
    out = {"metric": "support guard: cost per frame, guarded vs unguarded injections, accumulated dose",
           "config": {"workload": "N=134,826 Gaussians, SH degree 3, fp32, 800x800, per-primitive box "
                                  "(value -/+ |N(0,0.2)|, rounded outward)", "B": args.batch, "tile": args.tile,
                      "streams": args.streams, "host_threads": args.threads, "tuned": tuned is not None}}
    # guard cost: the scrub pass over the resident scene (identity on the clean scene)
    work = ds.clone()
    for _ in range(3):
        ctx.guard(work, box)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.pass_times()
    reps = 50
    for _ in range(reps):
        ctx.guard(work, box)
    torch.cuda.synchronize()
    g_ms = ctx.pass_times()["guard"][0] / reps
    # clamp-on-load: the projection pass with and without the box
    frame = prep.frame()
    proj = {}
    for name, bx in (("without", None), ("with", box)):
        ctx.pass_times()
        for _ in range(20):
            ctx.render(ds, cam, box=bx)
        torch.cuda.synchronize()
        proj[name] = ctx.pass_times()["project"][0] / 20
    ctx.timing(False)
    n = sc.n
    guarded_bytes = n * 14 * 4 * 3            # value + lo + hi words read per frame
    out["guard_cost"] = {"scrub_us_per_frame": round(g_ms * 1e3, 2),
                         "scrub_read_GB_s": round(guarded_bytes / (g_ms * 1e-3) / 1e9, 1),
                         "clamp_on_load_extra_us": round((proj["with"] - proj["without"]) * 1e3, 2),
                         "projection_us_without_guard": round(proj["without"] * 1e3, 2)}
    # single flips, unguarded and guarded
    steps_g = _side_batches(args, 2000)
    site_of = (np.arange(steps_g * args.batch) + args.warmup * args.batch) % len(sites)
    scale_sign = np.nonzero((sites.field[site_of] == 1) & (sites.bit[site_of] == 31))[0]
    for guard in (0, 1):
        rate, recs = _batched_rate(ctx, prep, sites, args.batch, args.streams, max(1, args.threads),
                                   steps_g, args.warmup, guard, box)
        out["guarded" if guard else "unguarded"] = {
            "inj_per_s": round(rate, 1), **_summ(recs),
            "contamination_all": _contamination(recs),
            "contamination_scale_sign": _contamination(recs, scale_sign)}
    # Table 3: the alternative defenses on the same fault grid
    grid = {}
    for name, kw in (("none", {}), ("support_guard", {"guard": 1}),
                     ("selective_guard", {"guard": 1, "box_mask": (1 << 1) | (1 << 3)}),
                     ("ecc_sign_exp", {"protect": sgb.SG_PROTECT_SIGN_EXP}),
                     ("vote_3_copies", {"protect": sgb.SG_PROTECT_VOTE})):
        rate, recs = _batched_rate(ctx, prep, sites, args.batch, args.streams, max(1, args.threads), steps_g,
                                   args.warmup, box=box, **kw)
        grid[name] = {"catastrophe_pct": round(100.0 * float(recs["catastrophic"].mean()), 4),
                      "mean_footprint_pct": round(100.0 * float(recs["footprint"].mean()), 5),
                      "inj_per_s": round(rate, 1)}
    grid["memory_factor"] = {"none": 1.0, "support_guard": 1.0, "selective_guard": 1.0,
                             "ecc_sign_exp": round(1.0 + 9.0 / 32.0, 3), "vote_3_copies": 3.0,
                             "model": "the code stores one check bit per protected bit (9 of 32); the vote "
                                      "stores three copies"}
    out["mitigation_grid"] = grid

    # accumulated dose: k simultaneous flips over all stored bits, 16 frames each
    dose = {}
    mt = sgb.metrics_tensor(1)
    for k, seed0 in ((1000, 31), (20000, 47)):
        for guard in (0, 1):
            recs, t = [], 0.0
            for f in range(16):
                s = synth.make_sites_dose(n, 3, k, seed=seed0 + f, width_bits=32)
                sa = sgb.sites_array(s.field, s.comp, s.prim, s.bit)
                va = sgb.variants_array([0], [k], guard)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.render_batch(prep, sa, va, box=box, metrics=mt)
                recs.append(sgb.read_metrics(mt)[0])
                t += time.perf_counter() - t0
            recs = np.array(recs)
            dose[f"k{k}_{'guarded' if guard else 'unguarded'}"] = {"ms_per_frame": round(t / 16 * 1e3, 3), **_summ(recs)}
    out["dose"] = dose
    print(json.dumps(out), flush=True)


def _large_scene():
    from paper_2606_21791_amd import synth
    sc = synth.make_scene(2_056_645, seed=5, sh_degree=3, means="clusters")
    cam = synth.make_camera(1600, 900, distance=25.0)
    sites = synth.make_sites_stratified(sc.n, 3, 1024, seed=15, width_bits=16)
    order = np.random.default_rng(98).permutation(len(sites))
    return sc, cam, sites.take(order)


def run_large(args):
    """The 2,056,645-primitive clustered scene (bf16, SH degree 3, 1600x900):
    batched incremental injections vs the plain path."""
    import torch
    from paper_2606_21791_amd import binding as sgb
    sc, cam, sites = _large_scene()
    ctx = sgb.Context(0)
    ds = sgb.DeviceScene.upload(ctx, sc, "bf16")
    del sc
    tuned = _tune_into(ctx, args, ds, cam, sites)
    t0 = time.perf_counter()
    prep = ctx.prepare(ds, cam, sgb.raster_struct(tile=args.tile))
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    rate, recs = _batched_rate(ctx, prep, sites, args.batch, args.streams, max(1, args.threads),
                               _side_batches(args, 2000), args.warmup)
    frame = prep.frame()
    mt1 = sgb.metrics_tensor(1)
    P = max(5, args.plain // 4)
    ctx.timing(True)
    ctx.pass_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(P):
        sa = sgb.sites_array(sites.field[k:k + 1], sites.comp[k:k + 1], sites.prim[k:k + 1], sites.bit[k:k + 1])
        ctx.inject(ds, sa)
        ctx.render(ds, cam, clean=frame, metrics=mt1)
        ctx.restore(ds, sa)
        sgb.read_metrics(mt1)
    plain_dt = time.perf_counter() - t0
    pp = ctx.pass_times()
    ctx.timing(False)
    # the same injections through the persistent engine (its own context,
    # checkpoint spacing 16)
    persist = None
    if args.persistent:
        ctx_p = sgb.Context(0)
        ctx_p.set_resume(PERSIST_RESUME)
        prep_p = ctx_p.prepare(ds, cam, sgb.raster_struct(tile=args.tile))
        n_p = len(recs)
        idx = (np.arange(n_p) + args.warmup * args.batch) % len(sites)
        sa_p = sgb.sites_array(sites.field[idx], sites.comp[idx], sites.prim[idx], sites.bit[idx])
        va_p = sgb.variants_array(np.arange(n_p), np.ones(n_p, np.uint32))
        mt_p = sgb.metrics_tensor(n_p)
        ctx_p.campaign(prep_p, sa_p, va_p, mt_p, engine=sgb.SG_ENGINE_PERSISTENT)
        torch.cuda.synchronize()
        with _no_gc():
            t0 = time.perf_counter()
            ctx_p.campaign(prep_p, sa_p, va_p, mt_p, engine=sgb.SG_ENGINE_PERSISTENT)
            torch.cuda.synchronize()
            dt_p = time.perf_counter() - t0
        rp = sgb.read_metrics(mt_p)
        persist = {"value": round(n_p / dt_p, 1), "unit": "injections/s", "injections": n_p,
                   "resume_spacing": PERSIST_RESUME,
                   "records_identical": bool(all(np.array_equal(rp[k], recs[k]) for k in rp.dtype.names
                                                 if k != "evals"))}
        del prep_p, ctx_p
    out = {"metric": "injections/s, 2,056,645-primitive scene, 1600x900, batched vs plain",
           "value": round(rate, 1), "unit": "injections/s",
           "config": {"workload": "N=2,056,645 Gaussians in 64 anisotropic clusters, SH degree 3, bf16 storage, "
                                  f"1600x900, B={args.batch}, 6 fields x 1,024 stratified sites",
                      "tile": args.tile, "streams": args.streams, "host_threads": args.threads,
                      "wgs_per_cu": args.wgs_per_cu, "resume_spacing": args.resume, "tuned": tuned is not None,
                      "instances_clean": prep.instances(), "prepare_s": round(prep_s, 3),
                      "device_bytes": ctx.bytes()},
           "plain": {"value": round(P / plain_dt, 1), "unit": "injections/s",
                     "pass_ms_per_injection": {k: round(v[0] / P, 4) for k, v in pp.items() if v[1]}},
           "speedup_vs_plain": round(rate / (P / plain_dt), 2),
           "persistent": persist,
           "dirty_tiles_per_injection": round(float(recs["dirty_tiles"].mean()), 2), **_summ(recs)}
    print(json.dumps(out), flush=True)


def run_stress(args):
    """One guarded render of 65,812,640 primitives (SH degree 0, fp32,
    1600x900): the box is reduced once, then the guard scrub and the render
    are timed separately, with the render's per-pass breakdown."""
    import torch
    from paper_2606_21791_amd import binding as sgb, synth
    n = 32 * 2_056_645
    t0 = time.perf_counter()
    sc = synth.make_scene(n, seed=6, sh_degree=0, means="clusters")
    gen_s = time.perf_counter() - t0
    cam = synth.make_camera(1600, 900, distance=25.0)
    ctx = sgb.Context(0)
    ds = sgb.DeviceScene.upload(ctx, sc, "f32")
    del sc
    box = ctx.guard_box(ds)
    img = torch.empty((900, 1600, 3), dtype=torch.float32, device="cuda")
    ctx.render(ds, cam, image=img)            # warm-up and workspace sizing
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.pass_times()
    reps = 3
    for _ in range(reps):
        cnt, _ = ctx.guard(ds, box)
    torch.cuda.synchronize()
    g = ctx.pass_times()["guard"][0] / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.render(ds, cam, image=img)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    pp = ctx.pass_times()
    ctx.timing(False)
    render_ms = sum(v[0] for v in pp.values()) / reps
    out = {"metric": "guarded render at 65,812,640 primitives: guard and render time per frame",
           "config": {"workload": "N=65,812,640 Gaussians (64 clusters), SH degree 0, fp32, 1600x900, "
                                  "global box from the clean model", "generate_s": round(gen_s, 1)},
           "guard_ms_per_frame": round(g, 3),
           "guard_read_GB_s": round(n * 14 * 4 / (g * 1e-3) / 1e9, 1),
           "guard_hbm_frac": round(n * 14 * 4 / (g * 1e-3) / 8e12, 4),
           "render_ms_per_frame": round(render_ms, 3), "render_wall_ms": round(wall * 1e3, 3),
           "guard_fraction_of_render": round(g / render_ms, 4),
           "render_mpix_per_s": round(1600 * 900 / wall / 1e6, 2),
           "pass_ms": {k: round(v[0] / reps, 3) for k, v in pp.items() if v[1]},
           "clamps_clean": int(cnt[0]), "device_bytes": ctx.bytes(),
           "paper_context": {"guard_ms": 9.66, "guard_fraction": 0.183, "hardware": "Blackwell-generation GPU"}}
    print(json.dumps(out), flush=True)


def run_views(args):
    """K views per injection (Def. 1 pools the footprint over K views): the
    scaling-sweep scene (N=134,826, SH3, fp32) seen by K orbit cameras at
    800x800, batched campaigns of B variants for K in 1, 2, 4, 8, 16;
    injections/s and view-pixels composited per second (K x 800 x 800 per
    injection, the unit of the paper's multi-view throughput)."""
    import torch
    from paper_2606_21791_amd import binding as sgb, synth
    sc, cam, sites = _workload("f32")
    ctx = sgb.Context(0)
    ds = sgb.DeviceScene.upload(ctx, sc, "f32")
    tuned = _tune_into(ctx, args, ds, cam, sites)
    B = args.batch
    n_inj = _side_batches(args, 1000) * B
    idx = np.arange(n_inj) % len(sites)
    sa = sgb.sites_array(sites.field[idx], sites.comp[idx], sites.prim[idx], sites.bit[idx])
    va = sgb.variants_array(np.arange(n_inj), np.ones(n_inj, np.uint32))
    curve = []
    for K in (1, 2, 4, 8, 16):
        cams = synth.make_orbit_cameras(K, 800, 800)
        preps = [ctx.prepare(ds, c, sgb.raster_struct(tile=args.tile)) for c in cams]
        n = n_inj   # the same injections in every K (each stream's pipeline stays full)
        mt = sgb.metrics_tensor(n)
        kw = dict(batch=B, streams=args.streams, threads=max(1, args.threads))
        ctx.campaign(preps, sa, va[:4 * B], mt, **kw)
        torch.cuda.synchronize()
        with _no_gc():
            t0 = time.perf_counter()
            ctx.campaign(preps, sa, va[:n], mt, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        r = sgb.read_metrics(mt)
        # the same injections through the persistent engine (every variant of
        # a chunk in all K views in one compositing launch)
        mp = sgb.metrics_tensor(n)
        ctx.campaign(preps, sa, va[:n], mp, engine=sgb.SG_ENGINE_PERSISTENT)
        torch.cuda.synchronize()
        with _no_gc():
            t0 = time.perf_counter()
            ctx.campaign(preps, sa, va[:n], mp, engine=sgb.SG_ENGINE_PERSISTENT)
            torch.cuda.synchronize()
            dt_p = time.perf_counter() - t0
        rp = sgb.read_metrics(mp)
        # dense equivalent: K full 800 x 800 frames per injection; the
        # incremental path re-composites only the dirty tiles (an upper bound
        # of the pixels it composites)
        curve.append({"K": K, "inj_per_s": round(n / dt, 1),
                      "persistent_inj_per_s": round(n / dt_p, 1),
                      "persistent_records_identical": bool(all(np.array_equal(rp[k], r[k]) for k in r.dtype.names)),
                      "dense_equiv_view_mpix_per_s": round(n * K * 0.64 / dt, 1),
                      "dirty_tile_mpix_per_s": round(float(r["dirty_tiles"].sum()) * args.tile ** 2 / dt / 1e6, 1),
                      "mean_footprint": round(float(r["footprint"].mean()), 6),
                      "catastrophic_fraction": round(float(r["catastrophic"].mean()), 4),
                      "dirty_tiles_per_injection": round(float(r["dirty_tiles"].mean()), 2)})
        del preps
        torch.cuda.synchronize()
    out = {"metric": "K-view injections: injections/s and (dense-equivalent) view-Mpix/s vs K",
           "config": {"workload": "N=134,826 Gaussians, SH degree 3, fp32, K orbit views at 800x800 "
                                  f"(elevation 15 deg), B={B}", "tile": args.tile, "streams": args.streams,
                      "host_threads": args.threads, "resume_spacing": args.resume, "tuned": tuned is not None},
           "curve": curve,
           "paper_context": {"view_mpix_per_s": 837, "saturation_views": 16, "hardware": "Blackwell-generation GPU, "
                             "full renders of K views per injection"}}
    print(json.dumps(out), flush=True)


def run_scenes(args):
    """Scenes of uneven size in one campaign: single-bit variants of three
    resident scenes (6,741 Gaussians fp32 at 512x512, 134,826 fp32 at
    800x800, 500,000 clustered bf16 at 1600x900, all SH degree 3) mixed in
    random order, B variants per launch.  The same variants as one
    sg_campaign_scenes call, and as one sg_campaign per scene back to back."""
    import torch
    from paper_2606_21791_amd import binding as sgb, synth
    specs = [(6741, "f32", 512, 512, "uniform"), (N_HI, "f32", 800, 800, "uniform"),
             (500_000, "bf16", 1600, 900, "clusters")]
    ctx = sgb.Context(0)
    ctx.set_persistent(args.wgs_per_cu)
    ctx.set_resume(args.resume)
    preps, keep, site_sets = [], [], []
    for j, (n, fmt, w, h, means) in enumerate(specs):
        sc = synth.make_scene(n, seed=90 + j, sh_degree=3, means=means)
        ds = sgb.DeviceScene.upload(ctx, sc, fmt)
        cam = synth.make_camera(w, h) if means == "uniform" else synth.make_camera(w, h, distance=25.0)
        preps.append(ctx.prepare(ds, cam, sgb.raster_struct(tile=args.tile)))
        keep.append(ds)
        W = 32 if fmt == "f32" else 16
        site_sets.append(synth.make_sites_stratified(n, 3, 1000, seed=95 + j, width_bits=W))
    torch.cuda.synchronize()
    cat = lambda key: np.concatenate([getattr(t, key) for t in site_sets])
    sa = sgb.sites_array(cat("field"), cat("comp"), cat("prim"), cat("bit"))
    base = np.cumsum([0] + [len(t.prim) for t in site_sets])
    B = args.batch
    n_inj = _side_batches(args, 1000) * B
    rng = np.random.default_rng(97)
    scene_of = rng.integers(0, len(specs), size=n_inj).astype(np.uint16)
    off = np.array([base[k] + rng.integers(0, len(site_sets[k].prim)) for k in scene_of])
    va = sgb.variants_array(off, np.ones(n_inj, np.uint32))
    kw = dict(batch=B, streams=args.streams, threads=max(1, args.threads))
    mt = sgb.metrics_tensor(n_inj)
    ctx.campaign_scenes(preps, sa, va[:4 * B], scene_of[:4 * B], mt, **kw)
    torch.cuda.synchronize()
    with _no_gc():
        t0 = time.perf_counter()
        ctx.campaign_scenes(preps, sa, va, scene_of, mt, **kw)
        torch.cuda.synchronize()
        dt_mixed = time.perf_counter() - t0
    mixed = sgb.read_metrics(mt)
    # one campaign per scene, on that scene's own sites
    per_scene = []
    for k in range(len(specs)):
        idx = np.nonzero(scene_of == k)[0]
        t = site_sets[k]
        vk = va[idx].copy()
        vk["site_off"] -= np.uint32(base[k])
        per_scene.append((idx, sgb.sites_array(t.field, t.comp, t.prim, t.bit), vk, sgb.metrics_tensor(len(idx))))
    for k, (idx, sak, vk, mk) in enumerate(per_scene):
        ctx.campaign(preps[k], sak, vk[:4 * B], mk, **kw)
    torch.cuda.synchronize()
    with _no_gc():
        t0 = time.perf_counter()
        for k, (idx, sak, vk, mk) in enumerate(per_scene):
            ctx.campaign(preps[k], sak, vk, mk, **kw)
        torch.cuda.synchronize()
        dt_split = time.perf_counter() - t0
    same = all(np.array_equal(sgb.read_metrics(mk)[key], mixed[key][idx])
               for idx, _, _, mk in per_scene for key in ("sse", "changed_px", "dirty_tiles", "evals"))
    # the mixed campaign through the persistent engine
    mp = sgb.metrics_tensor(n_inj)
    ctx.campaign_scenes(preps, sa, va, scene_of, mp, engine=sgb.SG_ENGINE_PERSISTENT)
    torch.cuda.synchronize()
    with _no_gc():
        t0 = time.perf_counter()
        ctx.campaign_scenes(preps, sa, va, scene_of, mp, engine=sgb.SG_ENGINE_PERSISTENT)
        torch.cuda.synchronize()
        dt_pers = time.perf_counter() - t0
    pers = sgb.read_metrics(mp)
    out = {"metric": "scenes of uneven size: injections/s of one mixed campaign vs one campaign per scene",
           "config": {"workload": "3 scenes (6,741 fp32 512x512; 134,826 fp32 800x800; 500,000 clustered bf16 "
                                  f"1600x900; SH degree 3), single-bit variants in random scene order, B={B}",
                      "injections": n_inj, "streams": args.streams, "host_threads": args.threads,
                      "wgs_per_cu": args.wgs_per_cu, "resume_spacing": args.resume},
           "mixed_inj_per_s": round(n_inj / dt_mixed, 1), "per_scene_inj_per_s": round(n_inj / dt_split, 1),
           "records_identical": bool(same),
           "persistent_mixed_inj_per_s": round(n_inj / dt_pers, 1),
           "persistent_records_identical": bool(all(np.array_equal(pers[k], mixed[k]) for k in mixed.dtype.names)),
           "per_scene_injections": [int(len(idx)) for idx, _, _, _ in per_scene]}
    print(json.dumps(out), flush=True)


def run_storm(args):
    """Fault storm on the largest model (Sec. 5.12): k random upsets over every
    stored bit are written into the resident scene every frame, for F frames;
    each frame is rendered from the corrupted scene, unguarded, guarded every
    frame, or scrubbed every M frames (Cor. 2's periodic scrub).  Reports
    per-frame latency (inject + guard + render) and the PSNR / SSIM of the
    frames against the clean frame."""
    import torch
    from paper_2606_21791_amd import binding as sgb, synth
    n = args.storm_n
    t0 = time.perf_counter()
    sc = synth.make_scene(n, seed=6, sh_degree=0, means="clusters")
    gen_s = time.perf_counter() - t0
    cam = synth.make_camera(1600, 900, distance=25.0)
    ctx = sgb.Context(0)
    clean_ds = sgb.DeviceScene.upload(ctx, sc, "f32")
    del sc
    box = ctx.guard_box(clean_ds)
    H, W = cam.height, cam.width
    clean = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    ctx.render(clean_ds, cam, image=clean)
    img = torch.empty((1, H, W, 3), dtype=torch.float32, device="cuda")
    mt = sgb.metrics_tensor(1)
    k, F = args.storm_k, args.storm_frames
    # the same upsets for every mode
    storm = [synth.make_sites_dose(n, 0, k, seed=10_000 + f, width_bits=32) for f in range(F)]
    storm = [sgb.sites_array(x.field, x.comp, x.prim, x.bit) for x in storm]
    modes = (("unguarded", 0), ("guard_every_frame", 1), ("scrub_every_10", 10), ("scrub_every_100", 100))
    out = {"metric": "fault storm: per-frame latency and fidelity under k upsets per frame",
           "config": {"workload": f"N={n:,} Gaussians (64 clusters), SH degree 0, fp32, 1600x900, {k} random "
                                  f"upsets over all stored bits per frame, {F} frames, global box",
                      "generate_s": round(gen_s, 1)},
           "paper_context": {"guarded_ms": 22.9, "unguarded_ms": 20.5, "k": 1000, "frames": 300,
                             "hardware": "Blackwell-generation GPU"}}
    sample = set(range(0, F, max(1, F // 10))) | {F - 1}
    for name, every in modes:
        work = clean_ds.clone()
        torch.cuda.synchronize()
        lat, psnr, ssim, nonfinite, clamps = [], [], [], 0, 0
        for f in range(F):
            t0 = time.perf_counter()
            ctx.inject(work, storm[f])
            if every and (f + 1) % every == 0:
                cnt, _ = ctx.guard(work, box)
            ctx.render(work, cam, image=img[0], clean=clean, metrics=mt)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            if every and (f + 1) % every == 0:
                clamps += int(cnt[0])
            if f in sample:
                r = sgb.read_metrics(mt)[0]
                psnr.append(float(r["psnr"]))
                ssim.append(float(ctx.ssim(img, clean).cpu()[0]))
                nonfinite += int(r["nonfinite"])
        lat_ms = np.array(lat) * 1e3
        out[name] = {"ms_per_frame_mean": round(float(lat_ms.mean()), 3),
                     "ms_per_frame_p50": round(float(np.median(lat_ms)), 3),
                     "ms_per_frame_p99": round(float(np.percentile(lat_ms, 99)), 3),
                     "psnr_db_sampled": [round(x, 2) for x in psnr], "ssim_sampled": [round(x, 5) for x in ssim],
                     "final_psnr_db": round(psnr[-1], 3), "final_ssim": round(ssim[-1], 5),
                     "nonfinite_sampled_frames": nonfinite, "clamps": clamps}
        del work
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


def serve_workload(seconds, rate=2000.0, plain_seconds=1.0, slots=8, include_large=True, seed=21):
    """Poisson stream (mean `rate` requests/s) over resident scenes of
    6,741 / 134,826 / 500,000 / 2,056,645 primitives in fp32, fp16 and bf16,
    viewed at 256x256, 512x512, 800x800 and 1600x900; half the requests are
    injection campaigns (32 sites in one random (field, bit) cell), half are
    guarded renders with k in {0, 1, 1000} simultaneous flips.  The same
    stream (its first `plain_seconds`) also runs through the plain FIFO path."""
    import torch
    from paper_2606_21791_amd import binding as sgb, synth
    sizes = [(6741, 3, "uniform", 3.0), (134_826, 3, "uniform", 3.0), (500_000, 3, "uniform", 3.0)]
    if include_large:
        sizes.append((2_056_645, 3, "clusters", 25.0))
    fmts = ["f32", "f16", "bf16"]
    res = [(256, 256), (512, 512), (800, 800), (1600, 900)]
    ctx = sgb.Context(0)
    scenes = []          # (n, sh, fmt, dist, DeviceScene, Box)
    for n, deg, dist, dist_z in sizes:
        sc = synth.make_scene(n, seed=7 + n % 97, sh_degree=deg, means=dist)
        for fmt in fmts:
            ds = sgb.DeviceScene.upload(ctx, sc, fmt)
            box = ctx.guard_box(ds)
            scenes.append((n, deg, fmt, dist_z, ds, box))
        del sc
    torch.cuda.synchronize()

    def build(server):
        views = []
        for n, deg, fmt, dz, ds, box in scenes:
            sid = server.add_scene(ds, box)
            for w, h in res:
                views.append((server.add_view(sid, synth.make_camera(w, h, distance=dz)), n, deg, fmt))
        return views

    rng = np.random.default_rng(seed)
    arrivals = synth.make_arrivals(rate, seconds, seed)
    n_views = len(scenes) * len(res)
    plan = []
    for t in arrivals:
        vi = int(rng.integers(0, n_views))
        n, deg, fmt = scenes[vi // len(res)][:3]
        W = 32 if fmt == "f32" else 16
        if rng.random() < 0.5:
            comps = synth.field_components(deg)
            f = int(rng.integers(0, 6))
            bit = int(rng.integers(0, W))
            sites = sgb.sites_array(np.full(32, f), rng.integers(0, comps[f], 32), rng.integers(0, n, 32),
                                    np.full(32, bit))
            plan.append((t, sgb.SG_REQ_CAMPAIGN, vi, sites))
        else:
            k = int(rng.choice([0, 1, 1000]))
            s = synth.make_sites_dose(n, deg, k, int(rng.integers(1 << 30)), width_bits=W)
            plan.append((t, sgb.SG_REQ_GUARDED_RENDER, vi, sgb.sites_array(s.field, s.comp, s.prim, s.bit)))

    def drive(server, views, horizon):
        tickets = []
        t0 = time.monotonic_ns()
        for t, kind, vi, sites in plan:
            if t > horizon:
                break
            due = t0 + int(t * 1e9)
            while time.monotonic_ns() < due:
                pass
            tickets.append(server.submit(kind, views[vi][0], sites, arrival_ns=due))
        for tk in tickets:
            r, _ = server.wait(tk, 600)
            assert r["status"] == 0, r
        return server.stats()

    srv = sgb.Server(0, budget=0, max_slots=slots, max_batch=64)
    t0 = time.perf_counter()
    views = build(srv)
    setup_s = time.perf_counter() - t0
    st = drive(srv, views, seconds)
    srv.close()
    out = {"requests": len(arrivals), "arrival_rate_per_s": rate, "seconds": seconds, "slots": slots,
           "views": len(views), "setup_s": round(setup_s, 1),
           "throughput_inj_per_s": round(st["inj_per_s"], 1), "req_per_s": round(st["req_per_s"], 1),
           "p50_ms": {"campaign": round(st["campaign"]["p50_us"] / 1e3, 3),
                      "guarded_render": round(st["guarded_render"]["p50_us"] / 1e3, 3)},
           "p99_ms": {"campaign": round(st["campaign"]["p99_us"] / 1e3, 3),
                      "guarded_render": round(st["guarded_render"]["p99_us"] / 1e3, 3)},
           "launches": st["launches"], "completed": st["completed"], "rejected": st["rejected"],
           "resident_GB": round(st["resident_bytes"] / 1e9, 3)}
    if plain_seconds > 0:
        ps = sgb.Server(0, max_slots=1, plain=True)
        pviews = build(ps)
        pst = drive(ps, pviews, plain_seconds)
        ps.close()
        out["plain_fifo"] = {"seconds_of_arrivals": plain_seconds, "completed": pst["completed"],
                             "throughput_inj_per_s": round(pst["inj_per_s"], 1),
                             "p50_ms": {"campaign": round(pst["campaign"]["p50_us"] / 1e3, 3),
                                        "guarded_render": round(pst["guarded_render"]["p50_us"] / 1e3, 3)},
                             "p99_ms": {"campaign": round(pst["campaign"]["p99_us"] / 1e3, 3),
                                        "guarded_render": round(pst["guarded_render"]["p99_us"] / 1e3, 3)}}
    return out


def run_serve(args):
    out = {"metric": "serving: throughput and p50/p99 request latency, continuous batching vs plain FIFO",
           **serve_workload(args.serve_seconds if args.serve_seconds > 0 else 5.0)}
    print(json.dumps(out), flush=True)


def run_copy(args):
    """Device-to-device copy of 1 GiB (fp32), 10 times: the stream-copy ceiling
    of the HBM, and the calibration point of the FETCH_SIZE / WRITE_SIZE
    counters (each launch reads and writes exactly 1 GiB)."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    print(json.dumps({"metric": "stream copy, 1 GiB read + 1 GiB write per launch", "bytes_per_launch": 2 * 4 * n,
                      "ms_per_launch": round(ms, 4), "GB_s": round(2 * 4 * n / (ms * 1e-3) / 1e9, 1),
                      "frac_of_8TB_s": round(2 * 4 * n / (ms * 1e-3) / 8e12, 4)}), flush=True)


if __name__ == "__main__":
    main()
