"""Oracle renders of many corrupted variants of full-size scenes, spread over
a pool of spawned host processes (the FP64 oracle is single-threaded and a
full 800 x 800 frame of the 134,826-primitive scene takes about 20 s).

Each worker regenerates the seeded scenes it is asked about (synth draws them
deterministically) and caches their stored words and clean projections, so
no large array crosses a process boundary.  A job names a scene, a camera, a
list of sites (field, comp, prim, bit) to flip, an optional guard box and a
window: an explicit (x0, y0, x1, y1), "full", or "changed" (the old and new
supports of the corrupted primitives, outside which the variant equals the
clean frame exactly).  Test infrastructure only.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

_CACHE = {}


def scene_spec(n, seed, sh_degree, fmt, means="uniform"):
    return (int(n), int(seed), int(sh_degree), str(fmt), str(means))


def _words(spec):
    key = ("w",) + spec
    if key not in _CACHE:
        from oracle import formats
        from paper_2606_21791_amd import synth
        n, seed, sh, fmt, means = spec
        sc = synth.make_scene(n, seed=seed, sh_degree=sh, means=means)
        _CACHE[key] = ([formats.store(f, fmt) for f in sc.fields], sc)
    return _CACHE[key]


def _clean_proj(spec, cam, cam_key):
    key = ("p",) + spec + (cam_key,)
    if key not in _CACHE:
        from oracle import render
        words, _ = _words(spec)
        _CACHE[key] = render.project(render.decode_scene(words, spec[3]), spec[2], cam)
    return _CACHE[key]


def _box_words(spec, box_seed):
    key = ("b",) + spec + (box_seed,)
    if key not in _CACHE:
        from oracle import formats
        from paper_2606_21791_amd import synth
        _, sc = _words(spec)
        lo32, hi32 = synth.make_box_jitter(sc, seed=box_seed)
        fmt = spec[3]
        lo = [None if a is None else formats.store(a, fmt, "rd") for a in lo32]
        hi = [None if a is None else formats.store(a, fmt, "ru") for a in hi32]
        _CACHE[key] = (lo, hi)
    return _CACHE[key]


def run_job(job):
    """job: dict(spec, cam, cam_key, sites [(f, c, p, b)], window, box_seed,
    guard_fields).  Returns dict(image, amb, T, nonfinite, window, clamps,
    prims)."""
    from oracle import formats, guard as oguard, render
    from tests._helpers import changed_window
    spec, cam = job["spec"], job["cam"]
    fmt, sh = spec[3], spec[2]
    words, _ = _words(spec)
    pc = _clean_proj(spec, cam, job["cam_key"])
    sites = job.get("sites") or []
    w = [x.copy() for x in words] if sites or job.get("box_seed") is not None else words
    prims = sorted({int(s[2]) for s in sites})
    for f, c, p, b in sites:
        w[f][c, p] = formats.flip(w[f][c, p:p + 1], int(b))[0]
    clamps = 0
    if job.get("box_seed") is not None:
        lo, hi = _box_words(spec, job["box_seed"])
        w, clamps = oguard.guard_scene(w, lo, hi, fmt, fields=job.get("guard_fields", oguard.DEFAULT_FIELDS))
    if sites:
        pv = render.project(render.decode_scene(w, fmt), sh, cam)
    else:
        pv = pc
    win = job.get("window", "full")
    if win == "full":
        win = (0, 0, cam.width, cam.height)
    elif win == "changed":
        win = changed_window(pc, pv, prims, cam) if prims else None
    if win is None:   # no pixel can change
        return dict(image=None, amb=None, T=None, nonfinite=bool(np.any(pv["nonfinite_param"])), window=None,
                    clamps=int(clamps), prims=prims)
    out = render.render(pv, cam, window=win)
    return dict(image=out["image"], amb=out["amb"], T=out["T"], nonfinite=out["nonfinite"], window=out["window"],
                clamps=int(clamps), prims=prims)


class Pool:
    """A spawn-context process pool running run_job (no worker touches the GPU)."""

    def __init__(self, workers=None):
        n = workers or min(16, os.cpu_count() or 1)
        self.ex = ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn"))

    def map(self, jobs):
        return list(self.ex.map(run_job, jobs))

    def close(self):
        self.ex.shutdown(wait=True, cancel_futures=True)
