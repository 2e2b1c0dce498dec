"""Shared helpers of the test-suite: oracle renders of corrupted variants and
the element-wise comparison used by every GPU parity test."""
import numpy as np

from oracle import formats, guard as oguard, metrics as ometrics, render as orender

PIXEL_TOL = 2e-4          # absolute, on [0, 1] images
PSNR_TOL_DB = 0.05
LEVEL = 1.0 / 255.0
LEVEL_BAND = 1e-5         # footprint decisions within this of the level are not compared


def stored(scene, fmt):
    return [formats.store(f, fmt) for f in scene.fields]


def apply_sites(words, sites, idx):
    w = [x.copy() for x in words]
    for k in np.atleast_1d(idx):
        f, c, p, b = int(sites.field[k]), int(sites.comp[k]), int(sites.prim[k]), int(sites.bit[k])
        w[f][c, p] = formats.flip(w[f][c, p:p + 1], b)[0]
    return w


def oracle_render(words, fmt, sh_degree, cam):
    return orender.render(orender.project(orender.decode_scene(words, fmt), sh_degree, cam), cam)


def oracle_guarded(words, lo, hi, fmt):
    g, n = oguard.guard_scene(words, lo, hi, fmt)
    return g, n


def compare_image(gpu_img, ref, extra_amb=None):
    """Max |gpu - oracle| over non-ambiguous pixels, and the ambiguous fraction."""
    amb = ref["amb"].copy()
    if extra_amb is not None:
        amb |= extra_amb
    ok = ~amb
    err = np.abs(np.asarray(gpu_img, np.float64) - ref["image"])
    worst = float(np.max(err[ok])) if ok.any() else 0.0
    return worst, float(amb.mean())


def compare_metrics(m, ref_img, clean_img, amb, nonfinite):
    """Check one sg_metrics_t record against the oracle's definition.  Pixels
    ambiguous in either frame are excluded from the PSNR comparison and from
    the footprint count, as are pixels whose oracle delta is within
    LEVEL_BAND of the level."""
    ok = ~amb
    d = np.abs(ref_img - clean_img).max(axis=2)
    near = np.abs(d - LEVEL) <= LEVEL_BAND
    ref_changed = int(np.count_nonzero((d > LEVEL) & ok & ~near))
    return dict(ref_changed=ref_changed, n_amb=int(np.count_nonzero(amb | near)), nonfinite=bool(nonfinite))


def ref_metrics(ref_img, clean_img, nonfinite, mask=None):
    return ometrics.frame_metrics(ref_img, clean_img, nonfinite, mask)
