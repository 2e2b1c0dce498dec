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


AMB_CAP = 1e-3           # largest fraction of ambiguous pixels a parity test accepts


def check_variant(img, m, ref, clean_ref, clean_gpu, amb_cap=AMB_CAP):
    """Pixel, PSNR and footprint parity of one variant (GPU image and record
    against the oracle's full frames of the variant and the clean scene);
    returns the ambiguous fraction."""
    amb = ref["amb"] | clean_ref["amb"]
    worst, amb_frac = compare_image(img, ref, clean_ref["amb"])
    assert worst <= PIXEL_TOL, worst
    assert amb_frac <= amb_cap, amb_frac
    assert bool(m["nonfinite"]) == ref["nonfinite"]
    ok = ~amb
    d_gpu = np.abs(img.astype(np.float64) - clean_gpu.astype(np.float64))
    d_ref = np.abs(ref["image"] - clean_ref["image"])
    # the record is what the image says (exact recount on the GPU image)
    dmax_gpu = d_gpu.max(axis=2)
    assert int(m["changed_px"]) == int(np.count_nonzero(dmax_gpu > LEVEL))
    assert abs(float(m["sse"]) - float(np.sum(d_gpu ** 2))) <= 1e-9 * max(1.0, float(np.sum(d_gpu ** 2)))
    # footprint: exact on pixels not within LEVEL_BAND of the level and not ambiguous
    dmax_ref = d_ref.max(axis=2)
    cmp = ok & (np.abs(dmax_ref - LEVEL) > LEVEL_BAND)
    assert np.array_equal((dmax_gpu > LEVEL)[cmp], (dmax_ref > LEVEL)[cmp])
    # PSNR over the non-ambiguous pixels of both frames
    mse_g = float(np.mean(d_gpu[ok] ** 2))
    mse_r = float(np.mean(d_ref[ok] ** 2))
    if mse_r == 0.0:
        assert mse_g == 0.0 or 10 * np.log10(1 / mse_g) > 69.95
    else:
        pr = 10 * np.log10(1 / mse_r)
        pg = 10 * np.log10(1 / mse_g) if mse_g > 0 else np.inf
        if pr <= 70.0:
            assert abs(pg - pr) <= PSNR_TOL_DB, (pg, pr)
        else:
            assert pg > 69.95
    return amb_frac


def ref_metrics(ref_img, clean_img, nonfinite, mask=None):
    return ometrics.frame_metrics(ref_img, clean_img, nonfinite, mask)


def support_window(proj, i, cam, pad=2.0):
    """Pixel window (x0, y0, x1, y1) holding every pixel centre that primitive
    i can reach (q <= 9 on the projection's conic), widened by `pad` pixels;
    None if the primitive is culled or its support misses the frame."""
    import math
    if not proj["valid"][i]:
        return None
    rx = math.sqrt(9.0 * proj["a"][i]) * 1.01 + pad
    ry = math.sqrt(9.0 * proj["c"][i]) * 1.01 + pad
    u, v = proj["u"][i], proj["v"][i]
    x0, x1 = max(0, math.floor(u - rx)), min(cam.width, math.ceil(u + rx) + 1)
    y0, y1 = max(0, math.floor(v - ry)), min(cam.height, math.ceil(v + ry) + 1)
    if x1 <= x0 or y1 <= y0:
        return None
    return (int(x0), int(y0), int(x1), int(y1))


def union_window(*wins):
    wins = [w for w in wins if w is not None]
    if not wins:
        return None
    return (min(w[0] for w in wins), min(w[1] for w in wins), max(w[2] for w in wins), max(w[3] for w in wins))


def splice_projection(proj, words, prims, fmt, sh_degree, cam):
    """The projection of a scene that differs from the projected one only in
    the primitives `prims`: those are projected alone and written into a copy
    of `proj`.  Projection treats every primitive on its own, so this equals
    projecting the whole corrupted scene (up to the rounding order of the
    library products)."""
    prims = np.unique(np.atleast_1d(prims).astype(np.int64))
    one = [w[:, prims] for w in words]
    q = orender.project(orender.decode_scene(one, fmt), sh_degree, cam)
    out = dict(proj)
    for k, v in proj.items():
        if isinstance(v, np.ndarray) and v.shape[:1] == (proj["n"],):
            v = v.copy()
            v[prims] = q[k]
            out[k] = v
    return out


def changed_window(clean_proj, var_proj, prims, cam):
    """Window outside which a variant whose corrupted primitives are `prims`
    equals the clean frame exactly: no pixel outside the old and new supports
    of those primitives has a different contributor list."""
    return union_window(*[support_window(p, int(i), cam) for i in np.atleast_1d(prims)
                          for p in (clean_proj, var_proj)])
