"""Pins for oracle.guard: Thm. 1 (identity on the clean model; a guarded
single flip stays within the in-box spread), Thm. 2 (guarded scales bounded
by exp(h)), and clamp counts recounted from the site list."""
import numpy as np
import pytest

from oracle import formats, guard
from paper_2606_21791_amd import synth


def _stored(scene, fmt):
    return [formats.store(f, fmt) for f in scene.fields]


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16"])
def test_thm1_identity_on_clean_model(fmt):
    sc = synth.make_scene(3000, seed=5, sh_degree=1)
    w = _stored(sc, fmt)
    lo, hi = [None] * 6, [None] * 6
    for f in guard.DEFAULT_FIELDS:
        lo[f], hi[f] = guard.box_global(w[f], fmt)
    g, n = guard.guard_scene(w, lo, hi, fmt)
    assert n == 0
    assert all(np.array_equal(a, b) for a, b in zip(g, w))
    # the box bounds are attained values of the model (min / max)
    for f in guard.DEFAULT_FIELDS:
        v = formats.decode(w[f], fmt)
        assert np.array_equal(formats.decode(lo[f], fmt), v.min(axis=1))
        assert np.array_equal(formats.decode(hi[f], fmt), v.max(axis=1))


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16"])
def test_thm1_single_flip_and_recount(fmt):
    sc = synth.make_scene(2000, seed=6, sh_degree=0)
    w = _stored(sc, fmt)
    W = formats.width(fmt)
    lo, hi = [None] * 6, [None] * 6
    for f in guard.DEFAULT_FIELDS:
        lo[f], hi[f] = guard.box_global(w[f], fmt)
    sites = synth.make_sites_uniform(sc.n, 0, 3000, seed=7, width_bits=W)
    for k in range(len(sites)):
        f, c, p, b = int(sites.field[k]), int(sites.comp[k]), int(sites.prim[k]), int(sites.bit[k])
        clean_w = w[f][c, p]
        x_w = formats.flip(np.array([clean_w]), b)[0]
        out, n = guard.clamp(np.array([[x_w]]), lo[f][c:c + 1], hi[f][c:c + 1], fmt)
        gv = formats.decode(out, fmt)[0, 0]
        cv = formats.decode(np.array([clean_w]), fmt)[0]
        xv = formats.decode(np.array([x_w]), fmt)[0]
        l, h = formats.decode(lo[f][c:c + 1], fmt)[0], formats.decode(hi[f][c:c + 1], fmt)[0]
        assert l <= gv <= h
        assert abs(gv - cv) <= h - l                     # Thm. 1 (ii)
        outside = np.isnan(xv) or xv < l or xv > h
        assert n == int(outside)                         # recount from the site
        if not outside:
            assert out[0, 0] == x_w                      # in-box values keep their bits
        if np.isnan(xv):
            assert out[0, 0] == lo[f][c]


def test_thm2_scale_bound_after_arbitrary_flips():
    sc = synth.make_scene(1500, seed=8)
    w = _stored(sc, "f32")
    lo, hi = [None] * 6, [None] * 6
    for f in guard.DEFAULT_FIELDS:
        lo[f], hi[f] = guard.box_global(w[f], "f32")
    sites = synth.make_sites_dose(sc.n, 0, 4000, seed=9, width_bits=32)
    bad = [x.copy() for x in w]
    for k in range(len(sites)):
        f, c, p, b = int(sites.field[k]), int(sites.comp[k]), int(sites.prim[k]), int(sites.bit[k])
        bad[f][c, p] = formats.flip(bad[f][c, p:p + 1], b)[0]
    g, n = guard.guard_scene(bad, lo, hi, "f32")
    s = np.exp(formats.decode(g[1], "f32"))
    assert np.all(s <= np.exp(formats.decode(hi[1], "f32"))[:, None])
    assert all(np.all(np.isfinite(formats.decode(g[f], "f32"))) for f in guard.DEFAULT_FIELDS)
    # the count is the number of guarded components that changed value class
    recount = 0
    for f in guard.DEFAULT_FIELDS:
        v = formats.decode(bad[f], "f32")
        l = formats.decode(lo[f], "f32")[:, None]
        h = formats.decode(hi[f], "f32")[:, None]
        recount += int(np.count_nonzero(np.isnan(v) | (v < l) | (v > h)))
    assert n == recount


def test_per_primitive_box_contains_clean_and_bounds_flips():
    sc = synth.make_scene(1000, seed=10)
    lo32, hi32 = synth.make_box_jitter(sc, seed=4)
    w = _stored(sc, "f32")
    lo = [None if a is None else formats.f32_words(a) for a in lo32]
    hi = [None if a is None else formats.f32_words(a) for a in hi32]
    g, n = guard.guard_scene(w, lo, hi, "f32")
    assert n == 0 and all(np.array_equal(a, b) for a, b in zip(g, w))
    for fmt in ("f16", "bf16"):                          # outward-rounded boxes still contain the cast
        ws = _stored(sc, fmt)
        lo_f = [None if a is None else formats.store(a, fmt, "rd") for a in lo32]
        hi_f = [None if a is None else formats.store(a, fmt, "ru") for a in hi32]
        g, n = guard.guard_scene(ws, lo_f, hi_f, fmt)
        assert n == 0


def test_zero_sign_tie_break_in_box():
    w = formats.f32_words(np.array([[0.0, -0.0, 0.0, -0.0]], np.float32))
    lo, hi = guard.box_global(w, "f32")
    assert lo[0] == 0x80000000 and hi[0] == 0
    out, n = guard.clamp(w, lo, hi, "f32")
    assert n == 0 and np.array_equal(out, w)


def test_health_alert():
    assert guard.health_alert(1, 0) and not guard.health_alert(0, 0) and not guard.health_alert(5, 5)
