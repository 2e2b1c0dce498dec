"""GPU parity of the render path through the C ABI against the FP64 oracle:
clean frames, corrupted variants (incremental and full paths), guarded and
multi-upset variants, metrics; plus the internal invariants (incremental ==
full render bit for bit, tile-size invariance)."""
import numpy as np
import pytest

from oracle import formats, guard as oguard, metrics as om, render as orender
from paper_2606_21791_amd import synth

from ._helpers import PIXEL_TOL, LEVEL, apply_sites, check_variant as _check_variant, compare_image, \
    oracle_render, stored

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2606_21791_amd import binding
    return binding.Context(0)


def _batch(ctx, prep, sites, idx_groups, guard=0, box=None, mode=0, want_images=True):
    import torch
    from paper_2606_21791_amd import binding as b
    flat = np.concatenate([np.atleast_1d(g) for g in idx_groups]) if idx_groups else np.zeros(0, int)
    sa = b.sites_array(sites.field[flat], sites.comp[flat], sites.prim[flat], sites.bit[flat])
    counts = np.array([len(np.atleast_1d(g)) for g in idx_groups])
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]])
    va = b.variants_array(offs, counts, guard)
    B = len(idx_groups)
    H, W = prep.cam.height, prep.cam.width
    imgs = torch.zeros((B, H, W, 3), dtype=torch.float32, device="cuda") if want_images else None
    mt = b.metrics_tensor(B)
    ctx.render_batch(prep, sa, va, box=box, images=imgs, metrics=mt, mode=mode)
    torch.cuda.synchronize()
    return (imgs.cpu().numpy() if want_images else None), b.read_metrics(mt)


def test_clean_frame_parity_w1_and_full_render_equal(ctx):
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(5000, seed=1)
    cam = synth.make_camera(256, 256)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam)
    frame = prep.frame().cpu().numpy()
    ref = oracle_render(stored(sc, "f32"), "f32", 0, cam)
    worst, amb = compare_image(frame, ref)
    print(f"W1 clean: max err {worst:.3g}, ambiguous {amb:.2e}, instances {prep.instances()}")
    assert worst <= PIXEL_TOL and amb <= 2e-4
    img = torch.zeros((256, 256, 3), dtype=torch.float32, device="cuda")
    ctx.render(ds, cam, image=img)
    torch.cuda.synchronize()
    assert np.array_equal(img.cpu().numpy(), frame)


def test_w1_variants_parity(ctx):
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(5000, seed=1)
    cam = synth.make_camera(256, 256)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam)
    clean_gpu = prep.frame().cpu().numpy()
    words = stored(sc, "f32")
    clean_ref = oracle_render(words, "f32", 0, cam)
    sites = synth.make_sites_uniform(sc.n, 0, 256, seed=11)
    # every sign and top exponent bit among the W1 sites plus a spread of others
    pick = sorted(set(np.nonzero(sites.bit >= 29)[0][:24].tolist()) | set(range(0, 256, 8)))
    imgs, ms = _batch(ctx, prep, sites, [np.array([k]) for k in pick])
    for j, k in enumerate(pick):
        ref = oracle_render(apply_sites(words, sites, k), "f32", 0, cam)
        _check_variant(imgs[j], ms[j], ref, clean_ref, clean_gpu)


@pytest.mark.parametrize("case", ["hidden", "single", "frame13x7", "frame1x1"])
def test_degenerate_scenes(ctx, case):
    """Degenerate scenes: every primitive behind the camera (no tile
    instances, a background frame), a one-primitive scene, and frames smaller
    than one tile (13 x 7 and 1 x 1 pixels).  Variants that bring hidden
    primitives into view, flips of every component of the single primitive
    and stratified sites of the small frames match the oracle; the
    incremental and full paths give the same images and the campaign the
    same records."""
    import torch
    from paper_2606_21791_amd import binding as b
    cam = synth.make_camera(96, 64)
    if case.startswith("frame"):
        w, h = (13, 7) if case == "frame13x7" else (1, 1)
        cam = synth.make_camera(w, h)
        sc = synth.make_scene(60, seed=65)
        sc.fields[1][:] += np.float32(2.0)   # splats larger than the small frame's pixels
        sh = 0
        sites = synth.make_sites_stratified(sc.n, 0, 32, seed=66, width_bits=32, fields=(0, 1, 2, 3, 4))
    elif case == "hidden":
        sc = synth.make_scene(400, seed=61)
        # z in [-4.25, -3.75]: behind the camera, which sits at z = -3
        sc.fields[0][2, :] = np.float32(-4.0) + np.float32(0.25) * sc.fields[0][2, :]
        sh = 0
        # the sign bit of z puts a primitive in front of the camera; the top
        # exponent bit of z (value 4 = 2^2) sends it towards z = 0
        rng = np.random.default_rng(63)
        prims = rng.choice(sc.n, 16, replace=False)
        sites = synth._mk_sites(np.zeros(32), np.full(32, 2), np.concatenate([prims, prims]),
                                np.concatenate([np.full(16, 31), np.full(16, 30)]))
        extra = synth.make_sites_uniform(sc.n, 0, 24, seed=64)
        sites = synth._mk_sites(np.concatenate([sites.field, extra.field]), np.concatenate([sites.comp, extra.comp]),
                                np.concatenate([sites.prim, extra.prim]), np.concatenate([sites.bit, extra.bit]))
    else:
        sc = synth.make_scene(1, seed=62, sh_degree=1)
        sc.fields[0][:, 0] = [0.1, -0.05, 0.0]
        sc.fields[1][:, 0] = [-1.2, -1.6, -1.4]
        sc.fields[3][:, 0] = [2.0]
        sh = 1
        comps = synth.field_components(1)
        f, c, bits = [], [], []
        for fld in range(6):
            for comp in range(comps[fld]):
                for bit in (31, 30, 26, 23, 20, 10):
                    f.append(fld); c.append(comp); bits.append(bit)
        sites = synth._mk_sites(f, c, np.zeros(len(f)), bits)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam)
    clean_gpu = prep.frame().cpu().numpy()
    words = stored(sc, "f32")
    clean_ref = oracle_render(words, "f32", sh, cam)
    if case == "hidden":
        assert prep.instances() == 0
        assert np.all(clean_gpu == 1.0) and np.all(clean_ref["image"] == 1.0)
    elif case.startswith("frame"):
        worst, _ = compare_image(clean_gpu, clean_ref)
        assert worst <= PIXEL_TOL, worst
    else:
        assert prep.instances() > 0 and np.any(clean_gpu < 1.0)
        worst, _ = compare_image(clean_gpu, clean_ref)
        assert worst <= PIXEL_TOL, worst
    groups = [np.array([k]) for k in range(len(sites))]
    inc, mi = _batch(ctx, prep, sites, groups, mode=0)
    full, mf = _batch(ctx, prep, sites, groups, mode=1)
    assert np.array_equal(inc, full)
    for key in ("changed_px", "max_abs", "nonfinite"):
        assert np.array_equal(mi[key], mf[key]), key
    visible = 0
    for k in range(len(sites)):
        ref = oracle_render(apply_sites(words, sites, k), "f32", sh, cam)
        _check_variant(inc[k], mi[k], ref, clean_ref, clean_gpu)
        visible += int(mi[k]["changed_px"] > 0)
    assert visible >= (1 if case == "frame1x1" else 8), visible
    sa = b.sites_array(sites.field, sites.comp, sites.prim, sites.bit)
    va = b.variants_array(np.arange(len(sites)), np.ones(len(sites), np.uint32))
    got = b.metrics_tensor(len(sites))
    ctx.campaign(prep, sa, va, got, batch=8, streams=3, threads=2)
    torch.cuda.synchronize()
    G = b.read_metrics(got)
    for key in mi.dtype.names:
        assert np.array_equal(G[key], mi[key]), key


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16"])
def test_incremental_equals_full_render(ctx, fmt):
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(6741, seed=3, sh_degree=3)
    cam = synth.make_camera(200, 160)
    ds = b.DeviceScene.upload(ctx, sc, fmt)
    prep = ctx.prepare(ds, cam)
    W = formats.width(fmt)
    sites = synth.make_sites_stratified(sc.n, 3, 2 * W, seed=12, width_bits=W)
    groups = [np.array([k]) for k in range(0, len(sites), 3)]
    groups += [np.array([0, 1, 2]), np.array([5, 6])]          # multi-site variants
    inc, mi = _batch(ctx, prep, sites, groups, mode=0)
    full, mf = _batch(ctx, prep, sites, groups, mode=1)
    assert np.array_equal(inc, full)
    for key in ("changed_px", "max_abs", "nonfinite"):
        assert np.array_equal(mi[key], mf[key]), key
    # the same per-pixel terms summed over different tile sets: equal up to the order of the double sum
    assert np.allclose(mi["sse"], mf["sse"], rtol=1e-12, atol=0.0)
    assert np.all(mi["path"] == 0) and np.all(mf["path"] == 1)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_elongated_footprints_equal_full_render(ctx, tile):
    """Exponent flips of one log-scale component stretch a Gaussian along one
    axis, into a footprint whose tile rectangle holds many tiles the ellipse
    never reaches.  The work-item listing drops those tiles (no changed record
    reaches a pixel centre of them) and the items drop the pixels that cannot
    change: the images and records still equal the full renders of the
    corrupted scenes bit for bit."""
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(6741, seed=5, sh_degree=1)
    cam = synth.make_camera(400, 400)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam, b.raster_struct(tile=tile))
    rng = np.random.default_rng(23)
    n = 96
    sites = synth.Sites(np.full(n, synth.LOG_SCALES, np.uint8), rng.integers(0, 3, n).astype(np.uint16),
                        rng.integers(0, sc.n, n).astype(np.uint32), rng.integers(23, 31, n).astype(np.uint8))
    groups = [np.array([k]) for k in range(n)] + [np.array([0, 1]), np.array([2, 3, 4])]
    inc, mi = _batch(ctx, prep, sites, groups, mode=0)
    full, mf = _batch(ctx, prep, sites, groups, mode=1)
    assert np.array_equal(inc, full)
    for key in ("changed_px", "max_abs", "nonfinite"):
        assert np.array_equal(mi[key], mf[key]), key
    assert np.allclose(mi["sse"], mf["sse"], rtol=1e-12, atol=0.0)
    assert (mi["changed_px"] > 0).sum() > n // 4          # the flips do change the frame
    assert mi["dirty_tiles"].max() > (400 // tile) ** 2 // 8   # and some rectangles hold many tiles


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_resume_spacing_invariance(ctx, tile):
    """Skipping pixels that stopped before the first changed list entry and
    resuming the others from clean checkpoints gives the same images and the
    same records as walking every merged list from its start, for every
    checkpoint spacing, and evaluates fewer entries."""
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(6741, seed=3, sh_degree=3)
    cam = synth.make_camera(200, 160)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    sites = synth.make_sites_stratified(sc.n, 3, 96, seed=17, width_bits=32)
    groups = [np.array([k]) for k in range(len(sites))]
    groups += [np.array([0, 1, 2]), np.array([5, 6]), np.array([7, 7])]
    out = {}
    try:
        for g in (0, 16, 64, 4096):
            ctx.set_resume(g)
            prep = ctx.prepare(ds, cam, b.raster_struct(tile=tile))
            out[g] = _batch(ctx, prep, sites, groups)
    finally:
        ctx.set_resume(64)
    img0, m0 = out[0]
    for g in (16, 64, 4096):
        img, m = out[g]
        assert np.array_equal(img, img0), g
        for key in ("changed_px", "max_abs", "nonfinite", "dirty_tiles"):
            assert np.array_equal(m[key], m0[key]), (g, key)
        # the same per-tile terms; tiles that cannot change get no item here,
        # so the double sums group them differently
        assert np.allclose(m["sse"], m0["sse"], rtol=1e-12, atol=0.0), g
        assert m["evals"].sum() < m0["evals"].sum(), g
    full, mf = _batch(ctx, prep, sites, groups, mode=1)
    assert np.array_equal(out[64][0], full)


@pytest.mark.parametrize("n", [14000, 40000])
def test_long_tile_lists(ctx, n):
    """Lists longer than one LDS sort (thousands of entries per 32x32 tile,
    cut into 4,096-key chunks: up to about 12,000 entries and two merge passes
    at n=14,000, about 34,000 and four passes at n=40,000) give the same
    frame as 8x8 tiles (lists within one LDS sort at n=14,000; up to about
    12,000 entries at n=40,000) and agree with the oracle on every decided
    pixel."""
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(n, seed=29)
    sc.fields[1][:] += 1.5                    # larger primitives: each covers several tiles
    cam = synth.make_camera(96, 96)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    frames, inst = {}, {}
    for t in (8, 32):
        p = ctx.prepare(ds, cam, b.raster_struct(tile=t))
        frames[t] = p.frame().cpu().numpy()
        inst[t] = p.instances()
    # 9 tiles of 32x32 with a mean list near or above one LDS sort; the
    # central tiles hold about 2.5 times the mean
    assert inst[32] / 9 > 3000
    assert np.array_equal(frames[8], frames[32])
    ref = oracle_render(stored(sc, "f32"), "f32", 0, cam)
    worst, amb = compare_image(frames[32], ref)
    print(f"long lists n={n}: max err {worst:.3g}, ambiguous {amb:.2e}", flush=True)
    assert worst <= PIXEL_TOL and amb <= 2e-3, (worst, amb)


def test_tile_size_invariance(ctx):
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(6000, seed=13, sh_degree=1)
    cam = synth.make_camera(160, 120)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    frames = [ctx.prepare(ds, cam, b.raster_struct(tile=t)).frame().cpu().numpy() for t in (8, 16, 32)]
    assert np.array_equal(frames[0], frames[1]) and np.array_equal(frames[1], frames[2])


def test_tile_grids_beyond_lds(ctx):
    """At 1100 x 1100 with 8x8 tiles the tile-count difference grid has
    139 x 139 = 19,321 entries and there are 18,769 tiles: the projection adds
    rectangles to the grid in global memory (one primitive per thread instead
    of a grid-stride loop over an LDS grid), the tile prefix sums the grid in
    global memory, and instances are emitted one thread per primitive.  The
    frame equals the one from 16x16 tiles (LDS grid, chunked emission) bit for
    bit and agrees with the oracle on three windows: the centre, one near the
    corner where the scene ends, and one reaching the frame's last row and
    column of tiles."""
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(20000, seed=41, sh_degree=1)
    sc.fields[1][:] -= 1.0                    # smaller primitives: many small tiles in use
    cam = synth.make_camera(1100, 1100)
    assert (1100 // 8 + 2) ** 2 > 16384 and (1100 // 8 + 1) ** 2 > 16384
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    frames = {t: ctx.prepare(ds, cam, b.raster_struct(tile=t)).frame().cpu().numpy() for t in (8, 16)}
    assert np.array_equal(frames[8], frames[16])
    proj = orender.project(orender.decode_scene(stored(sc, "f32"), "f32"), 1, cam)
    for win in ((500, 500, 564, 564), (960, 960, 1024, 1024), (980, 980, 1100, 1100)):
        ref = orender.render(proj, cam, window=win)
        x0, y0, x1, y1 = ref["window"]
        worst, amb = compare_image(frames[8][y0:y1, x0:x1], ref)
        print(f"window {win}: max err {worst:.3g}, ambiguous {amb:.2e}", flush=True)
        assert worst <= PIXEL_TOL and amb <= 2e-3, (win, worst, amb)


def test_incremental_on_tile_grids_beyond_lds(ctx):
    """The incremental path over 18,769 tiles of 8x8 (1100 x 1100): its frames
    equal full renders of the same variants bit for bit, and a pipelined
    campaign gives the records of sg_render_batch."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(20000, seed=41, sh_degree=1)
    sc.fields[1][:] -= 1.0
    cam = synth.make_camera(1100, 1100)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam, b.raster_struct(tile=8))
    sites = synth.make_sites_stratified(sc.n, 1, 32, seed=47, width_bits=32)
    groups = [np.array([k]) for k in range(0, len(sites), max(1, len(sites) // 10))][:10]
    groups.append(np.array([1, 2, 3]))                         # a multi-site variant
    inc, mi = _batch(ctx, prep, sites, groups, mode=0)
    full, mf = _batch(ctx, prep, sites, groups, mode=1)
    assert np.array_equal(inc, full)
    for key in ("changed_px", "max_abs", "nonfinite"):
        assert np.array_equal(mi[key], mf[key]), key
    assert np.all(mi["path"] == 0) and mi["dirty_tiles"].max() > 1
    flat = np.concatenate(groups)
    sa = b.sites_array(sites.field[flat], sites.comp[flat], sites.prim[flat], sites.bit[flat])
    counts = np.array([len(g) for g in groups])
    va = b.variants_array(np.concatenate([[0], np.cumsum(counts)[:-1]]), counts)
    got = b.metrics_tensor(len(va))
    ctx.campaign(prep, sa, va, got, batch=4, streams=2, threads=1)
    torch.cuda.synchronize()
    G = b.read_metrics(got)
    for key in mi.dtype.names:
        assert np.array_equal(G[key], mi[key]), key


def test_guarded_and_multi_upset_variants(ctx):
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(4000, seed=14)
    cam = synth.make_camera(128, 128)
    lo32, hi32 = synth.make_box_jitter(sc, seed=4)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    box = b.Box.per_prim(ctx, lo32, hi32, "f32")
    prep = ctx.prepare(ds, cam)
    clean_gpu = prep.frame().cpu().numpy()
    words = stored(sc, "f32")
    lo = [None if a is None else formats.f32_words(a) for a in lo32]
    hi = [None if a is None else formats.f32_words(a) for a in hi32]
    clean_ref = oracle_render(words, "f32", 0, cam)
    single = synth.make_sites_stratified(sc.n, 0, 32, seed=15, width_bits=32, fields=(1,))   # log-scale bits
    dose = synth.make_sites_dose(sc.n, 0, 300, seed=16, width_bits=32)
    allsites = synth.Sites(*(np.concatenate([a, c]) for a, c in zip(
        (single.field, single.comp, single.prim, single.bit), (dose.field, dose.comp, dose.prim, dose.bit))))
    groups = [np.array([k]) for k in range(32)] + [np.arange(32, 32 + 300)]
    for guard in (0, 1):
        imgs, ms = _batch(ctx, prep, allsites, groups, guard=guard, box=box)
        for j, g in enumerate(groups):
            w = apply_sites(words, allsites, g)
            n_cl = 0
            if guard:
                w, n_cl = oguard.guard_scene(w, lo, hi, "f32")
            ref = oracle_render(w, "f32", 0, cam)
            _check_variant(imgs[j], ms[j], ref, clean_ref, clean_gpu)
            assert int(ms[j]["clamps"]) == (n_cl if guard else 0)
        assert ms[-1]["path"] == 1 and np.all(ms["path"][:-1] == 0)
        if guard:   # Thm. 2: no guarded single flip explodes a primitive across the frame
            assert np.max(ms["footprint"][:32]) < 0.2


def test_campaign_matches_batches(ctx):
    """sg_campaign over several streams and host threads gives, per variant,
    exactly the records of sg_render_batch on the same batches one by one,
    with guarded, multi-site and full-path variants and a ragged last batch;
    without the full-path variant the campaign takes its pipelined path (the
    metrics of a batch reduced by the next prep on its stream), which must
    give the same records, also on campaigns back to back and with fewer
    variants than one batch."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(4000, seed=14, sh_degree=1)
    cam = synth.make_camera(160, 128)
    lo32, hi32 = synth.make_box_jitter(sc, seed=4)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    box = b.Box.per_prim(ctx, lo32, hi32, "f32")
    prep = ctx.prepare(ds, cam)
    single = synth.make_sites_stratified(sc.n, 1, 40, seed=19, width_bits=32)
    dose = synth.make_sites_dose(sc.n, 1, 12, seed=20, width_bits=32)      # 12 primitives: full path
    sites = synth.Sites(*(np.concatenate([a, c]) for a, c in zip(
        (single.field, single.comp, single.prim, single.bit), (dose.field, dose.comp, dose.prim, dose.bit))))
    ns = len(single.prim)
    sa = b.sites_array(sites.field, sites.comp, sites.prim, sites.bit)
    offs = list(range(ns)) + [0, ns]
    cnts = [1] * ns + [3, len(dose.prim)]
    guard = np.array([(k % 3 == 0) for k in range(len(offs))], np.uint32)
    va = b.variants_array(np.array(offs), np.array(cnts), 0)
    va["guard"] = guard
    B = 7
    keys = ("sse", "changed_px", "max_abs", "nonfinite", "dirty_tiles", "clamps", "path", "evals",
            "predicted_regions", "rendered_regions")

    def batches(vs):
        ref = []
        for v0 in range(0, len(vs), B):
            mt = b.metrics_tensor(len(vs[v0:v0 + B]))
            ctx.render_batch(prep, sa, vs[v0:v0 + B], box=box, metrics=mt)
            ref.append(b.read_metrics(mt))
        return np.concatenate(ref)

    ref = batches(va)
    # a variant without sites renders the clean frame
    empty = b.variants_array(np.array([0]), np.array([0]), 0)
    va_e = np.concatenate([va[:-1], empty])
    ref_e = batches(va_e)
    assert ref_e["sse"][-1] == 0 and ref_e["dirty_tiles"][-1] == 0
    for vs, r in ((va, ref), (va[:-1], ref[:-1]), (va[:5], ref[:5]), (va_e, ref_e)):
        for streams, threads in ((1, 1), (4, 2), (5, 3)):
            mt = b.metrics_tensor(len(vs))
            ctx.campaign(prep, sa, vs, mt, box=box, batch=B, streams=streams, threads=threads)
            torch.cuda.synchronize()
            got = b.read_metrics(mt)
            for key in keys:
                assert np.array_equal(got[key], r[key]), (len(vs), streams, threads, key)
    assert ref["path"][-1] == 1 and np.all(ref["path"][:-1] == 0)
    with pytest.raises(b.SgError):
        bad = va.copy()
        bad["site_off"][3] = len(sa)
        ctx.campaign(prep, sa, bad, b.metrics_tensor(len(va)), box=box, batch=B)


def test_campaign_scenes_of_uneven_size(ctx):
    """Variants of three scenes of uneven size (primitive counts, frame sizes,
    formats, SH degrees) mixed in one campaign share its launches: every
    record equals sg_render_batch's on the variant's own scene, guarded
    variants included; invalid scene indices and sites are rejected."""
    import torch
    from paper_2606_21791_amd import binding as b
    specs = [(6741, 1, "f32", 200, 160), (2500, 0, "bf16", 96, 64), (12000, 3, "f16", 256, 144)]
    preps, boxes, site_sets = [], [], []
    for j, (n, sh, fmt, w, h) in enumerate(specs):
        sc = synth.make_scene(n, seed=70 + j, sh_degree=sh)
        ds = b.DeviceScene.upload(ctx, sc, fmt)
        preps.append(ctx.prepare(ds, synth.make_camera(w, h)))
        preps[-1]._ds = ds   # keeps the scene's device arrays alive with its prepared state
        W = formats.width(fmt)
        if j == 0:
            lo, hi = synth.make_box_jitter(sc, seed=75)
            boxes.append(b.Box.per_prim(ctx, lo, hi, fmt))
        else:
            boxes.append(None)
        site_sets.append(synth.make_sites_stratified(n, sh, 2 * W, seed=80 + j, width_bits=W,
                                                     fields=(0, 1, 2, 3, 4)))
    # one shared site array; each variant one site of its own scene, interleaved
    cat = lambda key: np.concatenate([getattr(t, key) for t in site_sets])
    sa = b.sites_array(cat("field"), cat("comp"), cat("prim"), cat("bit"))
    base = np.cumsum([0] + [len(t.prim) for t in site_sets])
    rng = np.random.default_rng(77)
    scene_of = rng.integers(0, 3, size=150).astype(np.uint16)
    off = np.array([base[k] + rng.integers(0, len(site_sets[k].prim)) for k in scene_of])
    va = b.variants_array(off, np.ones(len(off), np.uint32))
    va["guard"] = (scene_of == 0) & (np.arange(len(off)) % 2 == 1)
    got = b.metrics_tensor(len(va))
    ctx.campaign_scenes(preps, sa, va, scene_of, got, boxes=boxes, batch=8, streams=5, threads=2)
    torch.cuda.synchronize()
    G = b.read_metrics(got)
    for k in range(3):
        # the reference: sg_render_batch on the scene's own sites (it checks every site it is given)
        idx = np.nonzero(scene_of == k)[0]
        t = site_sets[k]
        vk = va[idx].copy()
        vk["site_off"] -= np.uint32(base[k])
        mt = b.metrics_tensor(len(idx))
        ctx.render_batch(preps[k], b.sites_array(t.field, t.comp, t.prim, t.bit), vk, box=boxes[k], metrics=mt)
        ref = b.read_metrics(mt)
        assert np.all(ref["path"] == 0)
        for key in ref.dtype.names:
            assert np.array_equal(G[key][idx], ref[key]), (k, key)
    assert np.any(G["changed_px"] > 0) and np.any(G["clamps"] > 0)
    assert len(set(G["n_pixels"].tolist())) == 3
    with pytest.raises(b.SgError):
        bad = scene_of.copy()
        bad[4] = 3
        ctx.campaign_scenes(preps, sa, va, bad, b.metrics_tensor(len(va)), boxes=boxes)
    with pytest.raises(b.SgError):
        # a scene-2 site (component of SH degree 3) given to a variant of the SH0 scene
        wrong = scene_of.copy()
        wrong[:] = 1
        ctx.campaign_scenes(preps, sa, va, wrong, b.metrics_tensor(len(va)), boxes=boxes)


@pytest.mark.parametrize("tile", [8, 32])
def test_campaign_other_tile_sizes(ctx, tile):
    """The pipelined campaign at 8 x 8 and 32 x 32 tiles (one and sixteen
    waves per workgroup) gives the records of sg_render_batch at that tile
    size, guarded variants and a ragged last batch included."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(3000, seed=44, sh_degree=1)
    cam = synth.make_camera(150, 110)
    lo32, hi32 = synth.make_box_jitter(sc, seed=5)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    box = b.Box.per_prim(ctx, lo32, hi32, "f32")
    prep = ctx.prepare(ds, cam, b.raster_struct(tile=tile))
    s = synth.make_sites_stratified(sc.n, 1, 12, seed=45, width_bits=32)
    sa = b.sites_array(s.field, s.comp, s.prim, s.bit)
    n = len(sa)
    va = b.variants_array(np.arange(n), np.ones(n, np.uint32))
    va["guard"] = np.arange(n) % 2
    B = 10   # 72 variants: a last batch of 2
    ref = []
    for v0 in range(0, n, B):
        mt = b.metrics_tensor(len(va[v0:v0 + B]))
        ctx.render_batch(prep, sa, va[v0:v0 + B], box=box, metrics=mt)
        ref.append(b.read_metrics(mt))
    ref = np.concatenate(ref)
    got = b.metrics_tensor(n)
    ctx.campaign(prep, sa, va, got, box=box, batch=B, streams=3, threads=2)
    torch.cuda.synchronize()
    G = b.read_metrics(got)
    for key in ref.dtype.names:
        assert np.array_equal(G[key], ref[key]), (tile, key)
    assert G["dirty_tiles"].max() > 1 and np.all(G["path"] == 0)


def test_campaign_largest_batch(ctx):
    """Batches of SG_MAX_BATCH (2,048) variants, in a campaign and in
    sg_render_batch, give the same records (a full batch and a ragged one)."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(2500, seed=47)
    cam = synth.make_camera(64, 48)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam)
    s = synth.make_sites_stratified(sc.n, 0, 64, seed=48, width_bits=32, fields=(0, 1, 2, 3, 4))
    sa = b.sites_array(s.field, s.comp, s.prim, s.bit)
    n = 2048 + 52
    va = b.variants_array(np.arange(n) % len(sa), np.ones(n, np.uint32))
    ref = []
    for v0 in range(0, n, 2048):
        mt = b.metrics_tensor(len(va[v0:v0 + 2048]))
        ctx.render_batch(prep, sa, va[v0:v0 + 2048], metrics=mt)
        ref.append(b.read_metrics(mt))
    ref = np.concatenate(ref)
    # the full batch's variants walk items found by a search of the offsets
    # in global memory: the full-render path gives the same records
    mf = b.metrics_tensor(2048)
    ctx.render_batch(prep, sa, va[:2048], metrics=mf, mode=b.SG_FULL)
    F = b.read_metrics(mf)
    for key in ("changed_px", "max_abs", "nonfinite"):
        assert np.array_equal(F[key], ref[key][:2048]), key
    assert np.allclose(F["sse"], ref["sse"][:2048], rtol=1e-12, atol=0.0)
    got = b.metrics_tensor(n)
    ctx.campaign(prep, sa, va, got, batch=2048, streams=2, threads=1)
    torch.cuda.synchronize()
    G = b.read_metrics(got)
    for key in ref.dtype.names:
        assert np.array_equal(G[key], ref[key]), key
    with pytest.raises(b.SgError):
        ctx.campaign(prep, sa, va, got, batch=2049)


def test_campaign_across_prepass_chunks(ctx):
    """A campaign longer than one pre-pass chunk (524,288 variants) gives the
    same records as the same variants in two campaigns that each fit in one
    chunk: the chunk offsets of the states, the batches and the records are
    consistent, with a ragged last batch."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(1500, seed=41)
    cam = synth.make_camera(48, 40)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam)
    s = synth.make_sites_stratified(sc.n, 0, 64, seed=42, width_bits=32, fields=(0, 1, 2, 3, 4))
    sa = b.sites_array(s.field, s.comp, s.prim, s.bit)
    n = (1 << 19) + 1000 + 5
    va = b.variants_array(np.arange(n) % len(sa), np.ones(n, np.uint32))
    whole = b.metrics_tensor(n)
    ctx.campaign(prep, sa, va, whole, batch=32, streams=8, threads=2)
    cut = 300_000
    first, second = b.metrics_tensor(cut), b.metrics_tensor(n - cut)
    ctx.campaign(prep, sa, va[:cut], first, batch=32, streams=8, threads=2)
    ctx.campaign(prep, sa, va[cut:], second, batch=32, streams=8, threads=2)
    torch.cuda.synchronize()
    got = b.read_metrics(whole)
    ref = np.concatenate([b.read_metrics(first), b.read_metrics(second)])
    for key in ref.dtype.names:
        assert np.array_equal(got[key], ref[key]), key
    # a variant's record depends only on its site
    same = va["site_off"] == va["site_off"][0]
    assert np.all(got["sse"][same] == got["sse"][0]) and same.sum() > 100


def test_autotune_and_cache(ctx, tmp_path):
    """The autotuner returns a valid configuration, caches it (a second call
    is a hit and measures nothing), leaves the context's settings alone, and
    the tuned configuration gives the same records as the defaults."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(6741, seed=3, sh_degree=3)
    cam = synth.make_camera(200, 160)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    sites = synth.make_sites_stratified(sc.n, 3, 64, seed=23, width_bits=32)
    sa = b.sites_array(sites.field, sites.comp, sites.prim, sites.bit)
    cache = str(tmp_path / "tune.jsonl")
    t = ctx.autotune(ds, cam, sa[:512], max_batch=128, cache=cache)
    assert t["from_cache"] == 0 and t["trials"] >= 10 and t["inj_per_s"] > 0
    assert t["tile"] in (8, 16, 32) and t["batch"] in (32, 64, 128) and t["resume"] in (16, 32, 64, 128, 256)
    assert 1 <= t["threads"] <= t["streams"] and t["wgs_per_cu"] in (1, 2, 4, 8) and t["graphs"] == 0
    t2 = ctx.autotune(ds, cam, sa[:512], max_batch=128, cache=cache)
    assert t2["from_cache"] == 1 and t2["trials"] == 0
    assert {k: t2[k] for k in ("tile", "batch", "streams", "threads", "wgs_per_cu", "resume", "graphs")} == \
        {k: t[k] for k in ("tile", "batch", "streams", "threads", "wgs_per_cu", "resume", "graphs")}
    tf = ctx.autotune(ds, cam, sa[:512], fixed_batch=32, cache=cache)
    assert tf["batch"] == 32 and tf["from_cache"] == 0
    with pytest.raises(b.SgError):
        ctx.autotune(ds, cam, sa[:10])
    n = len(sa)
    va = b.variants_array(np.arange(n), np.ones(n, np.uint32))
    ref = b.metrics_tensor(n)
    prep = ctx.prepare(ds, cam)
    ctx.campaign(prep, sa, va, ref)
    tuned = b.Context(0)
    tuned.apply_tune(t)
    prep_t = tuned.prepare(ds, cam, b.raster_struct(tile=t["tile"]))
    got = b.metrics_tensor(n)
    tuned.campaign(prep_t, sa, va, got, batch=t["batch"], streams=t["streams"], threads=t["threads"])
    torch.cuda.synchronize()
    r, g = b.read_metrics(ref), b.read_metrics(got)
    for key in ("sse", "changed_px", "max_abs", "nonfinite"):
        assert np.array_equal(r[key], g[key]) or key == "sse" and np.allclose(r[key], g[key], rtol=1e-12, atol=0), key


def test_k_views_pooling(ctx):
    """K views per injection (Def. 1: footprint averaged over the views): the
    per-view records equal single-view batches exactly, the pooled record is
    the pooling of the per-view ones, and a K-view campaign over several
    streams equals the batch-by-batch calls."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(4000, seed=14, sh_degree=1)
    cams = synth.make_orbit_cameras(3, 96, 80)
    lo32, hi32 = synth.make_box_jitter(sc, seed=4)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    box = b.Box.per_prim(ctx, lo32, hi32, "f32")
    preps = [ctx.prepare(ds, c) for c in cams]
    single = synth.make_sites_stratified(sc.n, 1, 20, seed=31, width_bits=32)
    dose = synth.make_sites_dose(sc.n, 1, 12, seed=32, width_bits=32)
    sites = synth.Sites(*(np.concatenate([a, c]) for a, c in zip(
        (single.field, single.comp, single.prim, single.bit), (dose.field, dose.comp, dose.prim, dose.bit))))
    ns = len(single.prim)
    sa = b.sites_array(sites.field, sites.comp, sites.prim, sites.bit)
    va = b.variants_array(np.array(list(range(ns)) + [0, ns]), np.array([1] * ns + [3, len(dose.prim)]), 0)
    va["guard"] = np.arange(len(va)) % 2
    B, K = len(va), len(preps)
    pooled, per_view = b.metrics_tensor(B), b.metrics_tensor(K * B)
    ctx.render_batch_views(preps, sa, va, pooled, per_view=per_view, box=box)
    torch.cuda.synchronize()
    P, V = b.read_metrics(pooled), b.read_metrics(per_view).reshape(K, B)
    for k in range(K):
        mt = b.metrics_tensor(B)
        ctx.render_batch(preps[k], sa, va, box=box, metrics=mt)
        ref = b.read_metrics(mt)
        for key in ref.dtype.names:
            assert np.array_equal(V[k][key], ref[key]), (k, key)
    sse = V["sse"][0].copy()
    for k in range(1, K):
        sse = sse + V["sse"][k]
    assert np.array_equal(P["sse"], sse)
    for key in ("changed_px", "dirty_tiles", "n_pixels", "evals"):
        assert np.array_equal(P[key], V[key].sum(axis=0)), key
    assert np.array_equal(P["max_abs"], V["max_abs"].max(axis=0))
    assert np.array_equal(P["nonfinite"], V["nonfinite"].max(axis=0))
    assert np.array_equal(P["clamps"], V["clamps"][0])
    for key in ("predicted_regions", "rendered_regions"):
        assert np.array_equal(P[key], np.bitwise_or.reduce(V[key], axis=0)), key
    foot = (V["changed_px"] / V["n_pixels"]).mean(axis=0)
    assert np.array_equal(P["footprint"], foot.astype(np.float32))
    assert np.allclose(P["mse"], sse / (3.0 * V["n_pixels"].sum(axis=0)), rtol=1e-15, atol=0)
    assert np.array_equal(P["catastrophic"], ((P["nonfinite"] > 0) | (foot > 0.01)).astype(np.uint32))
    assert P["path"][-1] == 1 and V["n_pixels"][0][0] == 96 * 80
    # With the full-path variant the campaign renders batch by batch.
    # Without it, the pipelined campaign renders the K views of a batch in
    # the same launches; views of different sizes, and batches whose
    # variant-views exceed one launch (B * K > 2,048), run view after view.
    cams2 = synth.make_orbit_cameras(2, 96, 80) + [synth.make_camera(64, 48)]
    preps2 = [ctx.prepare(ds, c) for c in cams2]
    for pp, vs, bsz in ((preps, va, 7), (preps, va[:-1], 7), (preps2, va[:-1], 7), (preps, va[:-1], 700)):
        got = b.metrics_tensor(len(vs))
        ctx.campaign(pp, sa, vs, got, box=box, batch=bsz, streams=4, threads=2)
        torch.cuda.synchronize()
        G = b.read_metrics(got)
        ref = []
        for v0 in range(0, len(vs), bsz):
            mt = b.metrics_tensor(len(vs[v0:v0 + bsz]))
            ctx.render_batch_views(pp, sa, vs[v0:v0 + bsz], mt, box=box)
            ref.append(b.read_metrics(mt))
        ref = np.concatenate(ref)
        for key in ref.dtype.names:
            assert np.array_equal(G[key], ref[key]), (len(vs), len(pp), bsz, key)
    with pytest.raises(b.SgError):   # views of different scenes
        other = b.DeviceScene.upload(ctx, sc, "f32")
        ctx.render_batch_views([preps[0], ctx.prepare(other, cams[1])], sa, va, pooled)


def _region_mask(changed_tiles, tiles_x, tiles_y):
    m = 0
    for ty, tx in zip(*np.nonzero(changed_tiles)):
        m |= 1 << int((ty * 8 // tiles_y) * 8 + (tx * 8 // tiles_x))
    return m


@pytest.mark.parametrize("tile", [8, 16])
def test_contamination_regions(ctx, tile):
    """Sort-first contamination (Sec. 5.10) on the 8 x 8 region grid: the
    rendered regions are exactly those holding a tile with a pixel changed by
    more than one level in the variant's image, they lie inside the predicted
    (dirty-tile) regions, and full-path variants predict every region."""
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(6741, seed=3, sh_degree=3)
    cam = synth.make_camera(200, 160)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam, b.raster_struct(tile=tile))
    clean = prep.frame().cpu().numpy().astype(np.float64)
    sites = synth.make_sites_stratified(sc.n, 3, 24, seed=33, width_bits=32)
    dose = synth.make_sites_dose(sc.n, 3, 20, seed=34, width_bits=32)
    allsites = synth.Sites(*(np.concatenate([a, c]) for a, c in zip(
        (sites.field, sites.comp, sites.prim, sites.bit), (dose.field, dose.comp, dose.prim, dose.bit))))
    groups = [np.array([k]) for k in range(len(sites))] + [np.arange(len(sites), len(allsites))]
    imgs, ms = _batch(ctx, prep, allsites, groups)
    tx_n, ty_n = -(-200 // tile), -(-160 // tile)
    n_nonempty = 0
    for j in range(len(groups)):
        d = np.abs(imgs[j].astype(np.float64) - clean).max(axis=2) > LEVEL
        pad = np.zeros((ty_n * tile, tx_n * tile), bool)
        pad[:160, :200] = d
        changed_tiles = pad.reshape(ty_n, tile, tx_n, tile).any(axis=(1, 3))
        rend = int(ms["rendered_regions"][j])
        pred = int(ms["predicted_regions"][j])
        assert rend == _region_mask(changed_tiles, tx_n, ty_n), j
        assert rend & ~pred == 0, j
        n_nonempty += rend != 0
        if ms["path"][j] == 0:
            assert bin(pred).count("1") <= int(ms["dirty_tiles"][j])
        else:
            assert pred == (1 << 64) - 1
    assert n_nonempty >= 5 and ms["path"][-1] == 1


def test_emulated_defenses(ctx):
    """Table 3's alternatives on one fault grid: the sign+exponent code
    removes exactly the sites on sign and exponent bits (incremental and
    full-path variants), the three-copy vote removes every site, and the
    selective guard (log-scales and opacity only) matches the oracle's guard
    restricted to those fields."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(4000, seed=14)
    cam = synth.make_camera(128, 128)
    lo32, hi32 = synth.make_box_jitter(sc, seed=4)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    box = b.Box.per_prim(ctx, lo32, hi32, "f32")
    prep = ctx.prepare(ds, cam)
    single = synth.make_sites_stratified(sc.n, 0, 16, seed=35, width_bits=32, fields=(0, 1, 2, 3, 4))
    dose = synth.make_sites_dose(sc.n, 0, 12, seed=36, width_bits=32)
    sites = synth.Sites(*(np.concatenate([a, c]) for a, c in zip(
        (single.field, single.comp, single.prim, single.bit), (dose.field, dose.comp, dose.prim, dose.bit))))
    sa = b.sites_array(sites.field, sites.comp, sites.prim, sites.bit)
    ns, nd = len(single.prim), len(dose.prim)

    def run(offs, cnts, protect=0, guard=0, mask=b.SG_FIELD_MASK_GUARD, sarr=sa):
        va = b.variants_array(np.asarray(offs), np.asarray(cnts), guard, protect)
        mt = b.metrics_tensor(len(va))
        imgs = torch.zeros((len(va), 128, 128, 3), dtype=torch.float32, device="cuda")
        ctx.render_batch(prep, sarr, va, box=box, box_mask=mask, images=imgs, metrics=mt)
        torch.cuda.synchronize()
        return imgs.cpu().numpy(), b.read_metrics(mt)

    offs, cnts = list(range(ns)) + [ns], [1] * ns + [nd]
    _, plain = run(offs, cnts)
    _, ecc = run(offs, cnts, protect=b.SG_PROTECT_SIGN_EXP)
    _, vote = run(offs, cnts, protect=b.SG_PROTECT_VOTE)
    assert np.all(vote["sse"] == 0) and np.all(vote["changed_px"] == 0) and np.all(vote["nonfinite"] == 0)
    low = sites.bit < 23
    for j in range(ns):
        if low[j]:
            for key in ("sse", "changed_px", "max_abs", "nonfinite", "dirty_tiles"):
                assert ecc[key][j] == plain[key][j], (j, key)
        else:
            assert ecc["sse"][j] == 0 and ecc["changed_px"][j] == 0 and ecc["nonfinite"][j] == 0, j
    # the full-path variant under the code equals the variant of its low-bit sites alone
    keep = np.nonzero(low[ns:])[0] + ns
    sk = b.sites_array(sites.field[keep], sites.comp[keep], sites.prim[keep], sites.bit[keep])
    _, low_only = run([0], [len(keep)], sarr=sk)
    assert ecc["path"][-1] == 1
    for key in ("sse", "changed_px", "max_abs", "nonfinite"):
        assert ecc[key][-1] == low_only[key][0], key
    # selective guard: log-scales (1) and opacity (3) only
    words = stored(sc, "f32")
    lo = [None if a is None else formats.f32_words(a) for a in lo32]
    hi = [None if a is None else formats.f32_words(a) for a in hi32]
    pick = [j for j in range(ns) if sites.field[j] in (1, 3)][:6] + [j for j in range(ns) if sites.field[j] == 0][:2]
    imgs, ms = run(pick, [1] * len(pick), guard=1, mask=(1 << 1) | (1 << 3))
    clean_gpu = prep.frame().cpu().numpy()
    clean_ref = oracle_render(words, "f32", 0, cam)
    for k, j in enumerate(pick):
        w, n_cl = oguard.guard_scene(apply_sites(words, sites, j), lo, hi, "f32", fields=(1, 3))
        ref = oracle_render(w, "f32", 0, cam)
        _check_variant(imgs[k], ms[k], ref, clean_ref, clean_gpu)
        assert int(ms["clamps"][k]) == n_cl


def test_sg_metrics_matches_definition(ctx):
    import torch
    from paper_2606_21791_amd import binding as b
    rng = np.random.default_rng(17)
    B, K, H, W = 3, 2, 40, 30
    clean = rng.uniform(0, 1, (K, H, W, 3)).astype(np.float32)
    imgs = np.repeat(clean[None], B, 0).copy()
    imgs[0, 0, :5, :5] += 0.1
    imgs[1, 1, 10, 10, 2] += 1.5 / 255
    imgs[2, 0, 3, 4, 1] = np.inf
    out = b.metrics_tensor(B)
    ctx.metrics(torch.from_numpy(imgs).cuda(), torch.from_numpy(clean).cuda(), B, K, H, W, out)
    torch.cuda.synchronize()
    m = b.read_metrics(out)
    for v in range(2):
        ref = om.frame_metrics(imgs[v].astype(np.float64), clean.astype(np.float64))
        assert m["changed_px"][v] == ref["changed_px"]
        assert abs(m["psnr"][v] - ref["psnr"]) < 1e-9
        assert m["catastrophic"][v] == ref["catastrophic"]
    assert m["nonfinite"][2] == 1 and m["catastrophic"][2] == 1


def test_w2_hi_campaign_matches_batches(ctx):
    """Full W2 size (N = 134,826, SH degree 3, fp32, 800 x 800) in the launch
    configuration of the headline (B = 32, 64 streams, 2 host threads, the
    campaign pipeline): every record equals sg_render_batch's on the same
    batches, whose frames test_gpu_parity_full checks against the oracle over
    the whole frame."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(134_826, seed=3, sh_degree=3)
    cam = synth.make_camera(800, 800)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam)
    s = synth.make_sites_stratified(sc.n, 3, 64, seed=46, width_bits=32)
    sa = b.sites_array(s.field, s.comp, s.prim, s.bit)
    n = len(sa)
    va = b.variants_array(np.arange(n), np.ones(n, np.uint32))
    ref = []
    for v0 in range(0, n, 32):
        mt = b.metrics_tensor(len(va[v0:v0 + 32]))
        ctx.render_batch(prep, sa, va[v0:v0 + 32], metrics=mt)
        ref.append(b.read_metrics(mt))
    ref = np.concatenate(ref)
    got = b.metrics_tensor(n)
    ctx.campaign(prep, sa, va, got, batch=32, streams=64, threads=2)
    torch.cuda.synchronize()
    G = b.read_metrics(got)
    for key in ref.dtype.names:
        assert np.array_equal(G[key], ref[key]), key
    assert np.any(G["dirty_tiles"] > 0) and np.any(G["changed_px"] > 0)


def test_graph_replay_matches_eager(ctx):
    """The captured incremental batch, replayed several times with eager work
    and synchronisations in between, gives exactly the eager records."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(6741, seed=3, sh_degree=3)
    cam = synth.make_camera(200, 160)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam)
    sites = synth.make_sites_stratified(sc.n, 3, 64, seed=21, width_bits=32)
    B = 32
    st = torch.cuda.Stream()
    va = b.variants_array(np.arange(B), np.ones(B, np.uint32))
    eager, graphed = [], []
    for rep in range(4):
        idx = (np.arange(B) + rep * B) % len(sites)
        sa = b.sites_array(sites.field[idx], sites.comp[idx], sites.prim[idx], sites.bit[idx])
        for use_graph, out in ((False, eager), (True, graphed)):
            ctx.set_graphs(use_graph)
            mt = b.metrics_tensor(B)
            with torch.cuda.stream(st):
                ctx.render_batch(prep, sa, va, metrics=mt)
            st.synchronize()
            out.append(b.read_metrics(mt))
            # eager work of the program between replays
            _ = (torch.ones(1000, device="cuda") * 2).sum().item()
    ctx.set_graphs(True)
    for e, g in zip(eager, graphed):
        for key in ("sse", "changed_px", "max_abs", "nonfinite", "dirty_tiles", "evals"):
            assert np.array_equal(e[key], g[key]), key
    assert not all(np.array_equal(eager[0]["sse"], e["sse"]) for e in eager[1:])   # the batches differ


def test_persistent_campaign_matches_batches(ctx):
    """The persistent campaign engine (chunks of variants, each listed,
    composited in one persistent launch and reduced) gives exactly the
    records of sg_render_batch on the same variants: guarded and multi-site
    variants, an empty variant, chunks of one size and of several (the two
    buffer sets alternating, a ragged last chunk), campaigns of one variant
    and of one variant with no sites, and, with a variant of more than eight
    primitives, the batch-by-batch fallback."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(4000, seed=14, sh_degree=1)
    cam = synth.make_camera(160, 128)
    lo32, hi32 = synth.make_box_jitter(sc, seed=4)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    box = b.Box.per_prim(ctx, lo32, hi32, "f32")
    prep = ctx.prepare(ds, cam)
    single = synth.make_sites_stratified(sc.n, 1, 40, seed=19, width_bits=32)
    dose = synth.make_sites_dose(sc.n, 1, 12, seed=20, width_bits=32)      # 12 primitives: full path
    sites = synth.Sites(*(np.concatenate([a, c]) for a, c in zip(
        (single.field, single.comp, single.prim, single.bit), (dose.field, dose.comp, dose.prim, dose.bit))))
    ns = len(single.prim)
    sa = b.sites_array(sites.field, sites.comp, sites.prim, sites.bit)
    offs = list(range(ns)) + [0, 0, ns]
    cnts = [1] * ns + [3, 0, len(dose.prim)]
    va = b.variants_array(np.array(offs), np.array(cnts), 0)
    va["guard"] = np.arange(len(offs)) % 3 == 0
    ref = []
    for v0 in range(0, len(va), 7):
        mt = b.metrics_tensor(len(va[v0:v0 + 7]))
        ctx.render_batch(prep, sa, va[v0:v0 + 7], box=box, metrics=mt)
        ref.append(b.read_metrics(mt))
    ref = np.concatenate(ref)
    # also single variants and a variant that changes nothing alone (no work
    # items at all: every workgroup's first claim is past the count)
    for vs, r in ((va[:1], ref[:1]), (va[ns + 1:ns + 2], ref[ns + 1:ns + 2]), (va[:3], ref[:3]), (va[:-1], ref[:-1]),
                  (va, ref)):
        for batch in (0, 5, 64):
            mt = b.metrics_tensor(len(vs))
            ctx.campaign(prep, sa, vs, mt, box=box, batch=batch, engine=b.SG_ENGINE_PERSISTENT)
            torch.cuda.synchronize()
            got = b.read_metrics(mt)
            for key in ref.dtype.names:
                assert np.array_equal(got[key], r[key]), (len(vs), batch, key)
    assert ref["path"][-1] == 1 and np.all(ref["path"][:-1] == 0) and ref["sse"][-2] == 0


def test_persistent_campaign_views_and_scenes(ctx):
    """The persistent engine over K views (the views of a variant side by
    side in every launch, views of different sizes included) and over scenes
    of uneven size: records equal sg_render_batch_views per batch and
    sg_render_batch on each variant's own scene."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(4000, seed=14, sh_degree=1)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    lo32, hi32 = synth.make_box_jitter(sc, seed=4)
    box = b.Box.per_prim(ctx, lo32, hi32, "f32")
    s = synth.make_sites_stratified(sc.n, 1, 12, seed=31, width_bits=32)
    sa = b.sites_array(s.field, s.comp, s.prim, s.bit)
    va = b.variants_array(np.arange(len(sa)), np.ones(len(sa), np.uint32))
    va["guard"] = np.arange(len(va)) % 2
    for cams in (synth.make_orbit_cameras(3, 96, 80), synth.make_orbit_cameras(2, 96, 80) + [synth.make_camera(64, 48)]):
        preps = [ctx.prepare(ds, c) for c in cams]
        ref = []
        for v0 in range(0, len(va), 9):
            mt = b.metrics_tensor(len(va[v0:v0 + 9]))
            ctx.render_batch_views(preps, sa, va[v0:v0 + 9], mt, box=box)
            ref.append(b.read_metrics(mt))
        ref = np.concatenate(ref)
        for batch in (0, 10):
            got = b.metrics_tensor(len(va))
            ctx.campaign(preps, sa, va, got, box=box, batch=batch, engine=b.SG_ENGINE_PERSISTENT)
            torch.cuda.synchronize()
            G = b.read_metrics(got)
            for key in ref.dtype.names:
                assert np.array_equal(G[key], ref[key]), (len(cams), batch, key)
    # scenes of uneven size
    specs = [(6741, 1, "f32", 200, 160), (2500, 0, "bf16", 96, 64), (12000, 3, "f16", 256, 144)]
    preps, site_sets = [], []
    for j, (n, sh, fmt, w, h) in enumerate(specs):
        scj = synth.make_scene(n, seed=70 + j, sh_degree=sh)
        dsj = b.DeviceScene.upload(ctx, scj, fmt)
        preps.append(ctx.prepare(dsj, synth.make_camera(w, h)))
        preps[-1]._ds = dsj
        W = formats.width(fmt)
        site_sets.append(synth.make_sites_stratified(n, sh, 2 * W, seed=80 + j, width_bits=W, fields=(0, 1, 2, 3, 4)))
    cat = lambda key: np.concatenate([getattr(t, key) for t in site_sets])
    sa = b.sites_array(cat("field"), cat("comp"), cat("prim"), cat("bit"))
    base = np.cumsum([0] + [len(t.prim) for t in site_sets])
    rng = np.random.default_rng(77)
    scene_of = rng.integers(0, 3, size=150).astype(np.uint16)
    off = np.array([base[k] + rng.integers(0, len(site_sets[k].prim)) for k in scene_of])
    va = b.variants_array(off, np.ones(len(off), np.uint32))
    for batch in (0, 16):
        got = b.metrics_tensor(len(va))
        ctx.campaign_scenes(preps, sa, va, scene_of, got, batch=batch, engine=b.SG_ENGINE_PERSISTENT)
        torch.cuda.synchronize()
        G = b.read_metrics(got)
        for k in range(3):
            idx = np.nonzero(scene_of == k)[0]
            t = site_sets[k]
            vk = va[idx].copy()
            vk["site_off"] -= np.uint32(base[k])
            mt = b.metrics_tensor(len(idx))
            ctx.render_batch(preps[k], b.sites_array(t.field, t.comp, t.prim, t.bit), vk, metrics=mt)
            ref = b.read_metrics(mt)
            for key in ref.dtype.names:
                assert np.array_equal(G[key][idx], ref[key]), (batch, k, key)


def test_persistent_campaign_w2_hi_matches_pipelined(ctx):
    """Full W2 size (N = 134,826, SH degree 3, fp32, 800 x 800): the persistent
    engine's records over 2,000 stratified single-bit variants equal the
    pipelined engine's in the headline configuration (B = 32, 64 streams)."""
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(134_826, seed=3, sh_degree=3)
    cam = synth.make_camera(800, 800)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam)
    s = synth.make_sites_stratified(sc.n, 3, 400, seed=46, width_bits=32)
    sa = b.sites_array(s.field, s.comp, s.prim, s.bit)
    n = len(sa)
    va = b.variants_array(np.arange(n), np.ones(n, np.uint32))
    ref, got = b.metrics_tensor(n), b.metrics_tensor(n)
    ctx.campaign(prep, sa, va, ref, batch=32, streams=64, threads=2)
    ctx.campaign(prep, sa, va, got, engine=b.SG_ENGINE_PERSISTENT)
    torch.cuda.synchronize()
    R, G = b.read_metrics(ref), b.read_metrics(got)
    for key in R.dtype.names:
        assert np.array_equal(G[key], R[key]), key
    assert np.any(G["dirty_tiles"] > 1000) and np.any(G["changed_px"] > 0)
