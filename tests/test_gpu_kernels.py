"""GPU parity of the integer/byte work through the C ABI: casts, bit flips,
restore, the support box and the guard clamp with its count and alert --
all bit-exact against the oracle."""
import numpy as np
import pytest

from oracle import formats, guard as oguard
from paper_2606_21791_amd import synth

from ._helpers import stored

pytestmark = pytest.mark.gpu
FMTS = ["f32", "f16", "bf16"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2606_21791_amd import binding
    return binding.Context(0)


def _edge_values(rng):
    e = rng.uniform(-30, 20, size=50_000)
    x = (rng.choice([-1, 1], size=e.size) * np.exp2(e) * rng.uniform(1, 2, size=e.size)).astype(np.float32)
    extra = np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, 65536.0, 1e-8, 5.96e-8, 2.98e-8, 6.1e-5,
                      1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.3895314e38,
                      3.39e38, -3.4e38, 1e-40, -1e-42, np.inf, -np.inf, np.nan], dtype=np.float32)
    return np.concatenate([x, extra])


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("mode", ["rne", "rd", "ru"])
def test_cast_bit_exact(ctx, fmt, mode):
    import torch
    from paper_2606_21791_amd import binding as b
    x = _edge_values(np.random.default_rng(0))
    got = ctx.cast(torch.from_numpy(x).cuda(), b.DTYPES[fmt], {"rne": 0, "rd": 1, "ru": 2}[mode])
    got = got.cpu().numpy().view(np.uint16)
    ref = formats.cast(x.astype(np.float64), fmt, mode)
    nan = np.isnan(x)
    assert np.array_equal(got[~nan], ref[~nan])
    assert np.all(np.isnan(formats.decode(got[nan], fmt)))


@pytest.mark.parametrize("fmt", FMTS)
def test_inject_restore_bit_exact(ctx, fmt):
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(3000, seed=3, sh_degree=2)
    ds = b.DeviceScene.upload(ctx, sc, fmt)
    words = stored(sc, fmt)
    assert all(np.array_equal(a, c) for a, c in zip(ds.host_words(), words))
    W = formats.width(fmt)
    s = synth.make_sites_dose(sc.n, 2, 4000, seed=4, width_bits=W)
    # duplicate some sites on purpose: flips on a shared word compose (XOR)
    s = synth.Sites(*(np.concatenate([a, a[:50]]) for a in (s.field, s.comp, s.prim, s.bit)))
    sa = b.sites_array(s.field, s.comp, s.prim, s.bit)
    saved = torch.zeros(len(sa), dtype=torch.int32, device="cuda")
    ctx.inject(ds, sa, saved)
    torch.cuda.synchronize()
    ref = [w.copy() for w in words]
    for k in range(len(s)):
        f, c, p, bt = int(s.field[k]), int(s.comp[k]), int(s.prim[k]), int(s.bit[k])
        ref[f][c, p] = formats.flip(ref[f][c, p:p + 1], bt)[0]
    assert all(np.array_equal(a, c) for a, c in zip(ds.host_words(), ref))
    sv = saved.cpu().numpy().view(np.uint32)
    # a site's saved word is the value before its own flip; only words flipped
    # by a single site have a unique such value
    key = (s.field.astype(np.int64) << 48) | (s.comp.astype(np.int64) << 32) | s.prim.astype(np.int64)
    _, inv, counts = np.unique(key, return_inverse=True, return_counts=True)
    uniq = counts[inv] == 1
    for k in np.nonzero(uniq)[0][:500]:
        f, c, p = int(s.field[k]), int(s.comp[k]), int(s.prim[k])
        assert sv[k] == int(words[f][c, p])
    ctx.restore(ds, sa)
    torch.cuda.synchronize()
    assert all(np.array_equal(a, c) for a, c in zip(ds.host_words(), words))


def test_invalid_site_rejected_without_mutation(ctx):
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(100, seed=5)
    ds = b.DeviceScene.upload(ctx, sc, "bf16")
    before = ds.host_words()
    bad = [b.sites_array([1], [0], [100], [3]),       # primitive out of range
           b.sites_array([1], [3], [0], [3]),         # component out of range
           b.sites_array([5], [0], [0], [3]),         # field absent at SH degree 0
           b.sites_array([0], [0], [0], [16])]        # bit beyond a 16-bit word
    for sa in bad:
        good_then_bad = np.concatenate([b.sites_array([0], [0], [1], [2]), sa])
        with pytest.raises(b.SgError) as e:
            ctx.inject(ds, good_then_bad)
        assert e.value.code == b.SG_E_INVAL
    torch.cuda.synchronize()
    assert all(np.array_equal(a, c) for a, c in zip(ds.host_words(), before))


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("n", [20_000, 20_003])   # 20,003: rows start off the 16-byte grid, ragged ends
def test_guard_box_and_clamp_bit_exact(ctx, fmt, n):
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(n, seed=6, sh_degree=1)
    ds = b.DeviceScene.upload(ctx, sc, fmt)
    words = stored(sc, fmt)
    box = ctx.guard_box(ds)
    torch.cuda.synchronize()
    lo, hi = [None] * 6, [None] * 6
    for f in oguard.DEFAULT_FIELDS:
        lo[f], hi[f] = oguard.box_global(words[f], fmt)
        glo, ghi = box.host_words(f)
        assert np.array_equal(glo, lo[f]) and np.array_equal(ghi, hi[f])
    # Thm. 1 (i): the guard leaves the clean model untouched
    cnt, alert = ctx.guard(ds, box, threshold=0)
    torch.cuda.synchronize()
    assert int(cnt[0]) == 0 and int(alert[0]) == 0
    assert all(np.array_equal(a, c) for a, c in zip(ds.host_words(), words))
    # corrupt, guard on the GPU and in the oracle
    s = synth.make_sites_dose(sc.n, 1, 5000, seed=7, width_bits=formats.width(fmt))
    ctx.inject(ds, b.sites_array(s.field, s.comp, s.prim, s.bit))
    bad = [w.copy() for w in words]
    for k in range(len(s)):
        f, c, p, bt = int(s.field[k]), int(s.comp[k]), int(s.prim[k]), int(s.bit[k])
        bad[f][c, p] = formats.flip(bad[f][c, p:p + 1], bt)[0]
    ref, n_ref = oguard.guard_scene(bad, lo, hi, fmt)
    cnt, alert = ctx.guard(ds, box, threshold=n_ref - 1)
    torch.cuda.synchronize()
    assert int(cnt[0]) == n_ref > 0
    assert int(alert[0]) == 1
    assert all(np.array_equal(a, c) for a, c in zip(ds.host_words(), ref))
    cnt, alert = ctx.guard(ds, box, threshold=0)    # idempotent
    torch.cuda.synchronize()
    assert int(cnt[0]) == 0 and int(alert[0]) == 0


@pytest.mark.parametrize("n", [5000, 5003])   # 5,003: rows off the 16-byte grid, ragged ends
def test_per_primitive_box_guard(ctx, n):
    import torch
    from paper_2606_21791_amd import binding as b
    sc = synth.make_scene(n, seed=8)
    lo32, hi32 = synth.make_box_jitter(sc, seed=4)
    for fmt in FMTS:
        ds = b.DeviceScene.upload(ctx, sc, fmt)
        box = b.Box.per_prim(ctx, lo32, hi32, fmt)
        words = stored(sc, fmt)
        lo = [None if a is None else formats.store(a, fmt, "rd") for a in lo32]
        hi = [None if a is None else formats.store(a, fmt, "ru") for a in hi32]
        torch.cuda.synchronize()
        for f in oguard.DEFAULT_FIELDS:
            glo, ghi = box.host_words(f)
            assert np.array_equal(glo, lo[f]) and np.array_equal(ghi, hi[f])
        s = synth.make_sites_dose(sc.n, 0, 3000, seed=9, width_bits=formats.width(fmt))
        ctx.inject(ds, b.sites_array(s.field, s.comp, s.prim, s.bit))
        bad = [w.copy() for w in words]
        for k in range(len(s)):
            f, c, p, bt = int(s.field[k]), int(s.comp[k]), int(s.prim[k]), int(s.bit[k])
            bad[f][c, p] = formats.flip(bad[f][c, p:p + 1], bt)[0]
        ref, n_ref = oguard.guard_scene(bad, lo, hi, fmt)
        cnt, _ = ctx.guard(ds, box)
        torch.cuda.synchronize()
        assert int(cnt[0]) == n_ref
        assert all(np.array_equal(a, c) for a, c in zip(ds.host_words(), ref))


def test_ssim_matches_oracle(ctx):
    """sg_ssim against the oracle's SSIM on the same float32 frames: random
    frames with ragged tiles, identical frames, and corrupted renders."""
    import torch
    from oracle import ssim as oss
    from paper_2606_21791_amd import binding as b, synth
    rng = np.random.default_rng(7)
    H, W = 37, 45
    clean = rng.uniform(size=(H, W, 3)).astype(np.float32)
    imgs = np.stack([clean, np.clip(clean + rng.normal(0, 0.05, size=clean.shape), 0, 1),
                     rng.uniform(size=clean.shape), np.full(clean.shape, 0.5)]).astype(np.float32)
    got = ctx.ssim(torch.from_numpy(imgs).cuda(), torch.from_numpy(clean).cuda()).cpu().numpy()
    ref = np.array([oss.ssim(imgs[k], clean) for k in range(len(imgs))])
    assert abs(got[0] - 1.0) < 1e-12
    assert np.allclose(got, ref, rtol=0, atol=1e-10), (got, ref)
    # corrupted renders of a small scene
    sc = synth.make_scene(3000, seed=5)
    cam = synth.make_camera(96, 72)
    ds = b.DeviceScene.upload(ctx, sc, "f32")
    prep = ctx.prepare(ds, cam)
    s = synth.make_sites_stratified(sc.n, 0, 4, seed=8, width_bits=32, fields=(0, 1, 3))
    sa = b.sites_array(s.field, s.comp, s.prim, s.bit)
    B = len(sa)
    out = torch.zeros((B, 72, 96, 3), dtype=torch.float32, device="cuda")
    ctx.render_batch(prep, sa, b.variants_array(np.arange(B), np.ones(B)), images=out, metrics=b.metrics_tensor(B))
    frame = prep.frame()
    got = ctx.ssim(out, frame).cpu().numpy()
    o, f = out.cpu().numpy(), frame.cpu().numpy()
    ref = np.array([oss.ssim(o[k], f) for k in range(B)])
    assert np.allclose(got, ref, rtol=0, atol=1e-10)
    assert got.min() < 1.0
    with pytest.raises(b.SgError):
        ctx.ssim(out[:, :10], frame[:10])

