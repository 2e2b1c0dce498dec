"""The allocation-free metrics entry point (sg_metrics_noalloc) against
sg_metrics through the C ABI: identical records on two calls in a row, the
second with a smaller input (the shared scratch keeps the first call's
partials, which must not leak into the second), and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _frames(rng, B, K, H, W):
    clean = rng.uniform(0, 1, (K, H, W, 3)).astype(np.float32)
    imgs = np.repeat(clean[None], B, 0).copy()
    for v in range(B):
        k = v % K
        y, x = rng.integers(0, H), rng.integers(0, W)
        imgs[v, k, y:y + 7, x:x + 5] += np.float32(0.02 * (v + 1) / B)
        imgs[v, k, rng.integers(0, H), rng.integers(0, W), v % 3] += np.float32(1.5 / 255)
    if B > 2:
        imgs[2, 0, 1, 1, 0] = np.inf          # a non-finite frame
    imgs[0] = clean                           # an unchanged variant (PSNR +Inf)
    return imgs, clean


def test_metrics_noalloc_matches_sg_metrics():
    import torch
    from paper_2606_21791_amd import binding as b
    assert torch.cuda.is_available()
    ctx = b.Context(0)
    rng = np.random.default_rng(101)
    for (B, K, H, W) in ((24, 2, 300, 257), (5, 1, 61, 47)):
        imgs, clean = _frames(rng, B, K, H, W)
        ti, tc = torch.from_numpy(imgs).cuda(), torch.from_numpy(clean).cuda()
        ref, got = b.metrics_tensor(B), b.metrics_tensor(B)
        ctx.metrics(ti, tc, B, K, H, W, ref)
        ctx.metrics_noalloc(ti, tc, B, K, H, W, got)
        torch.cuda.synchronize()
        R, G = b.read_metrics(ref), b.read_metrics(got)
        for key in R.dtype.names:
            assert np.array_equal(R[key], G[key]), (B, key)
        assert G["changed_px"][1] > 0 and np.isinf(G["psnr"][0]) and G["nonfinite"][2 % B] == (1 if B > 2 else 0)
    # 520 variants of 800 x 800 frames need 520 * 256 partials: beyond the 4 MiB scratch
    big = torch.zeros((1, 800, 800, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(b.SgError) as e:
        ctx.metrics_noalloc(big, big[0], 520, 1, 800, 800, b.metrics_tensor(520))
    assert e.value.code == b.SG_E_INVAL
