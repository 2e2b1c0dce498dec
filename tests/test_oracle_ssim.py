"""Pins of the oracle's SSIM (Wang et al. 2004, as cited in Sec. 3 "Metrics")
against what the definition fixes independently of its code: identical
frames, constant frames (closed form), a pure brightness offset (closed form
per window), symmetry, the window's moments, and a hand loop on one window."""
import math

import numpy as np
import pytest

from oracle import ssim as S


def test_window_is_a_normalised_gaussian_of_sigma_1_5():
    w = S.window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    r = np.arange(11) - 5
    g = w.sum(axis=0)
    assert abs(float((g * r).sum())) < 1e-15                     # centred
    var = float((g * r * r).sum())
    # variance of a Gaussian of sigma 1.5 sampled on integers and truncated at +-5
    ref = sum(k * k * math.exp(-k * k / 4.5) for k in range(-5, 6)) / sum(math.exp(-k * k / 4.5) for k in range(-5, 6))
    assert abs(var - ref) < 1e-12 and 2.2 < var < 2.26
    assert np.allclose(w, w.T) and np.allclose(w, np.outer(g, g))


def test_identical_frames_give_one():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(23, 31, 3))
    assert S.ssim(x, x) == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("a,b", [(0.2, 0.7), (1.0, 0.0), (0.5, 0.5001)])
def test_constant_frames_closed_form(a, b):
    x = np.full((16, 16, 3), a)
    y = np.full((16, 16, 3), b)
    ref = (2 * a * b + S.C1) / (a * a + b * b + S.C1)       # zero variances: the contrast term is C2/C2
    assert S.ssim(x, y) == pytest.approx(ref, rel=1e-12)


def test_brightness_offset_closed_form():
    # y = x + c keeps every local variance and covariance, so each window's
    # index is the luminance term alone
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 0.5, size=(20, 20))
    c = 0.25
    m = S.ssim_map(x, x + c)
    # local means from an explicit loop over one window
    w = S.window()
    for (i, j) in ((0, 0), (4, 7), (9, 9)):
        mx = float((w * x[i:i + 11, j:j + 11]).sum())
        my = mx + c
        assert m[i, j] == pytest.approx((2 * mx * my + S.C1) / (mx * mx + my * my + S.C1), rel=1e-12)


def test_one_window_by_hand_and_symmetry():
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(11, 11))
    y = np.clip(x + rng.normal(0, 0.1, size=(11, 11)), 0, 1)
    w = S.window()
    mx, my = (w * x).sum(), (w * y).sum()
    vx = (w * (x - mx) ** 2).sum()
    vy = (w * (y - my) ** 2).sum()
    cxy = (w * (x - mx) * (y - my)).sum()
    ref = (2 * mx * my + S.C1) * (2 * cxy + S.C2) / ((mx * mx + my * my + S.C1) * (vx + vy + S.C2))
    m = S.ssim_map(x, y)
    assert m.shape == (1, 1) and m[0, 0] == pytest.approx(ref, rel=1e-12)
    assert S.ssim_map(y, x)[0, 0] == pytest.approx(m[0, 0], rel=1e-14)


def test_valid_positions_and_channel_mean():
    rng = np.random.default_rng(3)
    x = rng.uniform(size=(14, 12, 3))
    y = rng.uniform(size=(14, 12, 3))
    assert S.ssim_map(x[..., 0], y[..., 0]).shape == (4, 2)
    per = [S.ssim_map(x[..., c], y[..., c]).mean() for c in range(3)]
    assert S.ssim(x, y) == pytest.approx(np.mean(per), rel=1e-15)
    assert S.ssim(x, y) < 0.5                                   # unrelated noise is dissimilar
    with pytest.raises(ValueError):
        S.ssim(x[:10], y[:10])
