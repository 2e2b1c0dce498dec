"""Structural similarity of a corrupted frame and the clean frame (oracle;
test infrastructure only).

Sec. 3 "Metrics" records SSIM, citing Wang et al. (2004).  Reading of that
definition, with its published constants: images in [0, 1] (L = 1),
K1 = 0.01, K2 = 0.03, so C1 = (K1 L)^2 and C2 = (K2 L)^2; local statistics
under an 11 x 11 circular Gaussian window of standard deviation 1.5,
normalised to unit sum; the weighted (biased) variance and covariance
sigma_x^2 = E_w[x^2] - mu_x^2, sigma_xy = E_w[x y] - mu_x mu_y; the index at a
window is

    ((2 mu_x mu_y + C1) (2 sigma_xy + C2)) / ((mu_x^2 + mu_y^2 + C1) (sigma_x^2 + sigma_y^2 + C2)),

evaluated at every window position that lies wholly inside the frame (no
padding); the frame's SSIM is the mean over those positions and over the three
colour channels.  Everything is in FP64.
"""
from __future__ import annotations

import numpy as np

K1, K2 = 0.01, 0.03
C1, C2 = (K1 * 1.0) ** 2, (K2 * 1.0) ** 2
WIN, SIGMA = 11, 1.5


def window() -> np.ndarray:
    """The 11 x 11 Gaussian window (outer product of the normalised 1-D one)."""
    r = np.arange(WIN) - (WIN - 1) / 2.0
    g = np.exp(-(r * r) / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def _filter_valid(a: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Weighted window sums at every valid position: out[i, j] = sum w * a[i:i+11, j:j+11]."""
    H, W = a.shape
    out = np.zeros((H - WIN + 1, W - WIN + 1))
    for dy in range(WIN):
        for dx in range(WIN):
            out += w[dy, dx] * a[dy:dy + H - WIN + 1, dx:dx + W - WIN + 1]
    return out


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """SSIM index at every valid window position of two (H, W) channels."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    w = window()
    mx, my = _filter_valid(x, w), _filter_valid(y, w)
    sxx = _filter_valid(x * x, w) - mx * mx
    syy = _filter_valid(y * y, w) - my * my
    sxy = _filter_valid(x * y, w) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim(img: np.ndarray, clean: np.ndarray) -> float:
    """Mean SSIM of two (H, W, 3) frames over valid windows and channels."""
    img = np.asarray(img, np.float64)
    clean = np.asarray(clean, np.float64)
    if img.shape[0] < WIN or img.shape[1] < WIN:
        raise ValueError("frames smaller than the 11 x 11 window")
    return float(np.mean([ssim_map(img[..., c], clean[..., c]).mean() for c in range(img.shape[2])]))
