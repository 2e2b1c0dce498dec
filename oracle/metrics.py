"""Per-variant image metrics (oracle; test infrastructure only).

Sec. 3 "Metrics": each injection is compared with the clean render at the
same precision.  PSNR is over the full frame (peak 1, +Inf when the images
are equal); Def. 1: the corruption footprint is the fraction of pixels whose
colour changes by more than one 8-bit level, read here as max over RGB of
|delta| > 1/255 on float images, averaged over the K views; Def. 2: an upset
is catastrophic if the render is non-finite or the footprint exceeds 1%.
"""
from __future__ import annotations

import numpy as np

LEVEL = 1.0 / 255.0
CATASTROPHE_FOOTPRINT = 0.01


def frame_metrics(img, clean, nonfinite: bool = False, mask=None) -> dict:
    """img, clean: (K, H, W, 3) or (H, W, 3) float arrays in [0, 1].
    mask: optional boolean (K, H, W) / (H, W) of pixels to include."""
    img = np.asarray(img, np.float64)
    clean = np.asarray(clean, np.float64)
    if img.ndim == 3:
        img, clean = img[None], clean[None]
        if mask is not None:
            mask = np.asarray(mask)[None]
    d = img - clean
    if mask is None:
        mask = np.ones(d.shape[:3], bool)
    npix = int(mask.sum())
    sse = float(np.sum(d[mask] ** 2))
    mse = sse / (3 * npix) if npix else 0.0
    psnr = float("inf") if mse == 0.0 else 10.0 * np.log10(1.0 / mse)
    dmax = np.max(np.abs(d), axis=3)
    changed = int(np.count_nonzero((dmax > LEVEL) & mask))
    footprint = changed / npix if npix else 0.0
    return dict(sse=sse, mse=mse, psnr=psnr, changed_px=changed, footprint=footprint,
                max_abs=float(np.max(dmax[mask])) if npix else 0.0, nonfinite=bool(nonfinite),
                catastrophic=bool(nonfinite or footprint > CATASTROPHE_FOOTPRINT))


def wilson_interval(k: int, n: int, z: float = 1.959963984540054):
    """95% Wilson score interval of a binomial rate (Table 2 reports catastrophe
    rates with it)."""
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    den = 1.0 + z * z / n
    mid = (p + z * z / (2 * n)) / den
    half = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return (mid - half, mid + half)
