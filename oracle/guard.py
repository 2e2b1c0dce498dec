"""Support guard (oracle; test infrastructure only).

Alg. 1 of the paper: the box is a per-(field, component) min/max over the
clean primitives, computed once; each frame every guarded component is
clamped into its box, non-finite values are mapped into the box (Thm. 1), and
the number of clamped components is counted and compared with a health
threshold.

Readings fixed here (the paper leaves them open):
  * NaN maps to the lower bound; +-Inf clamp like any value above/below.
  * Comparisons are IEEE (-0 == +0); a value inside the box keeps its bits, so
    the guarded word is exactly one of {x, lo, hi}.
  * A tie between -0 and +0 in the box reduction picks -0 for the minimum and
    +0 for the maximum (IEEE total order).
  * The per-primitive box mode takes lo/hi arrays of the field's own shape.
  * Default guarded fields: means, log-scales, quaternions, opacity and the
    degree-0 colour (14 components); higher-order SH is skipped (Sec. 5.12).
"""
from __future__ import annotations

import numpy as np

from . import formats

DEFAULT_FIELDS = (0, 1, 2, 3, 4)


def box_global(field_words, fmt: str):
    """lo/hi words, shape (C,), of one field's stored words (C, N):
    the per-component minimum and maximum over primitives (Alg. 1, precompute)."""
    w = np.asarray(field_words)
    v = formats.decode(w, fmt)
    C = w.shape[0]
    lo = np.empty(C, w.dtype)
    hi = np.empty(C, w.dtype)
    for c in range(C):
        # primary key: value; secondary: +0 after -0
        order = np.lexsort((~np.signbit(v[c]), v[c]))
        lo[c] = w[c, order[0]]
        hi[c] = w[c, order[-1]]
    return lo, hi


def clamp(field_words, lo_words, hi_words, fmt: str):
    """Guard one field.  lo/hi are (C,) (global box) or (C, N) (per primitive).
    Returns (guarded words, number of clamped components)."""
    w = np.asarray(field_words)
    lo_w = np.asarray(lo_words)
    hi_w = np.asarray(hi_words)
    if lo_w.ndim == 1:
        lo_w = np.broadcast_to(lo_w[:, None], w.shape)
        hi_w = np.broadcast_to(hi_w[:, None], w.shape)
    x = formats.decode(w, fmt)
    lo = formats.decode(lo_w, fmt)
    hi = formats.decode(hi_w, fmt)
    to_lo = np.isnan(x) | (x < lo)
    to_hi = ~to_lo & (x > hi)
    out = np.where(to_lo, lo_w, np.where(to_hi, hi_w, w)).astype(w.dtype)
    return out, int(np.count_nonzero(to_lo | to_hi))


def guard_scene(words, lo, hi, fmt: str, fields=DEFAULT_FIELDS):
    """Apply `clamp` to every guarded field of a scene (list of 6 word arrays).
    lo/hi: lists indexed by field.  Returns (new word list, total clamp count)."""
    out = list(words)
    total = 0
    for f in fields:
        if words[f].shape[0] == 0:
            continue
        out[f], n = clamp(words[f], lo[f], hi[f], fmt)
        total += n
    return out, total


def health_alert(count: int, threshold: int) -> bool:
    """Alg. 1: alert the host when the clamp count exceeds the threshold."""
    return count > threshold
