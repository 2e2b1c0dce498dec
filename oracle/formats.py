"""Storage formats, casts and bit flips (oracle; test infrastructure only).

Sec. 3, "Single-bit upset model": a stored value is reinterpreted as an
unsigned integer of its width, one bit is flipped, and the word is read back.
fp32 is 1|8|23 (bias 127), fp16 is 1|5|10 (bias 15), bf16 is 1|8|7 (bias
127).  Reduced precisions hold the clean fp32 parameter cast to the format.

Stored values are represented here as unsigned integer words (uint32 for
fp32, uint16 otherwise).  Casts are written from the definition of rounding:
the value is divided by the quantum (the weight of the last mantissa bit at
its binade, or the subnormal quantum), rounded to an integer, and multiplied
back -- all exact in float64 for fp32 inputs.
"""
from __future__ import annotations

import numpy as np

# name -> (width, exponent bits, mantissa bits p, bias)
FORMATS = {
    "f32": (32, 8, 23, 127),
    "f16": (16, 5, 10, 15),
    "bf16": (16, 8, 7, 127),
}
DTYPE_CODE = {"f32": 0, "f16": 1, "bf16": 2}


def width(fmt: str) -> int:
    return FORMATS[fmt][0]


def _word_dtype(fmt):
    return np.uint32 if FORMATS[fmt][0] == 32 else np.uint16


def max_finite(fmt: str) -> float:
    _, eb, p, bias = FORMATS[fmt]
    emax = (1 << eb) - 2 - bias
    return float((2.0 - 2.0 ** (-p)) * 2.0 ** emax)


def decode(words, fmt: str) -> np.ndarray:
    """Exact float64 value of each stored word (Inf/NaN preserved)."""
    w = np.asarray(words).astype(np.int64)
    wbits, eb, p, bias = FORMATS[fmt]
    sign = (w >> (wbits - 1)) & 1
    e = (w >> p) & ((1 << eb) - 1)
    m = w & ((1 << p) - 1)
    emax_field = (1 << eb) - 1
    mag = np.where(
        e == 0,
        np.ldexp(m.astype(np.float64), 1 - bias - p),                       # subnormal / zero
        np.ldexp((m + (1 << p)).astype(np.float64), (e - bias - p).astype(np.int64)),
    )
    mag = np.where(e == emax_field, np.where(m == 0, np.inf, np.nan), mag)
    return np.where(sign == 1, -mag, mag)


def encode_exact(values, fmt: str) -> np.ndarray:
    """Bit pattern of values that are exactly representable in fmt
    (including +-0, +-Inf and NaN -> quiet NaN)."""
    v = np.asarray(values, dtype=np.float64)
    wbits, eb, p, bias = FORMATS[fmt]
    sign = np.signbit(v).astype(np.int64)
    a = np.abs(v)
    out = np.zeros(v.shape, np.int64)
    finite = np.isfinite(a) & (a > 0)
    # binade exponent: a = f * 2^E, f in [0.5, 1)  ->  unbiased exponent E - 1
    _, E = np.frexp(np.where(finite, a, 1.0))
    e_unb = E.astype(np.int64) - 1
    emin = 1 - bias
    sub = finite & (e_unb < emin)
    nor = finite & ~sub
    m_sub = np.ldexp(np.where(sub, a, 0.0), (bias - 1 + p))                     # a / 2^(emin - p)
    m_nor = np.ldexp(np.where(nor, a, 1.0), (p - e_unb)) - (1 << p)           # (a / 2^e - 1) 2^p
    out = np.where(sub, np.where(sub, m_sub, 0.0).astype(np.int64), out)
    out = np.where(nor, ((e_unb + bias) << p) | np.where(nor, m_nor, 0.0).astype(np.int64), out)
    emax_field = (1 << eb) - 1
    out = np.where(np.isinf(a), emax_field << p, out)
    out = np.where(np.isnan(a), (emax_field << p) | (1 << (p - 1)), out)
    out = out | (sign << (wbits - 1))
    return out.astype(_word_dtype(fmt))


def round_to_format(values, fmt: str, mode: str = "rne") -> np.ndarray:
    """Value of `values` (float64) rounded into fmt: mode 'rne' (nearest,
    ties to even, overflow to Inf), 'rd' (toward -Inf) or 'ru' (toward +Inf).
    Subnormals are kept (no flush to zero)."""
    x = np.asarray(values, dtype=np.float64)
    wbits, eb, p, bias = FORMATS[fmt]
    emin = 1 - bias
    fin = np.isfinite(x)
    a = np.where(fin, np.abs(x), 1.0)
    _, E = np.frexp(np.where(a > 0, a, 1.0))
    e = np.maximum(E.astype(np.int64) - 1, emin)               # binade of the quantum
    quantum_exp = e - p
    r = np.ldexp(np.where(fin, x, 0.0), -quantum_exp)           # exact: scale by a power of two
    if mode == "rne":
        ri = np.rint(r)                                         # round half to even
    elif mode == "rd":
        ri = np.floor(r)
    elif mode == "ru":
        ri = np.ceil(r)
    else:
        raise ValueError(mode)
    y = np.ldexp(ri, quantum_exp)
    mf = max_finite(fmt)
    if mode == "rne":
        y = np.where(np.abs(y) > mf, np.copysign(np.inf, x), y)
    elif mode == "rd":
        y = np.where(y > mf, mf, np.where(y < -mf, -np.inf, y))
    else:
        y = np.where(y < -mf, -mf, np.where(y > mf, np.inf, y))
    # keep the sign of zero results (e.g. -1e-30 -> -0)
    y = np.where(y == 0, np.copysign(0.0, x), y)
    return np.where(fin, y, x)


def cast(values, fmt: str, mode: str = "rne") -> np.ndarray:
    """Words of `values` cast into fmt with the given rounding mode."""
    return encode_exact(round_to_format(values, fmt, mode), fmt)


def f32_words(values_f32) -> np.ndarray:
    """fp32 words of fp32 values."""
    return np.ascontiguousarray(np.asarray(values_f32, dtype=np.float32)).view(np.uint32)


def store(values_f32, fmt: str, mode: str = "rne") -> np.ndarray:
    """Stored words of a clean fp32 parameter array in fmt (Sec. 3: reduced
    precisions cast the clean parameter to the target format)."""
    if fmt == "f32":
        return f32_words(values_f32)
    return cast(np.asarray(values_f32, np.float32).astype(np.float64), fmt, mode)


def flip(words, bit) -> np.ndarray:
    """Flip one bit of each word: w XOR (1 << bit) (Sec. 3)."""
    w = np.asarray(words)
    return (w ^ (np.asarray(1, w.dtype) << np.asarray(bit, w.dtype))).astype(w.dtype)
