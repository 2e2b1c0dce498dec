"""Pins for oracle.formats: decode/cast against numpy's IEEE types and brute
force, flips against Lemma 1 in exact rational arithmetic."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import formats

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _same(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(
        np.where(np.isnan(a), 0, a), np.where(np.isnan(b), 0, b)) and np.array_equal(
        np.signbit(np.where(np.isnan(a), 0, a)), np.signbit(np.where(np.isnan(b), 0, b)))


def test_decode_f16_all_words_match_numpy():
    w = np.arange(1 << 16, dtype=np.uint16)
    assert _same(formats.decode(w, "f16"), w.view(np.float16).astype(np.float64))


def test_decode_bf16_all_words_are_upper_half_of_f32():
    w = np.arange(1 << 16, dtype=np.uint16)
    ref = (w.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert _same(formats.decode(w, "bf16"), ref)


def test_decode_f32_random_words_match_numpy():
    rng = np.random.default_rng(0)
    w = rng.integers(0, 1 << 32, size=200_000, dtype=np.uint64).astype(np.uint32)
    w[:8] = [0, 0x80000000, 0x7F800000, 0xFF800000, 0x00000001, 0x007FFFFF, 0x7F7FFFFF, 0x7FC00000]
    assert _same(formats.decode(w, "f32"), w.view(np.float32).astype(np.float64))


def test_encode_roundtrip_all_16bit_words():
    for fmt in ("f16", "bf16"):
        w = np.arange(1 << 16, dtype=np.uint16)
        v = formats.decode(w, fmt)
        ok = ~np.isnan(v)
        assert np.array_equal(formats.encode_exact(v[ok], fmt), w[ok])


def _test_values(rng):
    e = rng.uniform(-30, 20, size=100_000)
    x = (rng.choice([-1, 1], size=e.size) * np.exp2(e) * rng.uniform(1, 2, size=e.size)).astype(np.float32)
    extra = np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, 65536.0, 1e-8, 5.96e-8, 2.98e-8, 2.9802322e-08,
                      6.1e-5, 1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, 3.3895314e38, 3.39e38, -3.4e38,
                      np.inf, -np.inf], dtype=np.float32)
    return np.concatenate([x, extra])


def test_cast_f16_rne_matches_numpy():
    x = _test_values(np.random.default_rng(1))
    got = formats.decode(formats.cast(x.astype(np.float64), "f16", "rne"), "f16")
    assert _same(got, x.astype(np.float16).astype(np.float64))


def _all_finite(fmt):
    w = np.arange(1 << 16, dtype=np.uint16)
    v = formats.decode(w, fmt)
    ok = np.isfinite(v) & ~((v == 0) & np.signbit(v))      # one zero
    vals = v[ok]
    order = np.argsort(vals, kind="stable")
    return vals[order], w[ok][order]


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_cast_rne_rd_ru_brute_force(fmt):
    vals, words = _all_finite(fmt)
    x = _test_values(np.random.default_rng(2)).astype(np.float64)
    x = x[np.isfinite(x)]
    hi_idx = np.searchsorted(vals, x, side="left")           # first >= x
    lo_idx = np.searchsorted(vals, x, side="right") - 1      # last <= x
    mf = formats.max_finite(fmt)
    ru_ref = np.where(hi_idx < vals.size, vals[np.minimum(hi_idx, vals.size - 1)], np.inf)
    rd_ref = np.where(lo_idx >= 0, vals[np.maximum(lo_idx, 0)], -np.inf)
    rd = formats.round_to_format(x, fmt, "rd")
    ru = formats.round_to_format(x, fmt, "ru")
    assert np.array_equal(rd, rd_ref) and np.array_equal(ru, ru_ref)
    # nearest, ties to the even last mantissa bit; beyond max + half ulp -> Inf
    dlo, dhi = x - rd_ref, ru_ref - x
    even_lo = (words[np.maximum(lo_idx, 0)] & 1) == 0
    pick_lo = (dlo < dhi) | ((dlo == dhi) & even_lo)
    rne_ref = np.where(pick_lo, rd_ref, ru_ref)
    half_ulp_top = 2.0 ** (np.floor(np.log2(mf)) - formats.FORMATS[fmt][2] - 1)
    rne_ref = np.where(np.abs(x) >= mf + half_ulp_top, np.copysign(np.inf, x), rne_ref)
    rne_ref = np.where(np.abs(x) > mf, np.where(np.abs(x) >= mf + half_ulp_top, rne_ref, np.copysign(mf, x)), rne_ref)
    rne = formats.round_to_format(x, fmt, "rne")
    nz = rne_ref != 0
    assert np.array_equal(rne[nz], rne_ref[nz])
    assert np.all(rne[~nz] == 0)


def test_flip_is_involution():
    rng = np.random.default_rng(3)
    w = rng.integers(0, 1 << 32, size=1000, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 32, size=1000)
    assert np.array_equal(formats.flip(formats.flip(w, b), b), w)


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16"])
def test_lemma1_exact(fmt):
    """Lemma 1: a mantissa flip at bit b changes a normal value by exactly
    2^(e+b-p); the sign flip gives -2 theta; exponent bit j scales the
    magnitude by 2^(+-2^j) or leaves the normal range."""
    wbits, eb, p, bias = formats.FORMATS[fmt]
    assert p == GOLD["lemma1_mantissa_widths"][fmt]
    rng = np.random.default_rng(4)
    x = rng.normal(0, 3, size=300).astype(np.float32)
    words = formats.store(x, fmt)
    vals = formats.decode(words, fmt)
    for wv, th in zip(words, vals):
        if th == 0 or not np.isfinite(th):
            continue
        E = (int(wv) >> p) & ((1 << eb) - 1)
        if E == 0:
            continue
        e = E - bias
        T = Fraction(float(th))
        for b in range(p):
            d = Fraction(float(formats.decode(formats.flip(np.array([wv]), b), fmt)[0])) - T
            assert abs(d) == Fraction(2) ** (e + b - p)
        s = float(formats.decode(formats.flip(np.array([wv]), wbits - 1), fmt)[0])
        assert Fraction(s) - T == -2 * T
        for j in range(eb):
            newE = E ^ (1 << j)
            y = float(formats.decode(formats.flip(np.array([wv]), p + j), fmt)[0])
            if newE == (1 << eb) - 1:
                assert not np.isfinite(y)
            elif newE == 0:
                assert abs(y) < 2.0 ** (1 - bias)            # subnormal or zero
            else:
                sign = 1 if newE > E else -1
                assert Fraction(y) == T * Fraction(2) ** (sign * (1 << j))


def test_fp32_bit_classes_match_paper():
    g = GOLD["fp32_bit_classes"]
    x = np.array([1.5], np.float32)
    w = formats.store(x, "f32")
    assert formats.decode(formats.flip(w, g["sign"]), "f32")[0] == -1.5
    assert formats.decode(formats.flip(w, g["exponent"][0]), "f32")[0] in (0.75, 3.0)
    assert formats.decode(formats.flip(w, g["mantissa"][1]), "f32")[0] in (1.0, 2.0)
