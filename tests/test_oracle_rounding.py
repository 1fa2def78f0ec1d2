"""Pins of the BF16 / FP16 stochastic-rounding oracle (oracle/rounding.py).

The hash is pinned to MurmurHash3's published test vectors; the rounding rule
to what defines stochastic rounding: the result brackets the value, exact BF16
values are kept, and averaged over all 2^16 random values the result equals the
input exactly (unbiasedness).
"""
import ast
import os

import numpy as np
import pytest

from oracle import rounding

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "murmur3_x86_32.txt")


def _vectors():
    out = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        key, seed, h = (t.strip() for t in line.split("|"))
        out.append((ast.literal_eval(key), int(seed, 16), int(h, 16)))
    return out


@pytest.mark.parametrize("key,seed,h", _vectors())
def test_murmur3_published_vectors(key, seed, h):
    assert rounding.murmur3_x86_32(key, seed) == h


def test_fmix32_array_form_matches_scalar_and_is_a_bijection():
    x = np.arange(1 << 20, dtype=np.uint32) * np.uint32(2654435761)
    h = rounding.fmix32(x)
    assert [int(v) for v in h[:64]] == [rounding.fmix32(int(v)) for v in x[:64]]
    assert np.unique(h).size == x.size          # distinct inputs, distinct outputs
    assert rounding.fmix32(1) == 0x514E28B7


def _bf16_neighbours(v):
    """(value toward zero, next BF16 value away from zero) of FP32 values."""
    b = np.asarray(v, dtype=np.float32).view(np.uint32)
    lo = (b & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    hi = ((b & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    return lo, hi


def _samples():
    rng = np.random.default_rng(11)
    v = np.concatenate([
        rng.standard_normal(40) * 10.0 ** rng.integers(-30, 30, 40),
        np.float32([1.0, -1.0, 3.0e-3, 1.0 / 3.0, -2.0 / 3.0, 1e-40, -3e-42]),  # incl. subnormals
    ]).astype(np.float32)
    return v


def test_unbiased_over_all_random_values():
    r = np.arange(1 << 16, dtype=np.uint32)
    for v in _samples():
        out = rounding.stochastic_bf16(np.full(r.size, v, dtype=np.float32), r)
        # every outcome is a multiple of the BF16 spacing with at most 8
        # significant bits: the FP64 sum of 2^16 of them is exact
        assert out.sum() / r.size == float(v), v


def test_brackets_and_extreme_random_values():
    v = _samples()
    lo, hi = _bf16_neighbours(v)
    exact = lo == v.astype(np.float64)
    for r in (0, 1, 0x7FFF, 0x8000, 0xFFFF):
        out = rounding.stochastic_bf16(v, np.full(v.size, r))
        assert np.all((out == lo) | (out == hi))
        assert np.all(out[exact] == lo[exact])
    assert np.all(rounding.stochastic_bf16(v, np.zeros(v.size)) == lo)          # r = 0: truncation
    up = rounding.stochastic_bf16(v, np.full(v.size, 0xFFFF))
    assert np.all(up[~exact] == hi[~exact])                                      # r = max: away from zero


def test_probability_of_rounding_up_is_the_fraction():
    v = np.float32(1.0 + 3 * 2.0 ** -9 + 5 * 2.0 ** -23)   # between 1 + 2^-8 and 1 + 2^-7
    r = np.arange(1 << 16, dtype=np.uint32)
    out = rounding.stochastic_bf16(np.full(r.size, v), r)
    lo, hi = _bf16_neighbours(np.float32([v]))
    frac = (float(v) - lo[0]) / (hi[0] - lo[0])
    assert np.mean(out == hi[0]) == frac


def test_sign_symmetry_and_special_values():
    v = _samples()
    r = np.random.default_rng(3).integers(0, 1 << 16, v.size)
    assert np.array_equal(rounding.stochastic_bf16(-v, r), -rounding.stochastic_bf16(v, r))
    sp = np.float32([np.inf, -np.inf, np.nan, 0.0, -0.0])
    out = rounding.stochastic_bf16(sp, np.full(sp.size, 0xFFFF))
    assert out[0] == np.inf and out[1] == -np.inf and np.isnan(out[2])
    assert out[3] == 0.0 and out[4] == 0.0 and np.signbit(out[4])
    big = np.float32(np.finfo(np.float32).max)     # rounds up to Inf, never wraps
    assert rounding.stochastic_bf16(np.float32([big]), [0xFFFF])[0] == np.inf


def test_random_bits_layout_and_statistics():
    q, N = 19, 1 << 14
    r = rounding.random_bits(N, q, step=7, seed=99)
    assert r.shape == (q, N) and r.max() < (1 << 16)
    # directions 2k, 2k+1 are the halves of one hash
    base = (np.arange(N, dtype=np.uint64) * 0x9E3779B1 + 7 * 0x85EBCA77 + 99) & 0xFFFFFFFF
    h3 = rounding.fmix32((base + 3 * 0xC2B2AE3D) & 0xFFFFFFFF)
    assert np.array_equal(r[6], h3 & 0xFFFF) and np.array_equal(r[7], h3 >> 16)
    # uniform: mean and variance of U{0..65535} within 5 sigma
    x = r.astype(np.float64).ravel()
    mu, var = (2.0 ** 16 - 1) / 2, (2.0 ** 32 - 1) / 12
    assert abs(x.mean() - mu) < 5 * np.sqrt(var / x.size)
    assert abs(x.var() / var - 1) < 0.02
    # neighbouring nodes, the two halves and consecutive steps are uncorrelated
    z = (r.astype(np.float64) - mu) / np.sqrt(var)
    lim = 5 / np.sqrt(N)
    assert abs(np.mean(z[:, 1:] * z[:, :-1])) < lim * 0.5
    assert abs(np.mean(z[0] * z[1])) < lim
    r8 = rounding.random_bits(N, q, step=8, seed=99)
    z8 = (r8.astype(np.float64) - mu) / np.sqrt(var)
    assert abs(np.mean(z * z8)) < lim * 0.5
    assert not np.array_equal(r, rounding.random_bits(N, q, step=7, seed=100))
    sel = np.array([0, 5, N - 1, 977])
    assert np.array_equal(rounding.random_bits_at(sel, q, 7, 99), r[:, sel])


# ------------------------------------------------------------------ FP16 ----
def _f16_neighbours(v):
    """(FP16 value toward zero, next FP16 value away from zero), from numpy's
    float16 rounding and nextafter."""
    v = np.asarray(v, dtype=np.float64)
    h = v.astype(np.float16)
    toward = np.where(np.abs(h.astype(np.float64)) > np.abs(v),
                      np.nextafter(h, np.float16(0)), h).astype(np.float64)
    inf16 = np.float16(np.inf)
    with np.errstate(over="ignore"):               # the neighbour of 65504 is Inf
        away = np.nextafter(toward.astype(np.float16), np.where(v < 0, -inf16, inf16))
    away = away.astype(np.float64)
    return toward, away


def _f16_samples():
    rng = np.random.default_rng(12)
    v = np.concatenate([
        rng.standard_normal(30) * 10.0 ** rng.uniform(-4, 4, 30),        # normal range
        rng.uniform(-6e-5, 6e-5, 20),                                    # FP16 subnormal range
        [1.0, -2.0 ** -14, 2.0 ** -14 * (1 - 2.0 ** -11), 3 * 2.0 ** -25, 65504.0, -1e-30,
         1234 * 2.0 ** -37, -5 * 2.0 ** -37],
    ]).astype(np.float32)
    return v


def test_f16_unbiased_over_all_random_values():
    r = np.arange(1 << 16, dtype=np.uint32)
    for v in _f16_samples():
        out = rounding.stochastic_f16(np.full(r.size, v, dtype=np.float32), r)
        mean = out.sum() / r.size                     # exact: 2^16 FP16 values
        if abs(v) >= 2.0 ** -14 or float(v) % 2.0 ** -37 == 0.0:
            assert mean == float(v), v
        else:   # subnormal range: resolved to 2^-37, 2^-13 of the 2^-24 spacing
            assert abs(mean - float(v)) <= 2.0 ** -38, v


def test_f16_brackets_and_extreme_random_values():
    v = _f16_samples()
    lo, hi = _f16_neighbours(v)
    exact = lo == v.astype(np.float64)
    for r in (0, 1, 7, 8, 0x7FFF, 0x8000, 0xFFFF):
        out = rounding.stochastic_f16(v, np.full(v.size, r))
        assert np.all((out == lo) | (out == hi)), r
        assert np.all(out[exact] == lo[exact])
    assert np.all(rounding.stochastic_f16(v, np.zeros(v.size)) == lo)       # r = 0: truncation
    up = rounding.stochastic_f16(v, np.full(v.size, 0xFFFF))
    resolved = np.abs(v.astype(np.float64) - lo) >= 2.0 ** -37              # not below the 2^-37 grid
    assert np.all(up[~exact & resolved] == hi[~exact & resolved])


def test_f16_probability_of_rounding_up():
    r = np.arange(1 << 16, dtype=np.uint32)
    for v, lo, hi in ((np.float32(1.0 + 5 * 2.0 ** -13), 1.0, 1.0 + 2.0 ** -10),
                      (np.float32(3.25 * 2.0 ** -24), 3 * 2.0 ** -24, 4 * 2.0 ** -24)):
        out = rounding.stochastic_f16(np.full(r.size, v), r)
        assert set(np.unique(out)) == {lo, hi}
        assert np.mean(out == hi) == (float(v) - lo) / (hi - lo)


def test_f16_sign_symmetry_and_special_values():
    v = _f16_samples()
    r = np.random.default_rng(4).integers(0, 1 << 16, v.size)
    assert np.array_equal(rounding.stochastic_f16(-v, r), -rounding.stochastic_f16(v, r))
    sp = np.float32([np.inf, -np.inf, np.nan, 0.0, -0.0, 7e4, -7e4])
    out = rounding.stochastic_f16(sp, np.full(sp.size, 0xFFFF))
    assert out[0] == np.inf and out[1] == -np.inf and np.isnan(out[2])
    assert out[3] == 0.0 and out[4] == 0.0 and np.signbit(out[4])
    assert out[5] == np.inf and out[6] == -np.inf                            # beyond 65504
    assert rounding.stochastic_f16(np.float32([65519.0]), [0])[0] == 65504.0
    assert rounding.stochastic_f16(np.float32([65519.0]), [0xFFFF])[0] == np.inf


# ------------------------------------------------------ property-based checks
from hypothesis import given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402

_finite32 = st.floats(width=32, allow_nan=False, allow_infinity=False)


@settings(max_examples=400, deadline=None)
@given(v=_finite32, r=st.integers(0, 0xFFFF))
def test_bf16_result_is_a_neighbour_for_any_value(v, r):
    lo, hi = _bf16_neighbours(np.float32([v]))
    out = rounding.stochastic_bf16(np.float32([v]), [r])[0]
    assert out == lo[0] or out == hi[0]


@settings(max_examples=400, deadline=None)
@given(v=st.floats(min_value=-65504.0, max_value=65504.0, width=32), r=st.integers(0, 0xFFFF))
def test_f16_result_is_a_neighbour_for_any_value(v, r):
    lo, hi = _f16_neighbours(np.float32([v]))
    out = rounding.stochastic_f16(np.float32([v]), [r])[0]
    assert out == lo[0] or out == hi[0]
    # monotone in r: a larger random value never rounds down where a smaller rounded up
    up = rounding.stochastic_f16(np.float32([v]), [min(r + 4096, 0xFFFF)])[0]
    assert abs(up) >= abs(out)
