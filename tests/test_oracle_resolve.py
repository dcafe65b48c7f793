"""Pins of the oracle's error-bound resolution against exact rational arithmetic.

The reading (Sec. V-A for the REL bound; the binary32 tightening that makes
the pointwise bound hold): eb is the binary64 value of the request (ABS) or
of value * (max - min) (REL, two binary64 operations); u = ulp(max|x|), the
gap from max|x| to the next larger binary32; requests with eb < 8u are
rejected; E = the largest binary32 <= 2 (eb - 4u), computed exactly; E is
clamped to 2^126 and must be a normal number; max|x| + E must stay finite;
inv = 1/E correctly rounded to binary32.  A zero-range REL field (constant c)
uses E = |c| (1 if c = 0).

Everything expected here is computed with Python's fractions.Fraction and
numpy's nextafter, not with the oracle's own arithmetic.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

F32_MAX = Fraction(float(np.finfo(np.float32).max))
F32_MIN_NORMAL = Fraction(2) ** -126


def f32_up(f):
    return np.nextafter(np.float32(f), np.float32(np.inf))


def f32_down(f):
    return np.nextafter(np.float32(f), np.float32(0))


def ulp_above(m):
    """Gap from the binary32 m >= 0 to the next larger binary32, exactly."""
    m = np.float32(m)
    return Fraction(float(f32_up(m))) - Fraction(float(m))


def largest_f32_not_above(v):
    """The largest binary32 <= v (v > 0 a Fraction; binary32 range assumed)."""
    f = np.float32(float(v))  # a nearby binary32: correct up to a step or two
    while Fraction(float(f)) > v:
        f = f32_down(f)
    while np.isfinite(f32_up(f)) and Fraction(float(f32_up(f))) <= v:
        f = f32_up(f)
    return f


def nearest_f32(v):
    """v (> 0, a Fraction) rounded to the nearest binary32, ties to even."""
    c = np.float32(float(v))
    best = None
    for cand in (f32_down(c), c, f32_up(c)):
        d = abs(Fraction(float(cand)) - v)
        key = (d, int(np.frombuffer(np.float32(cand).tobytes(), np.uint32)[0]) & 1)
        if best is None or key < best[0]:
            best = (key, cand)
    return best[1]


def expected(x, mode, value):
    """(status, E, inv, flags) by the reading above, in exact arithmetic."""
    x = np.asarray(x, dtype=np.float32)
    if x.size == 0:
        return oracle.OK, np.float32(1), np.float32(1), 0
    xmin, xmax = float(x.min()), float(x.max())
    M = np.float32(np.abs(x).max())
    if mode == oracle.REL and xmax == xmin:
        c = abs(np.float32(xmin))
        if c == 0:
            E = np.float32(1)
        elif Fraction(float(c)) < F32_MIN_NORMAL:
            return oracle.ERR_EB_TOO_SMALL, None, None, None
        else:
            E = c
        return oracle.OK, E, nearest_f32(1 / Fraction(float(E))), 1
    eb = value * (xmax - xmin) if mode == oracle.REL else value  # binary64 operations
    u = ulp_above(M)
    if Fraction(eb) < 8 * u:
        return oracle.ERR_EB_TOO_SMALL, None, None, None
    target = 2 * (Fraction(eb) - 4 * u)
    if target >= Fraction(2) ** 126:
        E = np.float32(2.0 ** 126)
    else:
        E = largest_f32_not_above(target)
    if Fraction(float(E)) < F32_MIN_NORMAL:
        return oracle.ERR_EB_TOO_SMALL, None, None, None
    if Fraction(float(M)) + Fraction(float(E)) > F32_MAX:
        return oracle.ERR_EB_TOO_LARGE, None, None, None
    return oracle.OK, E, nearest_f32(1 / Fraction(float(E))), 0


def check(x, mode, value):
    st, E, inv, flags = oracle.resolve(x, mode, value)
    est, eE, einv, eflags = expected(x, mode, value)
    assert st == est, (mode, value, st, est)
    if st == oracle.OK:
        assert np.float32(E) == eE, (mode, value, E, eE)
        assert np.float32(inv) == einv, (mode, value, inv, einv)
        assert flags == eflags
    return st


def _random_cases(seed, count):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        scale = 10.0 ** rng.uniform(-30, 30)
        n = int(rng.integers(1, 40))
        x = (rng.uniform(-1, 1, n) * scale).astype(np.float32)
        if rng.integers(4) == 0:
            x = np.abs(x) + np.float32(scale)  # offset field: narrow range, large max|x|
        mode = int(rng.integers(2))
        if mode == oracle.REL:
            value = 10.0 ** rng.uniform(-7, 0)
        else:
            value = scale * 10.0 ** rng.uniform(-7, 2)
        yield x.astype(np.float32), mode, float(value)


def test_step_matches_exact_rationals():
    outcomes = {}
    for x, mode, value in _random_cases(1, 3000):
        st = check(x, mode, value)
        outcomes[st] = outcomes.get(st, 0) + 1
    # the sample reaches both the accepted and the rejected side of the threshold
    assert outcomes.get(oracle.OK, 0) > 1000 and outcomes.get(oracle.ERR_EB_TOO_SMALL, 0) > 50


def test_step_is_truncated_not_rounded():
    """Round-to-nearest of 2 (eb - 4u) differs from the truncation on about half of the cases."""
    rng = np.random.default_rng(2)
    differs = 0
    for _ in range(400):
        x = rng.uniform(-1, 1, 16).astype(np.float32)
        value = float(10.0 ** rng.uniform(-6, -1))
        st = check(x, oracle.ABS, value)
        assert st == oracle.OK
        u = ulp_above(np.abs(x).max())
        target = 2 * (Fraction(value) - 4 * u)
        differs += nearest_f32(target) != largest_f32_not_above(target)
    assert differs > 100


def test_step_exact_when_binary64_difference_rounds():
    """eb far above max|x|: the binary64 difference eb - 4u rounds back to eb,
    while the exact 2 (eb - 4u) lies just below a binary32 number."""
    cases = 0
    for value in (0.5, 0.75, 3.0, 1024.0, 0.15625):
        for m in (1e-12, 3e-20, 7e-30):
            x = np.array([m, -m / 3, 0.0], dtype=np.float32)
            u = ulp_above(np.abs(x).max())
            naive = np.float32(2.0 * (value - float(4 * u)))  # binary64 difference, then binary32
            st, E, _, _ = oracle.resolve(x, oracle.ABS, value)
            assert st == oracle.OK
            assert Fraction(float(np.float32(E))) < 2 * (Fraction(value) - 4 * u)  # strictly below
            assert np.float32(E) == f32_down(naive)
            check(x, oracle.ABS, value)
            cases += 1
    assert cases == 15


@pytest.mark.parametrize("M", [1.0, 0.75, 3.0e-3, 1000.0, 6.0e37, 2.0 ** -100])
def test_threshold_at_eight_ulp_abs(M):
    x = np.array([M, -M / 2, 0.0], dtype=np.float32)
    u = ulp_above(np.float32(M))
    at = float(8 * u)  # a power of two: exact in binary64
    assert Fraction(at) == 8 * u
    st, E, _, _ = oracle.resolve(x, oracle.ABS, at)
    assert st == oracle.OK and Fraction(float(np.float32(E))) == 8 * u  # 2 (8u - 4u) = 8u exactly
    below = float(np.nextafter(at, 0.0))
    assert oracle.resolve(x, oracle.ABS, below)[0] == oracle.ERR_EB_TOO_SMALL
    check(x, oracle.ABS, at)
    check(x, oracle.ABS, below)


@pytest.mark.parametrize("M", [1.0, 0.5, 128.0, 2.0 ** -40])
def test_threshold_at_eight_ulp_rel(M):
    """REL with range 2M: value = 4u / M gives eb = 8u exactly (all powers of two)."""
    x = np.array([M, -M, M / 4], dtype=np.float32)
    u = ulp_above(np.float32(M))
    value = float(4 * u / Fraction(float(np.float32(M))))
    assert Fraction(value) * 2 * Fraction(float(np.float32(M))) == 8 * u
    st, E, _, _ = oracle.resolve(x, oracle.REL, value)
    assert st == oracle.OK and Fraction(float(np.float32(E))) == 8 * u
    below = float(np.nextafter(value, 0.0))
    assert oracle.resolve(x, oracle.REL, below)[0] == oracle.ERR_EB_TOO_SMALL
    check(x, oracle.REL, value)
    check(x, oracle.REL, below)


def test_two_ulp_threshold_would_accept_what_the_reading_rejects():
    """Between 2u and 8u the request is rejected (the quantizer's |q| <= 2^21 needs 8u)."""
    x = np.array([1.0, -0.25], dtype=np.float32)
    u = float(ulp_above(np.float32(1.0)))
    for k in (2.0, 3.0, 5.0, 7.0, 7.999):
        assert oracle.resolve(x, oracle.ABS, k * u)[0] == oracle.ERR_EB_TOO_SMALL, k
    assert oracle.resolve(x, oracle.ABS, 8.0 * u)[0] == oracle.OK


def test_subnormal_step_rejected_and_large_step_clamped():
    x = np.array([1e-40, -3e-41], dtype=np.float32)  # subnormal max|x|: u = 2^-149
    assert check(x, oracle.ABS, 1e-39) == oracle.ERR_EB_TOO_SMALL  # E would be subnormal
    assert check(x, oracle.ABS, 1e-37) == oracle.OK
    y = np.array([1.0, 2.0], dtype=np.float32)
    st, E, _, _ = oracle.resolve(y, oracle.ABS, 1e38)
    assert st == oracle.OK and np.float32(E) == np.float32(2.0 ** 126)
    check(y, oracle.ABS, 1e38)
    big = np.array([3.3e38, -1.0], dtype=np.float32)
    assert check(big, oracle.ABS, 1e37) == oracle.ERR_EB_TOO_LARGE
    assert check(big, oracle.ABS, 1e33) == oracle.OK  # 8u = 2^107 < 1e33


@pytest.mark.parametrize("c", [1013.25, -7.5, 3.0e-20, 0.0, 1e-40])
def test_constant_field_rel(c):
    check(np.full(7, c, dtype=np.float32), oracle.REL, 1e-3)
