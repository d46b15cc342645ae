"""Pins of the oracle's deterministic log2/exp2 and hash (CPU only).

The transcendental functions are the textbook series named in the oracle
(atanh series for ln, Taylor series for e^a).  They are pinned against
mpmath at 60 digits (accuracy) and against the independent brute-force
implementation of the same series (bit identity)."""
import math
import random

import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from tests import bruteforce as BF

mpmath.mp.dps = 60


def ulp(v):
    return math.ulp(abs(v)) if v != 0 else math.ulp(0.0)


def _inputs(n, seed=1):
    rng = random.Random(seed)
    xs = []
    for _ in range(n):
        e = rng.randint(-1074, 1023)
        xs.append(math.ldexp(1.0 + rng.random(), e) if e > -1023 else math.ldexp(rng.random(), -1022))
    xs = [x for x in xs if x > 0 and math.isfinite(x)]
    edge = [1.0, math.nextafter(1.0, 2), math.nextafter(1.0, 0), 2.0 ** -1074, 2.0 ** -1022,
            math.nextafter(2.0 ** -1022, 0), 1.7976931348623157e308, 1.4142135623730951,
            math.nextafter(1.4142135623730951, 2), 0.7071067811865476, 3.0, 10.0, 1.01]
    return edge + xs


def test_log2_accuracy_vs_mpmath():
    worst = 0.0
    for x in _inputs(20000):
        got = O.det_log2(x)
        ref = mpmath.log(mpmath.mpf(x), 2)
        err = abs(mpmath.mpf(got) - ref)
        if ref != 0:
            worst = max(worst, float(err / mpmath.mpf(ulp(float(ref)))))
        else:
            assert got == 0.0
    assert worst <= 4.0, worst


def test_log2_exact_on_powers_of_two():
    for k in range(-1074, 1024):
        assert O.det_log2(math.ldexp(1.0, k)) == float(k)


def test_exp2_accuracy_vs_mpmath():
    rng = random.Random(7)
    ts = [rng.uniform(-1020, 1020) for _ in range(20000)] + [rng.uniform(-2, 2) for _ in range(2000)]
    worst = 0.0
    for t in ts:
        got = O.det_exp2(t)
        ref = mpmath.power(2, mpmath.mpf(t))
        worst = max(worst, float(abs(mpmath.mpf(got) - ref) / mpmath.mpf(ulp(float(ref)))))
    assert worst <= 4.0, worst


def test_exp2_exact_on_integers():
    for k in range(-1074, 1024):
        assert O.det_exp2(float(k)) == math.ldexp(1.0, k)


def test_log2_exp2_bit_identical_to_independent_series():
    rng = random.Random(3)
    for x in _inputs(3000, seed=5):
        assert O.det_log2(x) == BF.det_log2(x), x
    for _ in range(3000):
        t = rng.uniform(-1100, 1030)
        assert O.det_exp2(t) == BF.det_exp2(t), t


def test_exp2_subnormal_results_match_exact_rounding():
    # results below 2^-1022 go through one rounding in ldexp
    for t in np.linspace(-1074.5, -1021.5, 4001):
        assert O.det_exp2(float(t)) == BF.det_exp2(float(t))


def test_splitmix64_published_first_output():
    # first output of splitmix64 seeded with 0 (reference implementation by Vigna)
    assert O.splitmix64(0) == 0xE220A8397B1DCDAF


def test_bf16_rounding_ties_to_even():
    # 1 + 2^-8 is halfway between bf16 1.0 and 1 + 2^-7: ties to even -> 1.0
    assert O.bf16_rne(1.0 + 2.0 ** -8) == 1.0
    assert O.bf16_rne(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert O.bf16_rne(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert O.bf16_rne(-3.0) == -3.0
