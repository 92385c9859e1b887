"""Pins for the oracle's do_reduce (Section 3: commutative reduction of operator values).

* Exact integer sums: sum_{i<n} i = n(n-1)/2, exactly representable below 2^53.
* math.fsum gives the correctly rounded sum; pairwise summation must be within
  a few ulps of it relative to sum |x|.
* Infinity norm: NaN propagates; empty-free special cases (one element, all equal).
"""
import math

import numpy as np

import oracle


def test_index_sum_exact():
    for n in (1, 2, 17, 1000, 1 << 20):
        x = np.arange(n, dtype=np.float64)
        assert oracle.sum(x) == n * (n - 1) / 2


def test_sum_and_sumsq_against_fsum():
    g = np.random.default_rng(0)
    for n in (1, 5, 33, 100000):
        x = g.standard_normal(n) * np.exp(g.uniform(-20, 20, n))
        s = oracle.sum(x)
        assert abs(s - math.fsum(x)) <= 1e-14 * math.fsum(np.abs(x))
        q = oracle.sumsq(x)
        exact = math.fsum(x * x)  # each square rounded once, as in the oracle
        assert abs(q - exact) <= 1e-14 * exact


def test_maxabs_and_nan():
    x = np.array([0.5, -3.25, 2.0])
    assert oracle.maxabs(x) == 3.25
    y = np.array([1.0, np.nan, 5.0])
    assert math.isnan(oracle.maxabs(y))
    assert oracle.maxabs(np.array([-7.0])) == 7.0
    assert oracle.sum(np.full(1000, 0.125)) == 125.0
