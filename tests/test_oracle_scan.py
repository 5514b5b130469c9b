"""Pins of the oracle's cumulative weights (Sec. I, Eq. 3).

The reference values are computed in exact rational arithmetic (every binary64
and binary32 number is a dyadic rational) and rounded once to binary64, which
Python's Fraction -> float conversion does correctly.
"""
from fractions import Fraction

import numpy as np
import pytest


def _exact_W(w):
    fr = [Fraction(float(x)) for x in w]
    T = sum(fr, Fraction(0))
    out = []
    S = Fraction(0)
    for x in fr:
        S += x
        out.append(float(S / T))
    out[-1] = 1.0
    return np.array(out)


def _ulp_diff(a, b):
    ia = a.view(np.int64)
    ib = b.view(np.int64)
    return np.abs(ia - ib)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("kind", ["lognormal", "zeros", "wide", "one"])
def test_W_exact_rounding(oracle_mod, dtype, kind):
    rng = np.random.default_rng(11)
    M = 1 if kind == "one" else 700
    if kind == "lognormal":
        w = np.exp(rng.normal(0, 3, M))
    elif kind == "zeros":
        w = np.exp(rng.normal(0, 1, M))
        w[rng.random(M) < 0.3] = 0.0
        w[-1] = 0.0                      # zero-weight last bin
    elif kind == "wide":
        w = np.exp(rng.uniform(-40, 40, M))   # 35 decades: catastrophic for naive sums
    else:
        w = np.array([0.3])
    w = w.astype(dtype)
    W, tot = oracle_mod.cumulative_weights(w)
    ref = _exact_W(w)
    d = _ulp_diff(W, ref)
    assert d.max() <= 1
    assert (d == 0).mean() >= 0.99
    assert W[-1] == 1.0
    assert np.all(np.diff(W) >= 0)
    exact_total = float(sum((Fraction(float(x)) for x in w), Fraction(0)))
    assert abs(tot - exact_total) <= 2 * np.spacing(exact_total)


def test_W_against_exact_large(oracle_mod):
    """A longer, heavy-tailed instance checked on a sample of positions."""
    rng = np.random.default_rng(12)
    M = 20000
    w = np.exp(rng.normal(0, 5, M))
    W, _ = oracle_mod.cumulative_weights(w)
    fr = [Fraction(float(x)) for x in w]
    T = sum(fr, Fraction(0))
    S = Fraction(0)
    idx = set(rng.integers(0, M, 200).tolist())
    for j, x in enumerate(fr):
        S += x
        if j in idx and j < M - 1:
            assert abs(W[j] - float(S / T)) <= np.spacing(W[j])


@pytest.mark.parametrize("bad", [-1.0, np.nan, np.inf])
def test_W_rejects_bad_weights(oracle_mod, bad):
    w = np.ones(10)
    w[4] = bad
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.cumulative_weights(w)


def test_W_rejects_zero_total(oracle_mod):
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.cumulative_weights(np.zeros(5))


def test_zero_weights_repeat_W_exactly(oracle_mod):
    """The oracle's exact sums give a weight of zero an empty interval: W_j ==
    W_{j-1} (and W_0 == 0 for a leading zero), the property the GPU tests pin
    the blocked sums to."""
    rng = np.random.Generator(np.random.PCG64(12))
    w = np.exp(rng.normal(0.0, 3.0, 100_000))
    w[:50] = 0.0
    w[rng.random(w.size) < 0.3] = 0.0
    w[-70:] = 0.0
    W, _ = oracle_mod.cumulative_weights(w)
    z = np.flatnonzero(w == 0)
    assert W[0] == 0.0
    assert np.array_equal(W[z[z > 0]], W[z[z > 0] - 1])
    assert W[-1] == 1.0
