"""Pins of the residual-resampling oracle (Alg. res_res) against what the algorithm fixes:

* masses that are integer multiples of the mean are split deterministically, with no draws;
* the output has P particles of equal mass a0, and P a0 equals the input mass to rounding;
* particle p appears at least k_p = floor(a_p / a0) times, at most k_p + 1 per draw, and a
  particle with no residual is never drawn;
* the mean is the exact rational mean, correctly rounded, divided by P;
* over many independent draws, the extra copies follow r_p / sum_q r_q (chi-square), with
  the residuals computed here in exact rational arithmetic.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import resample as RS
from paper_2605_20140_amd import workloads as W


def _X(P, seed=0):
    return np.random.default_rng(seed).random((P, 3))


def test_integer_multiples_split_deterministically():
    a = np.array([2.0, 0.0, 1.0, 1.0]) * 0.25
    X = _X(4)
    Xn, an, info = RS.residual_resample(X, a, n=3, sim_id=0, seed=1)
    assert info["a0"] == 0.25 and info["n_stoch"] == 0
    assert list(info["k"]) == [2, 0, 1, 1]
    assert list(info["src"]) == [0, 0, 2, 3]
    assert np.array_equal(Xn, X[[0, 0, 2, 3]])
    assert np.all(an == 0.25)


def test_equal_masses_are_unchanged():
    P = 64
    a = np.full(P, 1.0 / P)
    X = _X(P)
    Xn, an, info = RS.residual_resample(X, a, n=0, sim_id=0, seed=0)
    assert info["n_stoch"] == 0
    assert np.array_equal(Xn, X) and np.array_equal(an, a)


def test_empty():
    Xn, an, info = RS.residual_resample(np.zeros((0, 3)), np.zeros(0), 0, 0, 0)
    assert Xn.shape == (0, 3) and an.shape == (0,) and info["n_stoch"] == 0


@pytest.mark.parametrize("P,spread", [(1000, 0.5), (4097, 2.0), (50, 4.0)])
def test_counts_mass_and_residual_free_particles(P, spread):
    rng = np.random.default_rng(P)
    a = W.weighted_masses(P, spread, rng)
    a[::7] = 0.0                                   # particles with nothing left
    X = _X(P, 1)
    Xn, an, info = RS.residual_resample(X, a, n=11, sim_id=5, seed=9)
    a0 = info["a0"]
    assert Xn.shape == (P, 3) and np.all(an == a0)
    assert abs(P * a0 - a.sum()) <= 1e-13 * a.sum()
    cnt = np.bincount(info["src"], minlength=P)
    k = info["k"]
    assert cnt.sum() == P
    assert np.all(cnt >= k)
    extra = cnt - k
    assert extra.sum() == info["n_stoch"] == P - k.sum()
    assert np.all(extra[info["R"] == 0] == 0)
    assert np.all(extra[a == 0.0] == 0) and np.all(cnt[a == 0.0] == 0)
    # outputs are copies of inputs
    assert np.array_equal(Xn, X[info["src"]])


def test_mean_is_correctly_rounded():
    rng = np.random.default_rng(3)
    a = W.weighted_masses(3001, 3.0, rng) * 1e-3
    a[5] = 1e20 * a[4]                              # cancellation-prone magnitudes
    exact = sum((Fraction(float(x)) for x in a), Fraction(0))
    S = float(exact)                                # correctly rounded (round half even)
    assert RS.mean_mass(a) == S / a.shape[0]


def test_draw_frequencies_follow_residuals():
    a = np.array([0.5, 1.3, 2.2, 0.7, 0.3])        # mean 1: k = (0, 1, 2, 0, 0), 2 draws
    P = a.shape[0]
    X = _X(P)
    extra = np.zeros(P)
    calls = 3000
    for n in range(calls):
        _, _, info = RS.residual_resample(X, a, n=n, sim_id=2, seed=77)
        assert list(info["k"]) == [0, 1, 2, 0, 0] and info["n_stoch"] == 2
        extra += np.bincount(info["src"], minlength=P) - info["k"]
    # exact residuals r_p = a_p - k_p a0 with a0 the rational mean
    fa = [Fraction(float(x)) for x in a]
    a0 = sum(fa, Fraction(0)) / P
    r = [x - int(x / a0) * a0 for x in fa]
    prob = np.array([float(x / sum(r, Fraction(0))) for x in r])
    expected = prob * extra.sum()
    chi2 = float(((extra - expected) ** 2 / expected).sum())
    # 4 degrees of freedom: P(chi2 > 23.5) ~ 1e-4
    assert chi2 < 23.5, (extra, expected)


def test_distinct_steps_and_simulations_draw_differently():
    rng = np.random.default_rng(8)
    a = W.weighted_masses(2000, 1.0, rng)
    X = _X(2000)
    s1 = RS.residual_resample(X, a, n=4, sim_id=0, seed=1)[2]["src"]
    s2 = RS.residual_resample(X, a, n=5, sim_id=0, seed=1)[2]["src"]
    s3 = RS.residual_resample(X, a, n=4, sim_id=1, seed=1)[2]["src"]
    s4 = RS.residual_resample(X, a, n=4, sim_id=0, seed=1)[2]["src"]
    assert np.array_equal(s1, s4)
    assert not np.array_equal(s1, s2) and not np.array_equal(s1, s3)


def test_resampling_stream_is_not_a_step_stream():
    """The draws use counter word 3 with its top bit set: they never coincide with the words
    of a step's Wiener increments for sim_id < 2^63."""
    from oracle.philox import philox4x32_10
    u = RS.draws(4, n=7, sim_id=3, seed=5)
    r0, r1, _, _ = philox4x32_10(np.arange(4, dtype=np.uint64), np.uint64(7), np.uint64(3),
                                 np.uint64(0), np.uint64(5), np.uint64(0))
    step_words = [int(x) | (int(y) << 32) for x, y in zip(r0, r1)]
    assert all(x != y for x, y in zip(u, step_words))
