"""Pins the oracle's probability-q decision (threshold K and per-sample bit).

The paper makes probability-d bits from AND/OR of random words (Sec. 4.2:
d = 1/2 is one random word, d = 1/4 the AND of two) and probability-p bits as
the AND of independent 1/4-bits with one word-wide comparison against 4p
(Sec. 4.3, p < 1/4). The generalised decision must reduce to exactly those
constructions, and every sample's marginal must be exactly K / 2^34."""
import numpy as np
import pytest

from oracle import oracle

TWO32 = 1 << 32


def _bits(x, b):
    return (x >> b) & 1


def test_threshold_closed_forms():
    assert oracle.threshold(0.0) == 0
    assert oracle.threshold(0.25) == TWO32
    assert oracle.threshold(0.5) == 2 * TWO32
    assert oracle.threshold(0.75) == 3 * TWO32
    assert oracle.threshold(1.0) == 4 * TWO32
    # round half to even at the exact midpoint between two integers
    assert oracle.threshold(2.5 / 2**34) == 2
    assert oracle.threshold(3.5 / 2**34) == 4
    # outside [0, 1] is rejected
    assert oracle.threshold(-1e-300) == 2**64 - 1
    assert oracle.threshold(1.0000001) == 2**64 - 1
    assert oracle.threshold(float("nan")) == 2**64 - 1


@pytest.mark.parametrize("q", [0.1, 0.9, 0.123456, 0.191789, 0.5 + 2**-30])
def test_threshold_error_bound(q):
    K = oracle.threshold(q)
    assert abs(K / 2**34 - q) <= 2**-35


def _random_words(n, seed):
    rng = np.random.default_rng(seed)
    x1 = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    x2 = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    g = rng.integers(0, 2**32, size=n, dtype=np.uint64)
    return [int(v) for v in x1], [int(v) for v in x2], [int(v) for v in g]


@pytest.mark.parametrize("q,form", [
    (0.5, lambda a, b: 1 - a),                 # one random word (Sec. 4.2, d = 1/2)
    (0.25, lambda a, b: (1 - a) & (1 - b)),    # AND of two random words (d = 1/4)
    (0.75, lambda a, b: 1 - (a & b)),          # OR of two words (d = 3/4)
    (0.0, lambda a, b: 0),
    (1.0, lambda a, b: 1),
])
def test_dyadic_rates_reduce_to_and_or_of_words(q, form):
    K = oracle.threshold(q)
    x1, x2, g = _random_words(40, 7)
    for i in range(40):
        for b in range(64):
            expect = form(_bits(x1[i], b), _bits(x2[i], b))
            assert oracle.decide(x1[i], x2[i], g[i], K, b) == expect


@pytest.mark.parametrize("p", [0.05, 0.125141, 0.2, 0.249])
def test_small_p_is_two_quarter_bits_and_a_shared_comparison(p):
    """p < 1/4: bit b is set iff both its 1/4-bits fire and the word-wide
    uniform g/2^32 is below 4p, as in Sec. 4.3."""
    K = oracle.threshold(p)
    assert K < TWO32
    x1, x2, g = _random_words(30, 11)
    # force both sides of the shared comparison to occur
    g[0], g[1] = K - 1, K
    for i in range(30):
        shared = 1 if g[i] < K else 0
        for b in range(64):
            expect = (1 - _bits(x1[i], b)) & (1 - _bits(x2[i], b)) & shared
            assert oracle.decide(x1[i], x2[i], g[i], K, b) == expect


@pytest.mark.parametrize("q", [0.1, 0.3, 0.6, 0.9, 0.123456, 1.0 - 2**-34])
def test_marginal_is_exactly_K_over_2_34(q):
    """For fixed g, the number of prefixes u in {0..3} that fire is
    min(4, K>>32) + [K>>32 < 4 and g < K mod 2^32]; averaging over g gives
    K / 2^34 exactly. Checked at the boundary values of g and at random g."""
    K = oracle.threshold(q)
    Kh, Kl = K >> 32, K & (TWO32 - 1)
    gs = [0, TWO32 - 1, Kl, max(Kl - 1, 0), min(Kl + 1, TWO32 - 1), 12345]
    for g in gs:
        fired = 0
        for a in (0, 1):
            for bb in (0, 1):
                fired += oracle.decide(a, bb, g, K, 0)
        expect = min(4, Kh) + (1 if (Kh < 4 and g < Kl) else 0)
        assert fired == expect
    total = min(4, Kh) * TWO32 + (Kl if Kh < 4 else 0)
    assert total == K  # sum over g of fired prefixes / 4 / 2^32 = K / 2^34


@pytest.mark.parametrize("q", [0.1, 0.9, 0.123456])
def test_binomial_frequency(q):
    K = oracle.threshold(q)
    x1, x2, g = _random_words(400, 99)
    hits = sum(oracle.decide(x1[i], x2[i], g[i], K, b) for i in range(400) for b in range(0, 64, 3))
    n = 400 * len(range(0, 64, 3))
    sigma = (n * q * (1 - q)) ** 0.5
    # samples of one word share g, so allow a generous band
    assert abs(hits - n * q) < 8 * sigma
