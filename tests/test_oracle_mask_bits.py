"""Pins of the oracle's decorrelation bits m (paper Sec. 4.3: independent
random bits per sample under the shared, word-wide comparison). A decision of
probability q fires for sample b iff U_b = u_b * 2^32 + g < K = rint(q 2^(32+m)),
u_b the m-bit number of bit b of X1..Xm and g shared by the word's samples.

The expected values are closed forms of that definition, not the oracle's
arithmetic retyped: the paper's AND/OR constructions at dyadic rates, the
exact firing probability and the exact covariance the shared g induces
between two samples of one word, and whole trajectories that must not depend
on m where the two rules fire on the same bits."""
import numpy as np
import pytest

from oracle import oracle

ALL = (1 << 64) - 1


def _words(rng, n):
    return [int(x) for x in rng.integers(0, 1 << 63, size=n, dtype=np.int64) * 2
            + rng.integers(0, 2, size=n)]


@pytest.mark.parametrize("j", range(0, 17))
def test_sixteenths_are_comparisons_of_the_four_bits(j):
    """q = j/16 with m = 4: K = j 2^32 exactly, so g never matters and sample b
    fires iff its four bits read as a number are below j; j = 8 is 'bit of X1
    is 0' (the paper's d = 1/2 word), j = 4 'bits of X1 and X2 are 0' (its
    AND of two words), j = 16 always."""
    rng = np.random.default_rng(j)
    K = oracle.threshold_m(j / 16, 4)
    assert K == j << 32
    for _ in range(20):
        xs = _words(rng, 4)
        g = int(rng.integers(0, 1 << 32))
        for b in range(0, 64, 7):
            u = sum(((xs[i] >> b) & 1) << (3 - i) for i in range(4))
            assert oracle.decide_m(xs, g, K, b) == int(u < j)
    x1 = _words(rng, 1)[0]
    xs = [x1] + _words(rng, 3)
    if j == 8:
        assert all(oracle.decide_m(xs, 123, K, b) == 1 - ((x1 >> b) & 1) for b in range(64))


@pytest.mark.parametrize("q", [0.0, 0.25, 0.5, 0.75, 1.0])
def test_quarters_fire_on_the_same_bits_for_m_2_and_4(q):
    """At q in {0, 1/4, 1/2, 3/4, 1} both rules fire iff the top two bits
    (X1, X2) are below 4q, whatever X3, X4 and g are."""
    rng = np.random.default_rng(int(q * 100))
    K2, K4 = oracle.threshold_m(q, 2), oracle.threshold_m(q, 4)
    for _ in range(40):
        xs = _words(rng, 4)
        g = int(rng.integers(0, 1 << 32))
        for b in range(0, 64, 5):
            a = oracle.decide_m(xs[:2], g, K2, b)
            assert a == oracle.decide_m(xs, g, K4, b)
            assert a == oracle.decide(xs[0], xs[1], g, K2, b)


@pytest.mark.parametrize("model,p,d", [("pcpd", 0.25, 0.5), ("tcpd", 0.75, 0.25),
                                       ("dp", 0.5, 0.75), ("pcpd", 1.0, 0.0)])
def test_trajectories_do_not_depend_on_m_at_quarter_rates(model, p, d):
    """Whole runs at rates in quarters: m = 4 (which also draws X3, X4 from
    two more Philox calls) gives the m = 2 lattice and counts bit for bit."""
    runs = [oracle.Run(model=model, B=16, L=16 * 9, seed=3, stream=2, plane=1, p=p, d=d,
                       times=[2, 7], mask_bits=m) for m in (2, 4)]
    for r in runs:
        oracle.simulate(r)
    np.testing.assert_array_equal(runs[0].words, runs[1].words)
    np.testing.assert_array_equal(runs[0].n, runs[1].n)


def test_other_rates_differ_between_m_2_and_4():
    runs = [oracle.Run(model="pcpd", B=16, L=16 * 9, seed=3, stream=2, p=0.3, d=0.1,
                       times=[5], mask_bits=m) for m in (2, 4)]
    for r in runs:
        oracle.simulate(r)
    assert not np.array_equal(runs[0].words, runs[1].words)


@pytest.mark.parametrize("m", [2, 4])
def test_firing_rate_and_shared_tail_covariance(m):
    """Over random words: the firing rate of a sample is q, and two samples of
    one word are correlated only through the shared g, when both draw u equal
    to K's integer part kh: Cov = 2^-2m f (1 - f), f = (K mod 2^32) / 2^32,
    i.e. 16 times smaller with m = 4 than with m = 2."""
    q = 0.3
    K = oracle.threshold_m(q, m)
    f = (K & 0xFFFFFFFF) / 2.0 ** 32
    rng = np.random.default_rng(11 + m)
    n = 6000
    a = np.empty(n)
    c = np.empty(n)
    for i in range(n):
        xs = _words(rng, m)
        g = int(rng.integers(0, 1 << 32))
        a[i] = oracle.decide_m(xs, g, K, 5)
        c[i] = oracle.decide_m(xs, g, K, 41)
    assert abs(a.mean() - q) < 4 * np.sqrt(q * (1 - q) / n)
    cov = float(np.mean(a * c) - a.mean() * c.mean())
    want = 2.0 ** (-2 * m) * f * (1 - f)
    # standard error of a covariance estimate of two Bernoulli(q) variables
    se = q * (1 - q) / np.sqrt(n)
    assert abs(cov - want) < 4 * se, (cov, want, se)
    if m == 2:
        assert want > 0.009   # 1/16 x 0.2 x 0.8: large enough to be seen


def test_bad_mask_bits_are_refused():
    with pytest.raises(ValueError):
        oracle.simulate(oracle.Run(model="pcpd", B=16, L=32, p=0.1, d=0.5, times=[1],
                                   mask_bits=3))
    assert oracle.threshold_m(0.5, 3) == ALL
