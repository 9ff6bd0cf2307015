"""Pins the oracle's dynamics on tiny rings against the exact transition
matrix built from eq. (1).

Exact side: one attempt at site i chooses a reaction with probability equal to
its rate in eq. (1) (diffusion d, annihilation p(1-d), each fission
(1-p)(1-d)/2; they sum to 1) and applies it where its pattern matches. With
block width B the substep picks an offset uniformly and attempts every block
at that offset; blocks are independent. One Monte Carlo step is B substeps.

Empirical side: the oracle, one sample per (stream) so that runs are
independent, many streams. A chi-square test compares the histograms."""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle import oracle


def _attempt_distribution(n, state, L, i, p, d):
    """{new_state: probability} for one attempt at site i on a ring."""
    q = [(state >> k) & 1 for k in range(L)]
    out = {}

    def add(s, w):
        key = sum(v << k for k, v in enumerate(s))
        out[key] = out.get(key, 0.0) + w

    # diffusion: A0 <-> 0A on (i, i+1); on AA or 00 it changes nothing
    s = list(q)
    s[i % L], s[(i + 1) % L] = s[(i + 1) % L], s[i % L]
    add(s, d)
    tuple_full = all(q[(i + k) % L] for k in range(n))
    rest = [(p * (1 - d), "ann"), ((1 - p) * (1 - d) / 2, "hi"), ((1 - p) * (1 - d) / 2, "lo")]
    for w, kind in rest:
        s = list(q)
        if tuple_full:
            if kind == "ann":
                for k in range(n):
                    s[(i + k) % L] = 0
            elif kind == "hi":
                s[(i + n) % L] = 1
            else:
                s[(i - 1) % L] = 1
        add(s, w)
    return out


def _substep_matrix(n, L, B, p, d):
    S = 1 << L
    T = np.zeros((S, S))
    nb = L // B
    for state in range(S):
        for o in range(B):
            dist = {state: 1.0}
            for k in range(nb):
                nd = {}
                for st, w in dist.items():
                    for st2, w2 in _attempt_distribution(n, st, L, k * B + o, p, d).items():
                        nd[st2] = nd.get(st2, 0.0) + w * w2
                dist = nd
            for st, w in dist.items():
                T[state, st] += w / B
    return T


def _empirical(n, L, B, p, d, init_state, runs, steps=1, seed=5):
    init = np.array([((init_state >> j) & 1) for j in range(L)], dtype=np.uint64)
    model = {1: "dp", 2: "pcpd", 3: "tcpd", 4: "qcpd"}[n]
    rs = [oracle.Run(model=model, B=B, L=L, seed=seed, stream=r, plane=0, p=p, d=d,
                     samples=1, init="host", init_words=init, times=[steps])
          for r in range(runs)]
    oracle.simulate_many(rs)
    hist = np.zeros(1 << L)
    for r in rs:
        st = sum(int(r.words[j] & np.uint64(1)) << j for j in range(L))
        hist[st] += 1
    return hist


def _chi2_pvalue(hist, probs):
    n = hist.sum()
    exp = probs * n
    big = exp >= 5
    obs_b, exp_b = list(hist[big]), list(exp[big])
    if (~big).any():
        obs_b.append(hist[~big].sum())
        exp_b.append(exp[~big].sum())
    obs_b, exp_b = np.array(obs_b), np.array(exp_b)
    assert hist[probs == 0].sum() == 0, "oracle reached a state eq. (1) forbids"
    keep = exp_b > 0
    chi2 = ((obs_b[keep] - exp_b[keep]) ** 2 / exp_b[keep]).sum()
    dof = keep.sum() - 1
    return stats.chi2.sf(chi2, dof)


CASES = [
    # (n, L, B, p, d, initial state, MC steps)
    (2, 4, 4, 0.3, 0.4, 0b0110, 1),
    (2, 5, 5, 0.2, 0.25, 0b11011, 1),
    (2, 6, 6, 0.1, 0.5, 0b111111, 1),
    (2, 8, 4, 0.35, 0.3, 0b01101100, 1),
    (2, 8, 8, 0.15, 0.6, 0b11100110, 1),
    (3, 5, 5, 0.3, 0.2, 0b01110, 1),
    (3, 7, 7, 0.25, 0.35, 0b1110111, 1),
    (4, 6, 6, 0.3, 0.3, 0b011110, 1),
    (4, 7, 7, 0.2, 0.4, 0b1111011, 1),
    (1, 4, 4, 0.4, 0.3, 0b0010, 1),
    (1, 6, 3, 0.3, 0.2, 0b010010, 1),
]


@pytest.mark.parametrize("n,L,B,p,d,init,steps", CASES)
def test_tiny_ring_transition_frequencies(n, L, B, p, d, init, steps):
    T = _substep_matrix(n, L, B, p, d)
    np.testing.assert_allclose(T.sum(axis=1), 1.0, atol=1e-12)
    M = np.linalg.matrix_power(T, B * steps)
    probs = M[init]
    hist = _empirical(n, L, B, p, d, init, runs=6000, steps=steps)
    pv = _chi2_pvalue(hist, probs)
    assert pv > 1e-5, pv


def test_mistakes_in_the_rule_are_detected():
    """The exact matrix separates the true rates from plausible mistakes
    (rates of fission and annihilation exchanged), so the frequency test
    has power: the oracle's histogram must reject the wrong matrix."""
    n, L, B, p, d, init = 2, 6, 6, 0.1, 0.5, 0b111111
    wrong = np.linalg.matrix_power(_substep_matrix(n, L, B, 1 - p, d), B)[init]
    hist = _empirical(n, L, B, p, d, init, runs=6000)
    n_tot = hist.sum()
    exp = wrong * n_tot
    mask = exp > 0
    # states the wrong model cannot reach would already reject it; otherwise chi2
    if hist[~mask].sum() == 0:
        chi2 = ((hist[mask] - exp[mask]) ** 2 / exp[mask]).sum()
        assert stats.chi2.sf(chi2, mask.sum() - 1) < 1e-10
