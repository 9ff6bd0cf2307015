"""Pins of the oracle's connected multispin layout (paper Sec. 4: the 64 bits
of a plane joined into one ring of 64 L sites, site b*L + j in bit b of word
j, sites of one word L apart, a bit rotation at the seam).

Every expected value here is derived from the definition, not from the
oracle's simulation code: particle trajectories under pure diffusion from the
substep offsets alone, and the outcome of seam-straddling windows from the
Philox words and the decision rule (both pinned elsewhere) read at the bit of
the window's column.
"""
import numpy as np
import pytest

from oracle import oracle

ALL = (1 << 64) - 1


def words_from_sites(q, L):
    """uint64 words of a joined ring given in global site order."""
    q = np.asarray(q, dtype=np.uint64).reshape(64, L)        # [bit, word]
    w = np.zeros(L, dtype=np.uint64)
    for b in range(64):
        w |= q[b] << np.uint64(b)
    return w


def sites_from_words(w, L):
    bits = (np.asarray(w, dtype=np.uint64)[None, :] >> np.arange(64, dtype=np.uint64)[:, None]) & np.uint64(1)
    return bits.astype(np.uint8).reshape(64 * L)


def _run(**kw):
    r = oracle.Run(connected=True, **kw)
    return oracle.simulate(r)


@pytest.mark.parametrize("seed,stream,B,L", [(1, 0, 8, 16), (5, 3, 4, 8), (9, 7, 16, 16),
                                              (2, 11, 6, 12)])
def test_pure_diffusion_carries_a_particle_across_the_seam(seed, stream, B, L):
    """With d = 1 every attempt swaps (g, g+1): a lone particle at x moves to
    x+1 when x is a window site (x = o mod B), to x-1 when x-1 is, else stays.
    Its path is fixed by the offsets alone; on the joined ring it passes from
    one bit to the next at the seam instead of wrapping inside its own bit."""
    M = 64 * L
    T = 40
    starts = [3 * L + L - 1, 0, 63 * L + L - 1, 17 * L + 2]
    crossings = 0
    for x0 in starts:
        q = np.zeros(M, dtype=np.uint8)
        q[x0] = 1
        init = words_from_sites(q, L)
        r = _run(model="pcpd", B=B, L=L, seed=seed, stream=stream, p=0.3, d=1.0,
                 init="host", init_words=init, times=[T])
        x = x0
        for t in range(T):
            for sub in range(B):
                o = oracle.offset(seed, stream, 0, t * B + sub, B)
                before = x
                if (x - o) % B == 0:
                    x = (x + 1) % M
                elif (x - 1 - o) % B == 0:
                    x = (x - 1) % M
                crossings += (before // L) != (x // L)
        want = np.zeros(M, dtype=np.uint8)
        want[x] = 1
        np.testing.assert_array_equal(r.words, words_from_sites(want, L), err_msg=f"start {x0}")
        assert int(r.n.sum()) == 1
    assert crossings > 0   # the paths did cross between bits


def _seam_substep(B, L, o_want, seed, stream, lo=0):
    """A substep index whose offset is o_want."""
    for s in range(lo, lo + 100000):
        if oracle.offset(seed, stream, 0, s, B) == o_want:
            return s
    raise AssertionError("no substep with that offset")


def _draws(seed, stream, s, k):
    key = (seed, stream)
    x = [oracle.philox((k, d, s & 0xFFFFFFFF, s >> 32), key) for d in (0, 1, 2)]
    x1d, x2d = x[0][0] | x[0][1] << 32, x[0][2] | x[0][3] << 32
    x1a, x2a = x[1][0] | x[1][1] << 32, x[1][2] | x[1][3] << 32
    return x1d, x2d, x1a, x2a, x[2][0] | x[2][1] << 32, x[2][2], x[2][3]


@pytest.mark.parametrize("p", [0.0, 0.5])
def test_seam_pairs_fission_and_annihilate_by_their_columns_bit(p):
    """A pair that straddles the seam of every column (sites b*L + L-1 and
    (b+1)*L) in a substep whose windows sit on it (o = B-1): with d = 0 the
    window of column b annihilates the pair if bit b of its annihilation
    decision fires, else creates a particle at b*L + L-2 (low, R_b = 0) or at
    (b+1)*L + 1 (high, R_b = 1)."""
    B, L, seed, stream = 8, 16, 4, 2
    M = 64 * L
    s = _seam_substep(B, L, B - 1, seed, stream)
    q = np.zeros(M, dtype=np.uint8)
    for b in range(0, 64, 3):       # every third column, so the windows' reaches stay apart
        q[b * L + L - 1] = 1
        q[((b + 1) * L) % M] = 1
    out = oracle.connected_substep("pcpd", B, L, seed, stream, 0, p, 0.0, s, q)
    x1d, x2d, x1a, x2a, R, gd, ga = _draws(seed, stream, s, L // B - 1)
    Kp = oracle.threshold(p)
    want = q.copy()
    for b in range(0, 64, 3):
        g = b * L + L - 1
        A = oracle.decide(x1a, x2a, ga, Kp, b)
        if A:
            want[g] = 0
            want[(g + 1) % M] = 0
        elif (R >> b) & 1:
            want[(g + 2) % M] = 1
        else:
            want[g - 1] = 1
    np.testing.assert_array_equal(out, want)
    if p == 0.0:
        assert out.sum() > q.sum()


def test_diffusion_decision_of_a_seam_window_reads_its_columns_bit():
    """A lone particle on each seam window's first site (b*L + L-1, o = B-1,
    PCPD): with probability d it is swapped to (b+1)*L, decided by bit b of
    the diffusion draw; otherwise nothing happens (no pair)."""
    B, L, seed, stream = 8, 16, 6, 9
    M = 64 * L
    s = _seam_substep(B, L, B - 1, seed, stream, lo=500)
    q = np.zeros(M, dtype=np.uint8)
    for b in range(0, 64, 2):
        q[b * L + L - 1] = 1
    out = oracle.connected_substep("pcpd", B, L, seed, stream, 0, 0.1, 0.5, s, q)
    x1d, x2d, *_ , gd, ga = _draws(seed, stream, s, L // B - 1)
    Kd = oracle.threshold(0.5)
    want = q.copy()
    moved = 0
    for b in range(0, 64, 2):
        g = b * L + L - 1
        if oracle.decide(x1d, x2d, gd, Kd, b):
            want[g], want[(g + 1) % M] = 0, 1
            moved += 1
    np.testing.assert_array_equal(out, want)
    assert 0 < moved < 32


def test_simulation_is_the_substeps_in_order_with_column_counts():
    """orc_simulate in the connected layout equals its substeps applied one by
    one (substep index t*B + b), and its per-column counts sum to the
    particles and to the nearest-neighbour pairs of the joined ring."""
    B, L, seed, stream = 8, 24, 3, 5
    M = 64 * L
    rng = np.random.default_rng(1)
    q0 = (rng.random(M) < 0.4).astype(np.uint8)
    init = words_from_sites(q0, L)
    times = [2, 5]
    r = _run(model="tcpd", B=B, L=L, seed=seed, stream=stream, p=0.2, d=0.3, init="host",
             init_words=init, times=times)
    q = q0.copy()
    t = 0
    for k, T in enumerate(times):
        for tt in range(t, T):
            for sub in range(B):
                q = oracle.connected_substep("tcpd", B, L, seed, stream, 0, 0.2, 0.3,
                                             tt * B + sub, q)
        t = T
        assert int(r.n[k].sum()) == int(q.sum())
        assert int(r.pair[k].sum()) == int((q & np.roll(q, -1)).sum())
        for b in range(64):
            assert int(r.n[k, b]) == int(q[b * L:(b + 1) * L].sum())
    np.testing.assert_array_equal(r.words, words_from_sites(q, L))
    np.testing.assert_array_equal(sites_from_words(r.words, L), q)


def test_connected_invariants():
    B, L = 8, 16
    full = _run(model="pcpd", B=B, L=L, seed=1, p=0.1, d=0.5, times=[0, 1])
    assert int(full.n[0].sum()) == 64 * L and int(full.pair[0].sum()) == 64 * L
    empty = _run(model="pcpd", B=B, L=L, seed=1, p=0.1, d=0.5, init="empty", times=[3])
    assert int(empty.n.sum()) == 0
    rng = np.random.default_rng(2)
    init = words_from_sites((rng.random(64 * L) < 0.5).astype(np.uint8), L)
    diff = _run(model="pcpd", B=B, L=L, seed=2, p=0.7, d=1.0, init="host", init_words=init,
                times=[1, 4, 9])
    n0 = int(sites_from_words(init, L).sum())
    assert all(int(diff.n[k].sum()) == n0 for k in range(3))
    ann = _run(model="pcpd", B=B, L=L, seed=2, p=1.0, d=0.0, init="host", init_words=init,
               times=[1, 2, 3])
    totals = [n0] + [int(ann.n[k].sum()) for k in range(3)]
    assert all(a >= b for a, b in zip(totals, totals[1:])) and totals[-1] < n0


def test_connected_differs_from_classical_only_through_the_seam():
    """Away from the seam the two layouts apply identical windows with
    identical decisions: with d = 1 (deterministic moves) a particle that
    never reaches the first or last word of its bit follows the same path in
    both layouts."""
    B, L, seed, stream = 8, 64, 1, 0
    x0 = 5 * L + 30
    q = np.zeros(64 * L, dtype=np.uint8)
    q[x0] = 1
    init = words_from_sites(q, L)
    c = _run(model="pcpd", B=B, L=L, seed=seed, stream=stream, p=0.0, d=1.0, init="host",
             init_words=init, times=[2])
    k = oracle.Run(model="pcpd", B=B, L=L, seed=seed, stream=stream, p=0.0, d=1.0,
                   init="host", init_words=init, times=[2])
    oracle.simulate(k)
    np.testing.assert_array_equal(c.words, k.words)
