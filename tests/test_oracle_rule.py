"""Pins the oracle's window rule against the reaction list of eq. (1), written
as string rewrites, for every window state and every decision triple.

The rewrite form below is a second reading of the model, independent of the
oracle's if/else code: a decision selects one reaction (diffusion, pair
annihilation, fission right, fission left); the reaction fires only where its
left-hand pattern matches the window, and then its right-hand side replaces
the matched sites. For DP, TCPD and QCPD (paper Sec. 1) the reaction lists are
the n-tuple analogues: DP A->0, A0->AA, 0A->AA; TCPD AAA->000, AAA0->AAAA,
0AAA->AAAA; QCPD AAAA->0000, AAAA0->AAAAA, 0AAAA->AAAAA."""
import itertools

import pytest

from oracle import oracle


def reactions(n):
    """(name, offset from the window's first site j-1, lhs, rhs)."""
    tup = "A" * n
    return {
        "diffuse": [(1, "A0", "0A"), (1, "0A", "A0")],      # sites j, j+1
        "annihilate": [(1, tup, "0" * n)],                  # sites j..j+n-1
        "fission_high": [(1, tup + "0", tup + "A")],        # sites j..j+n
        "fission_low": [(0, "0" + tup, "A" + tup)],         # sites j-1..j+n-1
    }


def rewrite(n, window, choice):
    s = list(window)
    for off, lhs, rhs in reactions(n)[choice]:
        if "".join(s[off:off + len(lhs)]) == lhs:
            s[off:off + len(lhs)] = list(rhs)
            break
    return "".join(s)


def choice_of(D, A, R):
    """Which reaction the three decision bits select (Algorithm 1's order:
    diffusion first; otherwise annihilation; otherwise fission, R = high)."""
    if D:
        return "diffuse"
    if A:
        return "annihilate"
    return "fission_high" if R else "fission_low"


def to_str(bits, width):
    return "".join("A" if (bits >> i) & 1 else "0" for i in range(width))


def from_str(s):
    return sum(1 << i for i, c in enumerate(s) if c == "A")


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_rule_table_exhaustive(n):
    width = n + 2
    for state in range(1 << width):
        for D, A, R in itertools.product((0, 1), repeat=3):
            got = oracle.rule_window(n, state, D, A, R)
            want = from_str(rewrite(n, to_str(state, width), choice_of(D, A, R)))
            assert got == want, (n, to_str(state, width), D, A, R, to_str(got, width))


def test_pcpd_rule_examples():
    """Hand-worked windows (sites j-1, j, j+1, j+2) for the four PCPD reactions."""
    n = 2
    f = lambda s, D, A, R: to_str(oracle.rule_window(n, from_str(s), D, A, R), 4)
    assert f("0AA0", 0, 0, 1) == "0AAA"   # AA0 -> AAA
    assert f("0AA0", 0, 0, 0) == "AAA0"   # 0AA -> AAA
    assert f("0AA0", 0, 1, 1) == "0000"   # AA -> 00
    assert f("0A00", 1, 0, 0) == "00A0"   # A0 -> 0A
    assert f("00A0", 1, 1, 1) == "0A00"   # 0A -> A0 (diffusion wins over the rest)
    assert f("0A0A", 0, 1, 1) == "0A0A"   # no pair at (j, j+1): nothing happens
    assert f("AAAA", 0, 0, 0) == "AAAA"   # fission onto an occupied site
