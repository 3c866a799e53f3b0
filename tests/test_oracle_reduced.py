"""Pins for the reduced height oracle (oracle/reduced.py, derivation in oracle/REDUCED.md).

The reduced form is not an algorithm of the paper, so it is pinned only
against the paper's own algorithms: the key identity
Delta_1(f^(p-1)) = phi(Q) - D phi(H) mod p against Algorithm 1 applied to g,
and the heights against Algorithm 3 (integer tier at p = 3, 5; C tier at
p = 7, 11) and against the heights printed in the paper's tables.
"""
import json
import os

import numpy as np
import pytest

from oracle import fast, literal, reduced

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_heights.json")
B4 = literal.monomial_basis(4)


def _rand_quartic(rng, p, density):
    keep = rng.random(35) < density
    return {B4[i]: int(rng.integers(1, p)) for i in range(35) if keep[i]}


def _dense(f):
    return np.array([f.get(r, 0) for r in B4], dtype=np.uint8)


@pytest.mark.parametrize("p,densities", [(3, (0.15, 0.4, 1.0)), (5, (0.1, 0.2))])
def test_delta1_of_g_identity(p, densities):
    # Delta_1(f^(p-1)) = phi(Q) - D phi(H) mod p, against Algorithm 1 on g itself
    # (integer tier; sparse quartics at p = 5 keep g^p over Z small).
    rng = np.random.default_rng(40 + p)
    for density in densities:
        for _ in range(3):
            f = _rand_quartic(rng, p, density)
            g = literal.poly_mod(literal.poly_pow(literal.lift(f, p), p - 1), p)
            assert reduced.delta1_of_g_reduced(f, p) == literal.delta1(g, p)


def test_heights_match_algorithm3_integer_tier_p3():
    rng = np.random.default_rng(53)
    seen = set()
    for density in (0.1, 0.2, 0.35, 0.6, 1.0):
        for _ in range(8):
            f = _rand_quartic(rng, 3, density)
            h = literal.height(f, 3)
            assert reduced.height(f, 3) == h
            seen.add(h)
    assert len(seen) >= 3  # several heights, including deep ones, are exercised


def test_heights_match_algorithm3_c_tier_p5():
    # the C tier of Algorithm 3 is itself pinned against the integer tier at p = 5
    rng = np.random.default_rng(55)
    seen = set()
    for density in (0.1, 0.2, 0.35, 0.6, 1.0):
        for _ in range(12):
            f = _rand_quartic(rng, 5, density)
            h = fast.height(_dense(f), 5)
            assert reduced.height(f, 5) == h
            seen.add(h)
    assert len(seen) >= 3


def test_heights_match_algorithm3_c_tier_p7():
    rng = np.random.default_rng(77)
    deep = 0
    for density in (0.15, 0.3, 0.5):
        for _ in range(6):
            f = _rand_quartic(rng, 7, density)
            h = fast.height(_dense(f), 7)
            assert reduced.height(f, 7) == h
            deep += h != 1
    assert deep >= 2


def _paper_rows(p):
    doc = json.load(open(GOLDEN))
    return [({B4[i]: int(c) for i, c in enumerate(e["coeffs_b4"]) if c}, 0 if e["height"] == "inf" else e["height"])
            for e in doc["entries"] if e["p"] == p]


@pytest.mark.parametrize("p", [5, 7])
def test_reproduces_paper_heights(p):
    rows = _paper_rows(p)
    assert rows
    for f, h in rows:
        assert reduced.height(f, p) == h


def test_reproduces_paper_heights_p11():
    for f, h in _paper_rows(11):
        assert reduced.height(f, 11) == h


def test_fermat_quartic():
    fermat = {(4, 0, 0, 0): 1, (0, 4, 0, 0): 1, (0, 0, 4, 0): 1, (0, 0, 0, 4): 1}
    assert reduced.height(fermat, 3) == 0
    assert reduced.height(fermat, 5) == 1
    assert reduced.height(fermat, 7) == 0
