"""Pins for the splitting u (Algorithm 2) and the map theta(a) = u(Delta a).

u is pinned on monomials (its definition), by its p^-1-linearity, and theta is
pinned three ways: the literal product-then-split, the matrix of Algorithm 5
(TRIV), and the matching example of Section 4.3.
"""
from math import comb

import numpy as np
import pytest

import workloads
from oracle import fast, literal


@pytest.mark.parametrize("p", [3, 5, 7])
def test_split_on_monomials(p):
    e = (p - 1,) * 4
    assert literal.frobenius_split({e: 2}, p) == {(0, 0, 0, 0): 2}
    J = (1, 0, 2, 3)
    E = tuple(p - 1 + p * j for j in J)
    assert literal.frobenius_split({E: 1}, p) == {J: 1}
    # any exponent not = p-1 mod p is killed
    for bad in [(p - 2, p - 1, p - 1, p - 1), (p, p - 1, p - 1, 2 * p - 1), (0, 0, 0, 0)]:
        assert literal.frobenius_split({bad: 1}, p) == {}


@pytest.mark.parametrize("p", [3, 5])
def test_split_is_inverse_frobenius_linear(p):
    # u(b(x^p) * a) = b * u(a): u is a map of S^p-modules (Section 3.2).
    rng = np.random.default_rng(p)
    Bb = literal.monomial_basis(2)
    Ba = literal.monomial_basis(4 * (p - 1))
    for _ in range(3):
        b = {Bb[i]: int(rng.integers(1, p)) for i in rng.choice(len(Bb), 4, replace=False)}
        a = {Ba[i]: int(rng.integers(1, p)) for i in rng.choice(len(Ba), 30, replace=False)}
        phib = {tuple(p * x for x in e): c for e, c in b.items()}
        lhs = literal.poly_mod(literal.frobenius_split(literal.poly_mul(phib, a), p), p)
        rhs = literal.poly_mod(literal.poly_mul(b, literal.frobenius_split(a, p)), p)
        assert lhs == rhs


def test_matching_example():
    # Section 4.3 example: delta = (21,19,22,18), p = 5, B_16.  The printed list
    # has (8,7,0,1), which does not match (8,7,0,1) mod 5 = (3,2,0,1) != (3,0,2,1);
    # the reading is (8,5,2,1), the element of m(X) + 5*wics(2,4) it stands for.
    printed = {(13, 0, 2, 1), (8, 7, 0, 1), (8, 0, 7, 1), (8, 0, 2, 6), (3, 10, 2, 1),
               (3, 5, 7, 1), (3, 5, 2, 6), (3, 0, 12, 1), (3, 0, 7, 6), (3, 0, 2, 11)}
    reading = (printed - {(8, 7, 0, 1)}) | {(8, 5, 2, 1)}
    got = literal.matching_monomials((21, 19, 22, 18), 5, 16)
    assert set(got) == reading and len(got) == 10
    assert (8, 7, 0, 1) not in got
    # the matches are m(X) + p * wics(2, 4) with m(X) = (3,0,2,1) (Lemma "generate matching")
    assert set(got) == {tuple(3 * (i == 0) + 2 * (i == 2) + (i == 3) + 5 * w[i] for i in range(4))
                        for w in literal.weak_compositions(2, 4)}
    # Corollary "number of matches": at most binom(floor(16/5) + 3, 3)
    assert len(got) <= comb(16 // 5 + 3, 3)


@pytest.mark.parametrize("p,nterms_a", [(3, 165), (3, 40), (5, 25)])
def test_theta_c_tier_equals_product_then_split(p, nterms_a):
    d, D = 4 * (p - 1), 4 * p * (p - 1)
    ld, lD = comb(d + 3, 3), comb(D + 3, 3)
    for s in range(2):
        delta = workloads.random_dense(p, lD, seed=50 + s)
        a = workloads.random_poly(p, nterms_a, ld, seed=60 + s)
        want = literal.theta_literal(literal.poly_from_dense(delta, D), literal.poly_from_dense(a, d), p)
        got = literal.poly_from_dense(fast.theta(delta, a, p), d)
        assert got == want
        assert literal.theta_matched(literal.poly_from_dense(delta, D), literal.poly_from_dense(a, d), p) == want


def test_theta_equals_triv_matrix():
    # Algorithm 5 builds the matrix of g -> u(Delta g); theta must equal M a.
    p = 3
    d, D = 8, 24
    delta = workloads.random_dense(p, comb(D + 3, 3), seed=5)
    M, Bd, Bdp = literal.triv_matrix(literal.poly_from_dense(delta, D), p, d)
    assert Bd == Bdp and len(Bd) == 165
    for s in range(3):
        a = workloads.random_dense(p, 165, seed=70 + s)
        want = [0] * 165
        for (r, c), v in M.items():
            want[r] = (want[r] + v * int(a[c])) % p
        assert list(fast.theta(delta, a, p)) == want


def test_theta_sign_convention():
    # Negating Delta (the opposite sign convention for Delta_1) negates theta.
    p = 5
    delta = workloads.random_dense(p, comb(83, 3), seed=9)
    a = workloads.random_dense(p, 969, seed=10)
    neg = ((p - delta.astype(np.int64)) % p).astype(np.uint8)
    t1 = fast.theta(delta, a, p).astype(np.int64)
    t2 = fast.theta(neg, a, p).astype(np.int64)
    assert np.all((t1 + t2) % p == 0)
