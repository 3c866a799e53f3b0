"""Pins for Delta_1 (Algorithm 1) in both oracle tiers.

Delta_1 is pinned to: the binomial theorem (closed form for two terms), its
definition through Witt vector addition in W_2, independence of the integer
lift, the degree statement of Section 3.1, and -- for the C tier -- the
Python-integer tier computed over Z.
"""
from math import comb

import numpy as np
import pytest

import workloads
from oracle import fast, literal


def _rand_terms(rng, p, d, nterms):
    B = literal.monomial_basis(d)
    idx = rng.choice(len(B), size=min(nterms, len(B)), replace=False)
    return {B[i]: int(rng.integers(1, p)) for i in idx}


@pytest.mark.parametrize("p", [3, 5, 7, 11])
def test_binomial_closed_form(p):
    # Delta_1(a x^I + b x^J) = sum_{i=1}^{p-1} (binom(p,i)/p) a^i b^(p-i) x^(iI+(p-i)J) mod p.
    rng = np.random.default_rng(p)
    B = literal.monomial_basis(3)
    for _ in range(5):
        i1, i2 = rng.choice(len(B), size=2, replace=False)
        I, J = B[i1], B[i2]
        a, b = int(rng.integers(1, p)), int(rng.integers(1, p))
        want = {}
        for i in range(1, p):
            e = tuple(i * x + (p - i) * y for x, y in zip(I, J))
            want[e] = (want.get(e, 0) + (comb(p, i) // p) * a ** i * b ** (p - i)) % p
        want = {e: c for e, c in want.items() if c}
        assert literal.delta1({I: a, J: b}, p) == want
        g = np.array(literal.poly_to_dense({I: a, J: b}, 3), dtype=np.uint8)
        got = literal.poly_from_dense(fast.delta1(g, p, 3), 3 * p)
        assert got == want


@pytest.mark.parametrize("p", [3, 5, 7])
def test_monomial_has_zero_delta1(p):
    assert literal.delta1({(1, 2, 0, 1): 2}, p) == {}


@pytest.mark.parametrize("p,d,nterms", [(3, 4, 6), (3, 8, 10), (5, 4, 5), (5, 6, 4), (7, 4, 3)])
def test_delta1_equals_witt_vector_definition(p, d, nterms):
    rng = np.random.default_rng(100 * p + d)
    for _ in range(3):
        f = _rand_terms(rng, p, d, nterms)
        assert literal.delta1(f, p) == literal.delta1_witt(f, p)


@pytest.mark.parametrize("p", [3, 5])
def test_delta1_independent_of_lift(p):
    rng = np.random.default_rng(7 + p)
    for _ in range(3):
        f = _rand_terms(rng, p, 4, 6)
        other = {e: c + p * int(rng.integers(-3, 4)) for e, c in f.items()}
        assert literal.delta1_integer_lift(other, p) == literal.delta1(f, p)


@pytest.mark.parametrize("p", [3, 5, 7])
def test_delta1_degree(p):
    # Section 3.1, remark: Delta_1 of a form of degree d has degree p*d.
    rng = np.random.default_rng(p)
    f = _rand_terms(rng, p, 4, 8)
    D = literal.delta1(f, p)
    assert D and all(sum(e) == 4 * p for e in D)


@pytest.mark.parametrize("p,d,seeds", [(3, 8, range(4)), (5, 4, range(4)), (5, 8, range(2)), (7, 4, range(2))])
def test_c_tier_equals_integer_tier(p, d, seeds):
    ell = comb(d + 3, 3)
    for s in seeds:
        g = workloads.random_dense(p, ell, seed=1000 * p + 10 * d + s)
        want = literal.delta1(literal.poly_from_dense(g, d), p)
        got = literal.poly_from_dense(fast.delta1(g, p, d), p * d)
        assert got == want


def test_c_tier_equals_integer_tier_on_real_p3_shape():
    # g = f^2 for quartics over F_3: Delta_1(g) has 2,925 coefficients.
    F = workloads.bernoulli_support(3, 4, 0.7, seed=3)
    for f in F:
        g = fast.fpow(f, 3, 2)
        want = literal.delta1(literal.poly_from_dense(g, 8), 3)
        got = literal.poly_from_dense(fast.delta1(g, 3, 8), 24)
        assert got == want


@pytest.mark.slow
def test_c_tier_equals_integer_tier_on_real_p5_shape():
    # g = f^4 for a quartic over F_5 (969 terms); the Z computation takes ~10 s.
    F, _ = workloads.config_p5_single(0)
    g = fast.fpow(F[0], 5, 4)
    want = literal.delta1(literal.poly_from_dense(g, 16), 5)
    got = literal.poly_from_dense(fast.delta1(g, 5, 16), 80)
    assert got == want


@pytest.mark.parametrize("p,J,nterms", [(3, 1, 8), (5, 1, 6), (5, 2, 6), (7, 3, 4), (7, 1, 3)])
def test_delta1_of_g_from_chain_of_f_powers(p, J, nterms):
    # g = f^(p-1) mod p has the lift g~ = f~^(p-1) + p h, and (g~ + p h)^p = g~^p
    # mod p^2, so g~^p = m^(p(p-1)/J) mod p^2 for m = f~^J mod p^2 and any J
    # dividing p(p-1).  Delta_1(g) from that chain (the one the deep kernels
    # run) must equal Algorithm 1 applied to g.
    rng = np.random.default_rng(1000 * p + J)
    for _ in range(2):
        f = _rand_terms(rng, p, 4, nterms)
        ft = literal.lift(f, p)
        g = literal.poly_mod(literal.poly_pow(ft, p - 1), p)
        m = literal.poly_mod(literal.poly_pow(ft, J), p * p)
        A = m
        for _ in range(p * (p - 1) // J - 1):
            A = literal.poly_mod(literal.poly_mul(A, m), p * p)
        D = dict(A)
        for e, c in g.items():
            pe = tuple(p * x for x in e)
            D[pe] = (D.get(pe, 0) - c ** p) % (p * p)
        assert all(c % p == 0 for c in D.values())
        got = {e: (c // p) % p for e, c in D.items() if (c // p) % p}
        assert got == literal.delta1(g, p)
