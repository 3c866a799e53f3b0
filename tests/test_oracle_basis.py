"""Pins for the monomial bases B_d used by both oracle tiers (Section 4)."""
import itertools
from math import comb

import numpy as np

from oracle import fast, literal


def test_basis_sizes_match_paper_matrix_sizes():
    # Section 6 lists the square matrix sizes binom(4p-1, 3) for p = 3, 5, 7, 11, 13.
    printed = {3: 165, 5: 969, 7: 2925, 11: 12341, 13: 20825}
    for p, size in printed.items():
        d = 4 * (p - 1)
        assert fast.num_monomials(d) == size
        if p <= 7:
            assert len(literal.monomial_basis(d)) == size


def test_wics_example():
    # Section 4, example after the definition of wics: wics(2, 3).
    printed = {(2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1), (0, 1, 1)}
    got = list(literal.weak_compositions(2, 3))
    assert len(got) == len(set(got)) == 6
    assert set(got) == printed


def test_wics_size_by_brute_force():
    # Lemma "wics size": |wics(k, n)| = binom(k+n-1, n-1); brute force over a box.
    for n in (1, 2, 3, 4):
        for k in range(0, 9):
            brute = sum(1 for t in itertools.product(range(k + 1), repeat=n) if sum(t) == k)
            assert brute == len(list(literal.weak_compositions(k, n))) == comb(k + n - 1, n - 1)


def test_c_basis_order_matches_sorted_tuples():
    for d in list(range(0, 13)) + [16, 24]:
        c = [tuple(int(x) for x in row) for row in fast.basis(d)]
        py = literal.monomial_basis(d)
        assert c == py
        assert c[0] == (d, 0, 0, 0) and c[-1] == (0, 0, 0, d)
        # strictly descending lexicographic
        assert all(a > b for a, b in zip(c, c[1:]))


def test_only_monomial_outside_frobenius_power():
    # Section 3.4: in degree n(p-1) the only monomial not in m^[p] is (x1...xn)^(p-1).
    for p in (3, 5, 7):
        B = fast.basis(4 * (p - 1))
        outside = [tuple(r) for r in B if np.all(r < p)]
        assert outside == [(p - 1,) * 4]
