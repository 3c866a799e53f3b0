"""Literal CPU oracle over Z with Python integers -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The product path (the HIP library and its
binding) never imports, calls or links anything under ``oracle/``.

This tier follows the paper's algorithms step by step, with polynomials held
as ``{exponent tuple: int}`` dictionaries and every integer exact:

* ``monomial_basis``   -- B_d, the monomial basis of S_d listed in
  lexicographic order (Section 4, definition of B_ell and Lemma "wics size").
  The paper does not fix the direction; the reading taken is *descending*
  lex with x1 > x2 > x3 > x4, which is the order its tables print terms in
  (Section 7, Figures 4-7).
* ``delta1``           -- Algorithm 1 (Section 3.1, Proposition "delta1
  formula"): lift to Z with coefficients in [0, p), raise to the p-th power
  over Z, subtract the p-th power of every term, divide by p, reduce mod p.
* ``delta1_witt``      -- the same quantity from its definition in W_2
  (Section 3.1, Definition of Delta_1; Section 2.1, Remark on W_2 addition),
  adding the Teichmueller lifts of the terms one at a time.  Used only to pin
  ``delta1``.
* ``frobenius_split``  -- Algorithm 2 (Section 3.2): keep the terms whose
  exponents are all = p-1 mod p, subtract p-1 and divide the exponents by p;
  over F_p the p-th root of a coefficient is the coefficient itself.
* ``height``           -- Algorithm 3 (Section 3.3) with bound b.
* ``triv_matrix``      -- Algorithm 5 (Section 4.1), the matrix of
  "multiply then split"; ``theta_matched`` computes the same map through the
  unique-match property (Section 4.2, Lemma "tuples mod p" and Corollary
  "unique match").

Everything is exact; nothing here has a tolerance.
"""

from collections import defaultdict

INF = 0  # height value used for "infinite" (the boundary's convention)


# --------------------------------------------------------------------------
# Monomial bases (Section 4: weak integer compositions and B_ell)
# --------------------------------------------------------------------------

def weak_compositions(k, n):
    """wics(k, n): all ordered n-tuples of non-negative integers summing to k."""
    if n == 1:
        yield (k,)
        return
    for first in range(k + 1):
        for rest in weak_compositions(k - first, n - 1):
            yield (first,) + rest


def monomial_basis(d, n=4):
    """B_d as a list of exponent tuples in descending lexicographic order."""
    return sorted(weak_compositions(d, n), reverse=True)


def basis_index(d, n=4):
    """indexof() for B_d: exponent tuple -> position (a plain dictionary)."""
    return {e: i for i, e in enumerate(monomial_basis(d, n))}


# --------------------------------------------------------------------------
# Polynomials as {exponent: coefficient}
# --------------------------------------------------------------------------

def _add_exp(a, b):
    return tuple(x + y for x, y in zip(a, b))


def poly_mul(a, b):
    """Product over Z (schoolbook: every pair of terms)."""
    out = defaultdict(int)
    for ea, ca in a.items():
        for eb, cb in b.items():
            out[_add_exp(ea, eb)] += ca * cb
    return {e: c for e, c in out.items() if c != 0}


def poly_pow(a, k, n=4):
    """a**k over Z by repeated multiplication (a**0 = 1)."""
    out = {(0,) * n: 1}
    for _ in range(k):
        out = poly_mul(out, a)
    return out


def poly_mod(a, m):
    """Reduce every coefficient into [0, m) and drop zeros."""
    out = {}
    for e, c in a.items():
        r = c % m
        if r:
            out[e] = r
    return out


def poly_from_dense(coeffs, d, n=4):
    """Dense coefficient list in B_d order -> dict (zeros dropped)."""
    basis = monomial_basis(d, n)
    if len(coeffs) != len(basis):
        raise ValueError("expected %d coefficients, got %d" % (len(basis), len(coeffs)))
    return {e: int(c) for e, c in zip(basis, coeffs) if int(c) != 0}


def poly_to_dense(a, d, n=4):
    """dict -> dense coefficient list in B_d order (terms must have degree d)."""
    idx = basis_index(d, n)
    out = [0] * len(idx)
    for e, c in a.items():
        out[idx[e]] = c
    return out


def lift(f, p):
    """Integer lift with coefficients in [0, p) (Section 3.1, Remark on lifts)."""
    return poly_mod(f, p)


# --------------------------------------------------------------------------
# Delta_1 (Section 3.1)
# --------------------------------------------------------------------------

def delta1(f, p):
    """Algorithm 1: Delta_1(f) = (f~^p - sum_t t^p) / p mod p, computed over Z.

    f is a dict with coefficients read mod p.  Raises ArithmeticError if some
    coefficient of f~^p - sum_t t^p is not divisible by p (it always is).
    """
    ft = lift(f, p)
    D = dict(poly_pow(ft, p, len(next(iter(ft))) if ft else 4))
    for e, c in ft.items():
        pe = tuple(p * x for x in e)
        D[pe] = D.get(pe, 0) - c ** p
    out = {}
    for e, c in D.items():
        if c % p:
            raise ArithmeticError("coefficient at %r not divisible by p" % (e,))
        r = (c // p) % p
        if r:
            out[e] = r
    return out


def delta1_integer_lift(ft, p):
    """Algorithm 1 on a caller-chosen integer lift ft (any integer coefficients).

    Used to check that the result does not depend on the lift chosen.
    """
    D = dict(poly_pow(ft, p, len(next(iter(ft))) if ft else 4))
    for e, c in ft.items():
        pe = tuple(p * x for x in e)
        D[pe] = D.get(pe, 0) - c ** p
    out = {}
    for e, c in D.items():
        if c % p:
            raise ArithmeticError("coefficient at %r not divisible by p" % (e,))
        r = (c // p) % p
        if r:
            out[e] = r
    return out


def delta1_witt(f, p):
    """Delta_1 from its definition in W_2(S): (0, Delta_1(f)) = (f,0) - sum_I (a_I x^I, 0).

    W_2 addition of (X0, X1) and (Y0, Y1) has ghost components X0^p + p X1 and
    Y0^p + p Y1; matching them gives the second Witt component
    X1 + Y1 + (X0^p + Y0^p - (X0 + Y0)^p) / p.  Adding the Teichmueller lifts
    (t, 0) of the terms t of f one at a time yields (f, s1); subtracting this
    from (f, 0) leaves (0, -s1).  Computed with integer lifts in [0, p).
    """
    terms = sorted(lift(f, p).items(), reverse=True)
    n = len(terms[0][0]) if terms else 4
    s0 = {}
    s1 = {}
    for e, c in terms:
        t = {e: c}
        carry = poly_pow(s0, p, n) if s0 else {}
        # X0^p + Y0^p - (X0 + Y0)^p, divided exactly by p
        tp = {tuple(p * x for x in e): c ** p}
        new_s0 = dict(s0)
        new_s0[e] = new_s0.get(e, 0) + c
        num = defaultdict(int)
        for k, v in carry.items():
            num[k] += v
        for k, v in tp.items():
            num[k] += v
        for k, v in poly_pow(new_s0, p, n).items():
            num[k] -= v
        for k, v in num.items():
            if v % p:
                raise ArithmeticError("Witt carry not divisible by p")
            s1[k] = s1.get(k, 0) + v // p
        s0 = new_s0
    return poly_mod({e: -c for e, c in s1.items()}, p)


# --------------------------------------------------------------------------
# The splitting u (Section 3.2) and the height (Section 3.3)
# --------------------------------------------------------------------------

def frobenius_split(h, p):
    """Algorithm 2: u(h), with the identification S^p = S (p-th roots of exponents)."""
    out = {}
    for e, c in h.items():
        if all(x % p == p - 1 for x in e):
            r = tuple((x - (p - 1)) // p for x in e)
            out[r] = out.get(r, 0) + c
    return out


def in_frobenius_power(g, p):
    """True iff g lies in m^[p] = (x1^p, ..., xn^p), i.e. every nonzero term has some exponent >= p."""
    return all(any(x >= p for x in e) for e, c in g.items() if c % p)


def theta_literal(delta, a, p):
    """u(Delta * a) mod p with the full product formed first (Algorithm 3's loop body)."""
    return poly_mod(frobenius_split(poly_mul(delta, a), p), p)


def theta_matched(delta, a, p):
    """u(Delta * a) mod p summing only the pairs of terms that match.

    A pair (delta_term, a_term) survives u only if their exponents add to
    (p-1,...,p-1) mod p (Section 4, definition of "matches"); the residue class
    of the matching delta_term is determined by the a_term (Corollary "unique
    match").  Delta is bucketed by exponent class mod p.
    """
    buckets = defaultdict(list)
    for e, c in delta.items():
        buckets[tuple(x % p for x in e)].append((e, c))
    out = defaultdict(int)
    for ea, ca in a.items():
        want = tuple(p - 1 - (x % p) for x in ea)
        for ed, cd in buckets.get(want, ()):
            r = tuple((x + y - (p - 1)) // p for x, y in zip(ed, ea))
            out[r] += cd * ca
    return poly_mod(out, p)


def height(f, p, bound=10, theta=theta_matched):
    """Algorithm 3: the quasi-F-split height of a Calabi-Yau hypersurface f.

    Returns 1..bound, or INF (=0) when no h <= bound is found (Theorem C with
    the K3 bound h <= 10 or h = infinity).
    """
    g = poly_mod(poly_pow(poly_mod(f, p), p - 1), p)
    if not in_frobenius_power(g, p):
        return 1
    Delta = delta1(g, p)
    h = 2
    while True:
        if bound < h:
            return INF
        g = theta(Delta, g, p)
        if not in_frobenius_power(g, p):
            return h
        h += 1


# --------------------------------------------------------------------------
# Matrix of "multiply then split" (Section 4.1, Algorithm 5 TRIV)
# --------------------------------------------------------------------------

def triv_matrix(delta, p, d, n=4):
    """Algorithm 5: M with M[row, col] = coeff(delta_term) for every matching pair.

    d is the degree of the source space; the target degree is
    d' = (d + D - n(p-1)) / p where D = deg Delta.
    Returns (M as a dict {(row, col): value}, B_d, B_d').
    """
    if not delta:
        raise ValueError("empty Delta")
    D = sum(next(iter(delta)))
    num = d + D - n * (p - 1)
    if num % p:
        raise ValueError("target degree is not an integer")
    dprime = num // p
    Bd = monomial_basis(d, n)
    Bdp_index = basis_index(dprime, n)
    col_index = {m: i for i, m in enumerate(Bd)}
    M = {}
    for m in Bd:
        for ed, cd in delta.items():
            if all((x + y) % p == p - 1 for x, y in zip(ed, m)):
                res = tuple((x + y - (p - 1)) // p for x, y in zip(ed, m))
                M[(Bdp_index[res], col_index[m])] = cd
    return M, Bd, monomial_basis(dprime, n)


def matching_monomials(delta_exp, p, d, n=4):
    """Lemma "generate matching": the exponents in B_d that match delta_exp, by brute force over B_d."""
    return [m for m in monomial_basis(d, n)
            if all((x + y) % p == p - 1 for x, y in zip(delta_exp, m))]


# --------------------------------------------------------------------------
# Brute-force point count (used only to pin the height-1 test)
# --------------------------------------------------------------------------

def affine_zero_count(f, p):
    """#{x in F_p^n : f(x) = 0} by evaluating f at every point."""
    import itertools
    terms = list(f.items())
    n = len(terms[0][0]) if terms else 4
    count = 0
    for x in itertools.product(range(p), repeat=n):
        v = 0
        for e, c in terms:
            t = c
            for xi, ei in zip(x, e):
                t *= xi ** ei
            v += t
        if v % p == 0:
            count += 1
    return count
