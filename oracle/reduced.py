"""Reduced height oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.

Not an algorithm of the paper but a consequence of its formulas, derived in
``oracle/REDUCED.md``: with H = f^(p-2) mod p and D = Delta_1(f) (Algorithm 1
applied to f itself),

  * Delta_1(f^(p-1)) = phi(Q) - D phi(H) mod p, phi(P)(x) = P(x^p), for a form Q
    of degree 4(p-1) (Section 3.1, Proposition on the Delta_1 formula, and the
    binomial theorem mod p^2);
  * theta(a) = u(Delta_1(g) a) = c(a) Q - H u(D a) for a of degree 4(p-1)
    (Algorithm 2: u is p^-1-linear, and u(a) = c(a) is the coefficient of
    x^e, e = (p-1, ..., p-1));
  * along Algorithm 3's loop c(theta^(k-1)(g)) = 0 until the height is found,
    so theta^(k-1)(g) = H v_k for quartics v_1 = f, v_(k+1) = -u(D H v_k), and
    c(theta^(k-1)(g)) = <hvec, v_k> with hvec[r] = H[e - r].

So h = the least k <= bound with <hvec, N^(k-1) f> != 0 mod p, where N is the
35 x 35 matrix N[r', r] = (D H)[p r' + e - r] (the sign of N does not change
which terms vanish), else infinity (0).  Polynomials are ``{exponent tuple:
int}`` dictionaries (``oracle.literal``); every step is exact.
"""

import numpy as np

from . import literal

INF = 0


def reduced_parts(f, p):
    """H = f^(p-2) mod p and D = Delta_1(f) (dicts), for f a dict over F_p.

    D is Algorithm 1 on f; f~^p is formed mod p^2, which is exact for D mod p
    (the quotient (f~^p - sum a^p x^(pI)) / p mod p only needs f~^p mod p^2)."""
    F = literal.lift(f, p)
    H = literal.poly_mod(literal.poly_pow(F, p - 2), p)
    Fp = {(0, 0, 0, 0): 1}
    for _ in range(p):
        Fp = literal.poly_mod(literal.poly_mul(Fp, F), p * p)
    for e, a in F.items():
        pe = tuple(p * x for x in e)
        Fp[pe] = (Fp.get(pe, 0) - a ** p) % (p * p)
    D = {}
    for e, c in Fp.items():
        if c % p:
            raise ArithmeticError("coefficient at %r not divisible by p" % (e,))
        if (c // p) % p:
            D[e] = (c // p) % p
    return H, D


def reduced_matrix(f, p):
    """(N, hvec): N[i][j] = (D H)[p r'_i + e - r_j] mod p and hvec[j] = H[e - r_j] mod p,
    over the quartic basis r_0..r_34 (descending lex).  Each entry is the sum over
    the terms s of H of H[s] D[x - s] (x - s >= 0 in every exponent)."""
    H, D = reduced_parts(f, p)
    B4 = literal.monomial_basis(4)
    e = (p - 1,) * 4
    hvec = []
    for r in B4:
        s = tuple(a - b for a, b in zip(e, r))
        hvec.append(H.get(s, 0) % p if min(s) >= 0 else 0)
    hs = np.array(list(H.keys()), dtype=np.int64).reshape(-1, 4)
    hv = np.array(list(H.values()), dtype=np.int64)
    dmap = {t: v for t, v in D.items()}
    N = []
    for r2 in B4:
        row = []
        for r in B4:
            x = np.array([p * a + (p - 1) - b for a, b in zip(r2, r)], dtype=np.int64)
            T = x[None, :] - hs
            ok = (T >= 0).all(axis=1)
            acc = 0
            for t, c in zip(map(tuple, T[ok].tolist()), hv[ok].tolist()):
                acc += c * dmap.get(t, 0)
            row.append(acc % p)
        N.append(row)
    return N, hvec


def height(f, p, bound=10):
    """Height from the reduced form: least k <= bound with <hvec, N^(k-1) f> != 0, else INF."""
    f = literal.poly_mod(f, p)
    N, hvec = reduced_matrix(f, p)
    B4 = literal.monomial_basis(4)
    v = [f.get(r, 0) % p for r in B4]
    for k in range(1, bound + 1):
        if sum(a * b for a, b in zip(hvec, v)) % p:
            return k
        v = [sum(N[i][j] * v[j] for j in range(35)) % p for i in range(35)]
    return INF


def delta1_of_g_reduced(f, p):
    """Delta_1(f^(p-1)) as phi(Q) - D phi(H) mod p, with Q = (F_s^(p-1) - sum_J b_J^p x^J) / p,
    F_s = sum_I a_I^p x^I and b_J the coefficients of g = f^(p-1) mod p (a dict)."""
    F = literal.lift(f, p)
    H, D = reduced_parts(f, p)
    Fs = {e: a ** p for e, a in F.items()}
    G = literal.poly_pow(Fs, p - 1)
    g = literal.poly_mod(literal.poly_pow(F, p - 1), p)
    for e, b in g.items():
        G[e] = G.get(e, 0) - b ** p
    Q = {}
    for e, c in G.items():
        if c % p:
            raise ArithmeticError("F_s^(p-1) - sum b^p x^J not divisible by p at %r" % (e,))
        Q[e] = (c // p) % p
    out = {}
    for e, c in Q.items():
        pe = tuple(p * x for x in e)
        out[pe] = (out.get(pe, 0) + c) % p
    for t, dv in D.items():
        for s, hv in H.items():
            x = tuple(a + p * b for a, b in zip(t, s))
            out[x] = (out.get(x, 0) - dv * hv) % p
    return {e: c for e, c in out.items() if c}
