"""Seeded synthetic quartics for tests and benchmarks.

This module only draws inputs: it holds none of the height algorithm's
arithmetic, and both the HIP path's tests and the CPU oracle read their inputs
from here.  Every generator uses numpy's PCG64 (``np.random.default_rng``)
with an explicit seed.

A quartic over F_p is 35 uint8 coefficients in B_4 order: the monomials
x1^e1 x2^e2 x3^e3 x4^e4 of degree 4 in descending lexicographic order of
(e1, e2, e3, e4).  The paper draws surfaces as uniform points of F_p^35
(Section 7.1); the workloads below follow the shapes and value distributions of
the five benchmark configurations.
"""
import numpy as np

PRIMES = (3, 5, 7, 11)


def b4_exponents():
    """The 35 exponent tuples of degree 4, in the coefficient order used everywhere."""
    out = []
    for e1 in range(4, -1, -1):
        for e2 in range(4 - e1, -1, -1):
            for e3 in range(4 - e1 - e2, -1, -1):
                out.append((e1, e2, e3, 4 - e1 - e2 - e3))
    return out


B4 = b4_exponents()
DIAG = [B4.index(e) for e in ((4, 0, 0, 0), (0, 4, 0, 0), (0, 0, 4, 0), (0, 0, 0, 4))]
OFF_DIAG = [i for i in range(35) if i not in DIAG]


def fermat():
    """x1^4 + x2^4 + x3^4 + x4^4."""
    f = np.zeros(35, dtype=np.uint8)
    f[DIAG] = 1
    return f


def uniform(p, n, seed, low=0):
    """n quartics with every coefficient uniform in {low..p-1}."""
    rng = np.random.default_rng(seed)
    return rng.integers(low, p, size=(n, 35), dtype=np.int64).astype(np.uint8)


def bernoulli_support(p, n, density, seed):
    """Coefficients kept with probability `density` (scalar or per-row array), kept values uniform in {1..p-1}."""
    rng = np.random.default_rng(seed)
    dens = np.broadcast_to(np.asarray(density, dtype=np.float64).reshape(-1, 1), (n, 1))
    keep = rng.random((n, 35)) < dens
    vals = rng.integers(1, p, size=(n, 35), dtype=np.int64)
    return np.where(keep, vals, 0).astype(np.uint8)


def config_p5_single(seed=0):
    """One quartic over F_5 with coefficients uniform in {0..4}, plus the Fermat quartic."""
    f = uniform(5, 1, seed)[0]
    return np.stack([f, fermat()]), np.array([5, 5], dtype=np.int32)


def config_p7_single(seed=0, n=16):
    """Quartics over F_7, one per seed seed..seed+n-1: support Bernoulli(0.5), kept values uniform {1..6}."""
    F = np.concatenate([bernoulli_support(7, 1, 0.5, seed + s) for s in range(n)])
    return F, np.full(n, 7, dtype=np.int32)


def config_p5_batch(n=8192, seed=0):
    """p=5 batch: density cycles through 0.1, 0.3, 0.6, 1.0 by row; kept values uniform {1..4}."""
    dens = np.array([0.1, 0.3, 0.6, 1.0])[np.arange(n) % 4]
    return bernoulli_support(5, n, dens, seed), np.full(n, 5, dtype=np.int32)


def config_p7_batch(n=65536, seed=0):
    """p=7 batch of uneven structure.

    Half are diagonal a x1^4 + b x2^4 + c x3^4 + d x4^4 (a..d uniform {1..6})
    plus k ~ U{1..8} cross terms chosen without replacement from the other 31
    monomials with values uniform {1..6}; half are dense with all 35
    coefficients uniform {1..6}.  Rows are shuffled by a seeded permutation.
    """
    rng = np.random.default_rng(seed)
    half = n // 2
    F = np.zeros((n, 35), dtype=np.uint8)
    F[:half, DIAG] = rng.integers(1, 7, size=(half, 4))
    ks = rng.integers(1, 9, size=half)
    off = np.array(OFF_DIAG)
    for i in range(half):
        cols = rng.choice(off, size=ks[i], replace=False)
        F[i, cols] = rng.integers(1, 7, size=ks[i])
    F[half:] = rng.integers(1, 7, size=(n - half, 35))
    perm = rng.permutation(n)
    return F[perm], np.full(n, 7, dtype=np.int32)


def config_mixed(n=4096, seed=0):
    """Mixed primes: p uniform over {3,5,7,11}, density uniform [0.1,1], kept values uniform {1..p-1}."""
    rng = np.random.default_rng(seed)
    P = rng.choice(np.array(PRIMES), size=n).astype(np.int32)
    dens = rng.uniform(0.1, 1.0, size=n)
    keep = rng.random((n, 35)) < dens[:, None]
    u = rng.random((n, 35))
    vals = 1 + np.floor(u * (P[:, None] - 1)).astype(np.int64)
    return np.where(keep, vals, 0).astype(np.uint8), P


def random_poly(p, nterms, ell, seed):
    """A random coefficient vector of length ell with about nterms nonzero entries in {1..p-1}."""
    rng = np.random.default_rng(seed)
    v = np.zeros(ell, dtype=np.uint8)
    idx = rng.choice(ell, size=min(nterms, ell), replace=False)
    v[idx] = rng.integers(1, p, size=idx.size)
    return v


def random_dense(p, ell, seed):
    """A coefficient vector of length ell uniform in {0..p-1}."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, p, size=ell, dtype=np.int64).astype(np.uint8)


CONFIGS = {
    "p5_single": config_p5_single,
    "p7_single": config_p7_single,
    "p5_batch8192": config_p5_batch,
    "p7_batch65536": config_p7_batch,
    "mixed4096": config_mixed,
}
