"""ctypes binding of the plain C oracle (qfs_oracle.c) -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this module.  Arrays are numpy uint8 in B_d order (descending lex).
ctypes releases the GIL during each call, so a thread pool runs surfaces in
parallel.
"""
import ctypes
import os

import numpy as np

from . import build as _build

INF = 0
_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.oracle_num_monomials.argtypes = [ctypes.c_int]
        L.oracle_num_monomials.restype = ctypes.c_int64
        L.oracle_basis.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]
        L.oracle_fpow.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p]
        L.oracle_delta1.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p]
        L.oracle_theta.argtypes = [ctypes.c_int, u8p, u8p, u8p]
        L.oracle_height.argtypes = [ctypes.c_int, u8p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        for fn in (L.oracle_basis, L.oracle_fpow, L.oracle_delta1, L.oracle_theta, L.oracle_height):
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _check(rc, what):
    if rc < 0:
        raise RuntimeError("%s failed with code %d" % (what, rc))
    return rc


def num_monomials(d):
    return int(lib().oracle_num_monomials(d))


def basis(d):
    n = num_monomials(d)
    ex = np.zeros((n, 4), dtype=np.int32)
    _check(lib().oracle_basis(d, ex.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "basis")
    return ex


def fpow(f, p, k):
    """f^k mod p; f has 35 coefficients in B_4 order."""
    f, fp = _u8(f)
    out = np.zeros(num_monomials(4 * k), dtype=np.uint8)
    _check(lib().oracle_fpow(p, k, fp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "fpow")
    return out


def delta1(g, p, d):
    """Delta_1(g) for g of degree d in B_d order; result in B_{pd} order."""
    g, gp = _u8(g)
    out = np.zeros(num_monomials(p * d), dtype=np.uint8)
    _check(lib().oracle_delta1(p, d, gp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "delta1")
    return out


def theta(delta, a, p):
    """u(Delta * a) mod p for a of degree 4(p-1)."""
    delta, dp = _u8(delta)
    a, ap = _u8(a)
    out = np.zeros(a.shape[0], dtype=np.uint8)
    _check(lib().oracle_theta(p, dp, ap, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "theta")
    return out


def theta_pow(delta, a, p, iters):
    for _ in range(iters):
        a = theta(delta, a, p)
    return a


def height(f, p, bound=10, with_iters=False):
    f, fp = _u8(f)
    it = ctypes.c_int(0)
    h = _check(lib().oracle_height(p, fp, bound, ctypes.byref(it)), "height")
    return (h, it.value) if with_iters else h


def heights(F, P, bound=10, threads=None):
    """Heights of a batch (rows of F, primes P) on a thread pool."""
    from concurrent.futures import ThreadPoolExecutor
    F = np.ascontiguousarray(F, dtype=np.uint8)
    P = np.asarray(P).reshape(-1)
    if P.size == 1:
        P = np.full(F.shape[0], int(P[0]))
    threads = threads or os.cpu_count() or 1
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda i: height(F[i], int(P[i]), bound), range(F.shape[0])))
    return np.array(res, dtype=np.int32)
