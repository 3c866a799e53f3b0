"""Python binding of libqfs, the MI355X (gfx950) library for quasi-F-split
heights of quartic K3 surfaces (arXiv 2502.12428).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libqfs.so`` (built by ``paper_2502_12428_amd.build``).  PyTorch
provides device memory and the current stream.  The functions mirror the C
ABI in ``include/qfs.h``:

* ``delta1(f, p)``            -> (g, delta, status)    Algorithm 1 on g = f^(p-1)
* ``theta(delta, a, p, iters)`` -> theta^iters(a)       Section 3.4
* ``height(f, p, bound=10)``  -> int32 heights          Algorithm 3, batched
* ``height_plain(f, p, bound=10)`` -> heights           the per-surface baseline

Heights: 1..bound, 0 for infinity, negative for a per-surface error code.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqfs.so")

QFS_OK = 0
QFS_EINVAL = -1
QFS_ENOMEM = -2
QFS_EDEVICE = -3
QFS_EUNSUPPORTED = -4
QFS_EARITH = -5
HEIGHT_INF = 0
PRIMES = (3, 5, 7, 11)

EXPORTS = (
    "qfs_num_monomials", "qfs_monomial_rank", "qfs_monomial_unrank", "qfs_len_g", "qfs_len_delta",
    "qfs_delta1_workspace_bytes", "qfs_delta1", "qfs_theta_workspace_bytes", "qfs_theta",
    "qfs_height_workspace_bytes", "qfs_height", "qfs_height_plain_workspace_bytes", "qfs_height_plain",
    "qfs_height_reduced_workspace_bytes", "qfs_height_reduced", "qfs_mfma_peak",
    "qfs_profile_enable", "qfs_profile_collect", "qfs_mfma_per_surface", "qfs_set_option", "qfs_get_option",
    "qfs_autotune", "qfs_load_tuning", "qfs_last_error", "qfs_shutdown",
)


class QfsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libqfs error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load libqfs.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqfs.so is not built (%s); run python -c 'import __graft_entry__ as g; g.build()'"
                          % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, sz, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
    L.qfs_num_monomials.argtypes, L.qfs_num_monomials.restype = [i32], i64
    L.qfs_monomial_rank.argtypes, L.qfs_monomial_rank.restype = [vp], i64
    L.qfs_monomial_unrank.argtypes, L.qfs_monomial_unrank.restype = [i32, i64, vp], i32
    L.qfs_len_g.argtypes, L.qfs_len_g.restype = [i32], i64
    L.qfs_len_delta.argtypes, L.qfs_len_delta.restype = [i32], i64
    L.qfs_delta1_workspace_bytes.argtypes, L.qfs_delta1_workspace_bytes.restype = [i32, i32], sz
    L.qfs_delta1.argtypes, L.qfs_delta1.restype = [i32, i32, vp, vp, vp, vp, vp, sz, vp], i32
    L.qfs_theta_workspace_bytes.argtypes, L.qfs_theta_workspace_bytes.restype = [i32, i32], sz
    L.qfs_theta.argtypes, L.qfs_theta.restype = [i32, i32, vp, vp, vp, i32, vp, sz, vp], i32
    L.qfs_height_workspace_bytes.argtypes, L.qfs_height_workspace_bytes.restype = [i32, i32], sz
    L.qfs_height.argtypes, L.qfs_height.restype = [i32, vp, vp, i32, i32, vp, vp, sz, vp], i32
    L.qfs_height_plain_workspace_bytes.argtypes, L.qfs_height_plain_workspace_bytes.restype = [i32], sz
    L.qfs_height_plain.argtypes, L.qfs_height_plain.restype = [i32, i32, vp, i32, vp, vp, sz, vp], i32
    L.qfs_height_reduced_workspace_bytes.argtypes, L.qfs_height_reduced_workspace_bytes.restype = [i32, i32], sz
    L.qfs_height_reduced.argtypes, L.qfs_height_reduced.restype = [i32, vp, vp, i32, i32, vp, vp, sz, vp], i32
    L.qfs_mfma_peak.argtypes, L.qfs_mfma_peak.restype = [i32, vp, ctypes.POINTER(ctypes.c_double), vp], i32
    L.qfs_profile_enable.argtypes, L.qfs_profile_enable.restype = [i32], i32
    L.qfs_profile_collect.argtypes, L.qfs_profile_collect.restype = [vp, vp], i32
    L.qfs_mfma_per_surface.argtypes, L.qfs_mfma_per_surface.restype = [i32, i32], i64
    L.qfs_set_option.argtypes, L.qfs_set_option.restype = [ctypes.c_char_p, i64], i32
    L.qfs_get_option.argtypes, L.qfs_get_option.restype = [ctypes.c_char_p], i64
    L.qfs_autotune.argtypes, L.qfs_autotune.restype = [i32, vp, vp, i32, i32, vp, vp, sz, vp, ctypes.c_char_p, i32], i32
    L.qfs_load_tuning.argtypes, L.qfs_load_tuning.restype = [ctypes.c_char_p, i32], i32
    L.qfs_last_error.argtypes, L.qfs_last_error.restype = [], ctypes.c_char_p
    L.qfs_shutdown.argtypes, L.qfs_shutdown.restype = [], None
    _lib = L
    return L


def _check(rc):
    if rc != QFS_OK:
        raise QfsError(rc, lib().qfs_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _device_u8(x, name):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if x.dtype != torch.uint8:
        raise TypeError("%s must be uint8" % name)
    return x.contiguous()


class Workspace:
    """A reusable device scratch buffer (256-byte aligned)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes + 256 or self.buf.device != device:
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        addr = self.buf.data_ptr()
        off = (-addr) % 256
        return self.buf[off:off + nbytes]


_ws = Workspace()


# --------------------------------------------------------------------------- sizes / index
def num_monomials(deg):
    return int(lib().qfs_num_monomials(int(deg)))


def len_g(p):
    return int(lib().qfs_len_g(int(p)))


def len_delta(p):
    return int(lib().qfs_len_delta(int(p)))


def monomial_rank(e):
    arr = (ctypes.c_int32 * 4)(*[int(x) for x in e])
    return int(lib().qfs_monomial_rank(ctypes.cast(arr, ctypes.c_void_p)))


def monomial_unrank(deg, rank):
    arr = (ctypes.c_int32 * 4)()
    _check(lib().qfs_monomial_unrank(int(deg), int(rank), ctypes.cast(arr, ctypes.c_void_p)))
    return tuple(arr)


# --------------------------------------------------------------------------- entry points
def delta1(f, p, workspace=None):
    """(g, Delta_1(g), status) for every quartic row of f (uint8 [B,35] on the GPU)."""
    f = _device_u8(f, "f")
    B = f.shape[0]
    g = torch.empty((B, len_g(p)), dtype=torch.uint8, device=f.device)
    dl = torch.empty((B, len_delta(p)), dtype=torch.uint8, device=f.device)
    st = torch.empty(B, dtype=torch.int32, device=f.device)
    ws = (workspace or _ws).get(lib().qfs_delta1_workspace_bytes(int(p), B), f.device)
    _check(lib().qfs_delta1(int(p), B, _ptr(f), _ptr(g), _ptr(dl), _ptr(st), _ptr(ws), ws.numel(), _stream()))
    return g, dl, st


def theta(delta, a, p, iters=1, workspace=None):
    """theta^iters(a) for each row (Delta uint8 [B, len_delta], a uint8 [B, len_g])."""
    delta = _device_u8(delta, "delta")
    a = _device_u8(a, "a")
    B = a.shape[0]
    out = torch.empty_like(a)
    ws = (workspace or _ws).get(lib().qfs_theta_workspace_bytes(int(p), B), a.device)
    _check(lib().qfs_theta(int(p), B, _ptr(delta), _ptr(a), _ptr(out), int(iters), _ptr(ws), ws.numel(),
                           _stream()))
    return out


def height(f, p, bound=10, max_p=None, workspace=None, out=None):
    """Heights of the quartics in f (uint8 [B,35] on the GPU); p is an int or an int32 tensor [B].
    out: optional int32 [B] device tensor to write (repeated calls with the same tensors replay one graph)."""
    f = _device_u8(f, "f")
    B = f.shape[0]
    if isinstance(p, torch.Tensor):
        pt = p.to(device=f.device, dtype=torch.int32).contiguous()
        if max_p is None:
            max_p = int(pt.max().item()) if B else 3
            max_p = min([q for q in PRIMES if q >= max_p] or [11])
    else:
        pt = torch.full((B,), int(p), dtype=torch.int32, device=f.device)
        max_p = max_p or int(p)
    if out is None:
        h = torch.empty(B, dtype=torch.int32, device=f.device)
    else:
        if out.dtype != torch.int32 or out.device != f.device or out.numel() != B or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor of %d elements on %s" % (B, f.device))
        h = out
    ws = (workspace or _ws).get(lib().qfs_height_workspace_bytes(B, int(max_p)), f.device)
    _check(lib().qfs_height(B, _ptr(pt), _ptr(f), int(bound), int(max_p), _ptr(h), _ptr(ws), ws.numel(),
                            _stream()))
    return h


def height_reduced(f, p, bound=10, max_p=None, workspace=None, out=None):
    """Heights from the reduced form (qfs_height_reduced): the same values as height()."""
    f = _device_u8(f, "f")
    B = f.shape[0]
    if isinstance(p, torch.Tensor):
        pt = p.to(device=f.device, dtype=torch.int32).contiguous()
        if max_p is None:
            max_p = int(pt.max().item()) if B else 3
            max_p = min([q for q in PRIMES if q >= max_p] or [11])
    else:
        pt = torch.full((B,), int(p), dtype=torch.int32, device=f.device)
        max_p = max_p or int(p)
    if out is None:
        h = torch.empty(B, dtype=torch.int32, device=f.device)
    else:
        if out.dtype != torch.int32 or out.device != f.device or out.numel() != B or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor of %d elements on %s" % (B, f.device))
        h = out
    ws = (workspace or _ws).get(lib().qfs_height_reduced_workspace_bytes(B, int(max_p)), f.device)
    _check(lib().qfs_height_reduced(B, _ptr(pt), _ptr(f), int(bound), int(max_p), _ptr(h), _ptr(ws), ws.numel(),
                                    _stream()))
    return h


def mfma_peak(iters=20000):
    """Sustained int8 matrix-core rate of this device in TOP/s (qfs_mfma_peak)."""
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    tops = ctypes.c_double(0.0)
    _check(lib().qfs_mfma_peak(int(iters), _ptr(sink), ctypes.byref(tops), _stream()))
    return tops.value


def autotune(f, p, bound=10, max_p=None, workspace=None, cache_path=None, reps=2):
    """Time qfs_height on this batch over the launch-setting grid, keep the fastest setting
    (and append it to cache_path); returns the heights of the last trial."""
    f = _device_u8(f, "f")
    B = f.shape[0]
    pt = p.to(device=f.device, dtype=torch.int32).contiguous() if isinstance(p, torch.Tensor) else \
        torch.full((B,), int(p), dtype=torch.int32, device=f.device)
    max_p = int(max_p or (int(pt.max().item()) if B else 3))
    h = torch.empty(B, dtype=torch.int32, device=f.device)
    slots = get_option("deep_slots")
    set_option("deep_slots", 0)
    try:
        nbytes = lib().qfs_height_workspace_bytes(B, max_p)
    finally:
        set_option("deep_slots", slots)
    ws = (workspace or _ws).get(nbytes, f.device)
    path = cache_path.encode() if cache_path else None
    _check(lib().qfs_autotune(B, _ptr(pt), _ptr(f), int(bound), max_p, _ptr(h), _ptr(ws), ws.numel(), _stream(),
                              path, int(reps)))
    return h


def load_tuning(cache_path, max_p):
    """Apply the settings qfs_autotune stored for this device and max_p."""
    _check(lib().qfs_load_tuning(cache_path.encode(), int(max_p)))


def height_plain(f, p, bound=10, workspace=None):
    """Heights computed one surface at a time by the plain vector-ALU kernels (the baseline)."""
    f = _device_u8(f, "f")
    B = f.shape[0]
    h = torch.empty(B, dtype=torch.int32, device=f.device)
    ws = (workspace or _ws).get(lib().qfs_height_plain_workspace_bytes(int(p)), f.device)
    _check(lib().qfs_height_plain(int(p), B, _ptr(f), int(bound), _ptr(h), _ptr(ws), ws.numel(), _stream()))
    return h


# --------------------------------------------------------------------------- diagnostics
STAGES = ("stage1", "plan", "band_p3", "band_p5", "band_p7", "band_p11",
          "deep_p3", "deep_p5", "deep_p7", "deep_p11")


def profile(on):
    """Record hipEvents around the stages of every height() call while on."""
    _check(lib().qfs_profile_enable(1 if on else 0))


def profile_collect():
    """(summed milliseconds per stage, number of calls) since the last collect."""
    ms = (ctypes.c_double * len(STAGES))()
    calls = ctypes.c_int(0)
    _check(lib().qfs_profile_collect(ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(ctypes.pointer(calls), ctypes.c_void_p)))
    return dict(zip(STAGES, list(ms))), calls.value


def mfma_per_surface(p, band=False):
    """v_mfma_i32_16x16x64_i8 instructions the g~^p product issues per surface at prime p
    (band: the capped chain qfs_height runs first; otherwise the full chain)."""
    return int(lib().qfs_mfma_per_surface(int(p), 1 if band else 0))


def set_option(name, value):
    """Set a process-wide library option (see qfs_set_option in include/qfs.h)."""
    _check(lib().qfs_set_option(name.encode(), int(value)))


def get_option(name):
    v = int(lib().qfs_get_option(name.encode()))
    if v < 0:
        raise QfsError(v, lib().qfs_last_error().decode())
    return v
