"""Oracle for exact digital circular convolution modulo a prime m.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library neither imports nor links it, and it shares no code with the product.

It wraps ``oracle.c`` (plain C, exact 128-bit integer arithmetic, O(N^2)
definitions) through ctypes.  Paper: S. S. Chandra, "Fast Digital Convolutions
using Bit-Shifts" (arXiv:1005.1497).

Parity-pinned routines (see ``tests/test_oracle_pins.py``):
  is_prime, order, powers, inverse, ntt (forward Eq. 2 / inverse Eq. 3),
  ntt_bins, conv_direct (Eq. 1), conv_entries, conv_via_ntt (Sec. I).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            U64, INT = ctypes.c_uint64, ctypes.c_int
            lib.oracle_threads.restype = INT
            lib.oracle_set_threads.argtypes = [INT]
            lib.oracle_set_threads.restype = None
            lib.oracle_is_prime.argtypes = [U64]
            lib.oracle_is_prime.restype = INT
            lib.oracle_powers.argtypes = [U64, U64, U64, _u64p]
            lib.oracle_order.argtypes = [U64, U64, U64]
            lib.oracle_order.restype = U64
            lib.oracle_inverse.argtypes = [U64, U64]
            lib.oracle_inverse.restype = U64
            lib.oracle_ntt.argtypes = [_u64p, _u64p, U64, U64, U64, INT]
            lib.oracle_ntt.restype = INT
            lib.oracle_ntt_bins.argtypes = [_u64p, U64, U64, U64, _u64p, U64, _u64p]
            lib.oracle_ntt_bins.restype = INT
            lib.oracle_ntt_bins_rows.argtypes = [_u64p, U64, U64, U64, U64, _u64p, U64, _u64p]
            lib.oracle_ntt_bins_rows.restype = INT
            lib.oracle_ntt2d_bins.argtypes = [_u64p, U64, U64, U64, U64, U64, _u64p, _u64p, U64, _u64p]
            lib.oracle_ntt2d_bins.restype = INT
            lib.oracle_conv_direct.argtypes = [_u64p, _u64p, _u64p, U64, U64]
            lib.oracle_conv_entries.argtypes = [_u64p, _u64p, U64, U64, _u64p, U64, _u64p]
            lib.oracle_conv_via_ntt.argtypes = [_u64p, _u64p, _u64p, U64, U64, U64]
            lib.oracle_conv_via_ntt.restype = INT
            lib.oracle_deconv_via_ntt.argtypes = [_u64p, _u64p, _u64p, U64, U64, U64]
            lib.oracle_deconv_via_ntt.restype = INT
            lib.oracle_conv_integer.argtypes = [_u64p, _u64p, _u64p, U64]
            lib.oracle_conv_integer.restype = INT
            lib.oracle_conv_integer_entries.argtypes = [_u64p, _u64p, U64, _u64p, U64, _u64p]
            lib.oracle_conv_integer_entries.restype = INT
            lib.oracle_conv2d_direct.argtypes = [_u64p, _u64p, _u64p, U64, U64, U64]
            lib.oracle_conv2d_entries.argtypes = [_u64p, _u64p, U64, U64, U64, _u64p, U64, _u64p]
            _lib = lib
    return _lib


def _arr(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x).astype(np.uint64, copy=False))
    return a


def _p(a: np.ndarray):
    return a.ctypes.data_as(_u64p)


def threads() -> int:
    """Number of OpenMP threads the oracle's parallel loops use."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Number of OpenMP threads of the parallel loops from here on."""
    _load().oracle_set_threads(int(n))


def is_prime(m: int) -> bool:
    """Trial-division primality (Sec. III-A picks m prime)."""
    return bool(_load().oracle_is_prime(int(m)))


def powers(a: int, m: int, count: int) -> np.ndarray:
    """Digital circle of a mod m (Eq. 5, Fig. 1): [a^0, a^1, ..., a^(count-1)] mod m."""
    out = np.zeros(count, dtype=np.uint64)
    _load().oracle_powers(int(a), int(m), int(count), _p(out))
    return out


def order(a: int, m: int, limit: int | None = None) -> int:
    """Smallest nu >= 1 with a^nu = 1 mod m (Eq. 7); 0 if not found within limit."""
    if limit is None:
        limit = int(m)
    return int(_load().oracle_order(int(a), int(m), int(limit)))


def inverse(b: int, m: int) -> int:
    """b^-1 mod m by the extended Euclidean algorithm (Appendix A); 0 if none."""
    return int(_load().oracle_inverse(int(b), int(m)))


def ntt(x, m: int, root: int, inverse: bool = False) -> np.ndarray:
    """O(N^2) transform: Eq. 2 (forward) or Eq. 3 including N^-1 (inverse)."""
    a = _arr(x)
    out = np.zeros_like(a)
    rc = _load().oracle_ntt(_p(a), _p(out), a.size, int(m), int(root), 1 if inverse else 0)
    if rc:
        raise ValueError("oracle_ntt failed with code %d" % rc)
    return out


def ntt_bins(x, m: int, root: int, bins) -> np.ndarray:
    """Selected forward outputs X(u) of Eq. 2, each an O(N) sum."""
    a = _arr(x)
    b = _arr(bins)
    out = np.zeros(b.size, dtype=np.uint64)
    _load().oracle_ntt_bins(_p(a), a.size, int(m), int(root), _p(b), b.size, _p(out))
    return out


def ntt_bins_rows(x, m: int, root: int, bins) -> np.ndarray:
    """x: rows x N array; bins: rows x nbins array.  Returns X_r(bins[r, i])
    of Eq. 2 for every row r (same root), each an O(N) sum."""
    a = np.asarray(x)
    b = np.asarray(bins)
    if a.ndim != 2 or b.ndim != 2 or b.shape[0] != a.shape[0]:
        raise ValueError("x must be rows x N and bins rows x nbins")
    rows, N = a.shape
    flat, fb = _arr(a.ravel()), _arr(b.ravel())
    out = np.zeros(fb.size, dtype=np.uint64)
    _load().oracle_ntt_bins_rows(_p(flat), rows, N, int(m), int(root), _p(fb), b.shape[1], _p(out))
    return out.reshape(b.shape)


def ntt2d_bins(x, m: int, root_r: int, root_c: int, bu, bv) -> np.ndarray:
    """Selected outputs X(bu[i], bv[i]) of the 2-D transform of an R x C array
    (Eq. 2 along each dimension), each the O(R C) double sum."""
    a = np.asarray(x)
    if a.ndim != 2:
        raise ValueError("x must be 2-D")
    R, C = a.shape
    u, v = _arr(bu), _arr(bv)
    if u.size != v.size:
        raise ValueError("bu and bv must have the same length")
    out = np.zeros(u.size, dtype=np.uint64)
    rc = _load().oracle_ntt2d_bins(_p(_arr(a.ravel())), R, C, int(m), int(root_r), int(root_c), _p(u), _p(v),
                                   u.size, _p(out))
    if rc:
        raise ValueError("oracle_ntt2d_bins failed with code %d" % rc)
    return out


def conv_direct(f, g, m: int) -> np.ndarray:
    """Circular convolution of Eq. 1 as the O(N^2) direct sum."""
    fa, ga = _arr(f), _arr(g)
    if fa.size != ga.size:
        raise ValueError("f and g must have the same length")
    out = np.zeros_like(fa)
    _load().oracle_conv_direct(_p(fa), _p(ga), _p(out), fa.size, int(m))
    return out


def conv_entries(f, g, m: int, idx) -> np.ndarray:
    """Selected outputs h(j) of Eq. 1, each the O(N) direct sum."""
    fa, ga, ia = _arr(f), _arr(g), _arr(idx)
    out = np.zeros(ia.size, dtype=np.uint64)
    _load().oracle_conv_entries(_p(fa), _p(ga), fa.size, int(m), _p(ia), ia.size, _p(out))
    return out


def conv_via_ntt(f, g, m: int, root: int) -> np.ndarray:
    """Convolution theorem (Sec. I): inverse(forward(f) * forward(g)), all O(N^2)."""
    fa, ga = _arr(f), _arr(g)
    out = np.zeros_like(fa)
    rc = _load().oracle_conv_via_ntt(_p(fa), _p(ga), _p(out), fa.size, int(m), int(root))
    if rc:
        raise ValueError("oracle_conv_via_ntt failed with code %d" % rc)
    return out


class Singular(ValueError):
    """A spectral coefficient of the divisor is zero: no unique quotient."""


def deconv_via_ntt(f, h, m: int, root: int) -> np.ndarray:
    """Exact deconvolution (Sec. III-A, prime modulus): the g with f * g = h,
    inverse(forward(h) / forward(f)), all O(N^2).  Raises Singular when some
    forward(f) bin is zero."""
    fa, ha = _arr(f), _arr(h)
    out = np.zeros_like(fa)
    rc = _load().oracle_deconv_via_ntt(_p(fa), _p(ha), _p(out), fa.size, int(m), int(root))
    if rc == 4:
        raise Singular("a spectral coefficient of f is zero")
    if rc:
        raise ValueError("oracle_deconv_via_ntt failed with code %d" % rc)
    return out


def conv_integer(f, g) -> np.ndarray:
    """The true integer circular convolution (Eq. 1 without the modulus), as
    the O(N^2) direct sum; uint64 results (ValueError if one reaches 2^64)."""
    fa, ga = _arr(f), _arr(g)
    if fa.size != ga.size:
        raise ValueError("f and g must have the same length")
    out = np.zeros_like(fa)
    rc = _load().oracle_conv_integer(_p(fa), _p(ga), _p(out), fa.size)
    if rc:
        raise ValueError("oracle_conv_integer: a result does not fit 64 bits")
    return out


def conv_integer_entries(f, g, idx) -> np.ndarray:
    """Selected outputs of conv_integer, each the O(N) direct sum."""
    fa, ga = _arr(f), _arr(g)
    ia = _arr(idx)
    out = np.zeros(ia.size, dtype=np.uint64)
    rc = _load().oracle_conv_integer_entries(_p(fa), _p(ga), fa.size, _p(ia), ia.size, _p(out))
    if rc:
        raise ValueError("oracle_conv_integer_entries: a result does not fit 64 bits")
    return out


def conv2d_direct(f, g, m: int) -> np.ndarray:
    """Two-dimensional circular convolution of R x C arrays, the O(R^2 C^2)
    direct sum modulo m; returns an R x C uint64 array."""
    fa, ga = np.asarray(f), np.asarray(g)
    if fa.shape != ga.shape or fa.ndim != 2:
        raise ValueError("f and g must be equal 2-D arrays")
    R, C = fa.shape
    out = np.zeros(R * C, dtype=np.uint64)
    _load().oracle_conv2d_direct(_p(_arr(fa.ravel())), _p(_arr(ga.ravel())), _p(out), R, C, int(m))
    return out.reshape(R, C)


def conv2d_entries(f, g, m: int, idx) -> np.ndarray:
    """Selected outputs (flat row-major indices) of conv2d_direct."""
    fa, ga = np.asarray(f), np.asarray(g)
    R, C = fa.shape
    ia = _arr(idx)
    out = np.zeros(ia.size, dtype=np.uint64)
    _load().oracle_conv2d_entries(_p(_arr(fa.ravel())), _p(_arr(ga.ravel())), R, C, int(m), _p(ia), ia.size,
                                  _p(out))
    return out
