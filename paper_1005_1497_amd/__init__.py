"""nttmi: exact digital circular convolution modulo a prime on AMD MI355X.

Thin ctypes binding over the C ABI declared in ``include/nttmi.h``
(``libnttmi.so``, built in-tree by ``paper_1005_1497_amd/build.py``).  This
module only marshals arguments: every step of every transform and convolution
runs in the library's HIP kernels.  PyTorch supplies device memory and streams.

Method: S. S. Chandra, "Fast Digital Convolutions using Bit-Shifts"
(arXiv:1005.1497): circular convolution (Eq. 1) by the convolution theorem with
a number-theoretic transform (Eqs. 2, 3) whose root of unity is a power of two
modulo a Rader prime (Prop. 2, Table 1).

Tensors are CUDA (HIP) tensors of 32-bit words (torch.int32 or torch.uint32,
values read as unsigned); results are canonical residues in [0, m).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

__all__ = [
    "NttError", "lib", "ntt_forward", "ntt_inverse", "conv_circular", "conv_circular_noalloc", "conv_batched", "deconvolve", "conv_crt", "conv2d",
    "default_root", "modulus_order", "release_caches", "status_string",
    "FLAG_CHECK_RANGE", "FLAG_PER_ITEM", "FLAG_PER_CLASS", "FLAG_AUTOTUNE", "FLAG_EULER", "FLAG_TRANSIENT", "STATUS",
    "euler_root", "max_log2n", "copy_batch", "launch_counts",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnttmi.so")

STATUS = {
    0: "NTT_OK", 1: "NTT_E_ARG", 2: "NTT_E_MODULUS", 3: "NTT_E_LENGTH", 4: "NTT_E_ROOT",
    5: "NTT_E_RANGE", 6: "NTT_E_NOMEM", 7: "NTT_E_DEVICE", 8: "NTT_E_UNSUPPORTED", 9: "NTT_E_SINGULAR",
    10: "NTT_E_TIMEOUT", 11: "NTT_E_NOPLAN",
}
FLAG_CHECK_RANGE = 0x1
FLAG_PER_ITEM = 0x2
FLAG_PER_CLASS = 0x4
FLAG_AUTOTUNE = 0x8
FLAG_EULER = 0x10
FLAG_TRANSIENT = 0x20

EXPORTS = ("ntt_forward", "ntt_inverse", "conv_circular", "conv_circular_noalloc", "conv_batched", "conv_deconvolve", "conv_crt",
           "conv2d_circular",
           "ntt_default_root",
           "ntt_modulus_order", "ntt_max_log2n", "ntt_euler_root", "ntt_status_string", "ntt_release_caches",
           "ntt_release_stream", "ntt_launch_counts")


class NttError(RuntimeError):
    """A library call returned a status other than NTT_OK."""

    def __init__(self, status: int, where: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__("%s: %s (%s)" % (where, self.name, status_string(status)))


class _BatchDesc(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint32),
                ("log2n", ctypes.POINTER(ctypes.c_uint8)),
                ("offset", ctypes.POINTER(ctypes.c_uint64))]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libnttmi.so is not built: run `python paper_1005_1497_amd/build.py` "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    U64, U32, I32, VP = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
    for name in ("ntt_forward", "ntt_inverse"):
        fn = getattr(L, name)
        fn.argtypes = [U64, U32, U64, U32, VP, VP, U32, U32, VP]
        fn.restype = I32
    L.conv_circular.argtypes = [U64, U32, U64, U32, VP, VP, VP, U32, VP]
    L.conv_circular.restype = I32
    L.conv_circular_noalloc.argtypes = [U64, U32, U64, U32, VP, VP, VP, U32, VP]
    L.conv_circular_noalloc.restype = I32
    L.conv_deconvolve.argtypes = [U64, U32, U64, U32, VP, VP, VP, U32, U32, VP]
    L.conv_deconvolve.restype = I32
    L.conv_crt.argtypes = [U32, VP, VP, VP, U32, U32, VP]
    L.conv_crt.restype = I32
    L.conv2d_circular.argtypes = [U64, U32, U32, U64, U64, U32, VP, VP, VP, U32, VP]
    L.conv2d_circular.restype = I32
    L.conv_batched.argtypes = [U64, U64, U32, U32, ctypes.POINTER(_BatchDesc), VP, VP, VP, U32, VP]
    L.conv_batched.restype = I32
    L.ntt_default_root.argtypes = [U64, U32, ctypes.POINTER(U64)]
    L.ntt_default_root.restype = I32
    L.ntt_modulus_order.argtypes = [U64, ctypes.POINTER(U32)]
    L.ntt_modulus_order.restype = I32
    L.ntt_max_log2n.argtypes = [U64, ctypes.POINTER(U32)]
    L.ntt_max_log2n.restype = I32
    L.ntt_euler_root.argtypes = [U64, U32, ctypes.POINTER(U64)]
    L.ntt_euler_root.restype = I32
    L.ntt_copy_batch.argtypes = [VP, VP, VP, U32, VP]
    L.ntt_copy_batch.restype = I32
    D = ctypes.c_double
    L.ntt_server_create.argtypes = [U64, U64, U32, U32, U32, U32, U32, U64, U32, ctypes.POINTER(VP)]
    L.ntt_server_create.restype = I32
    L.ntt_server_create_host.argtypes = [U64, U64, U32, U32, U32, U32, U32, U64, U32, ctypes.POINTER(VP)]
    L.ntt_server_create_host.restype = I32
    L.ntt_server_submit.argtypes = [VP, VP, VP, U32, ctypes.POINTER(U64)]
    L.ntt_server_submit.restype = I32
    L.ntt_server_stage.argtypes = [VP, U32, ctypes.POINTER(VP), ctypes.POINTER(VP), ctypes.POINTER(U64)]
    L.ntt_server_stage.restype = I32
    L.ntt_server_submit_staged.argtypes = [VP, U64]
    L.ntt_server_submit_staged.restype = I32
    L.ntt_server_wait.argtypes = [VP, U64, VP, D]
    L.ntt_server_wait.restype = I32
    L.ntt_server_stats.argtypes = [VP, ctypes.POINTER(U64), ctypes.POINTER(D), ctypes.POINTER(D),
                                   ctypes.POINTER(D), U32]
    L.ntt_server_stats.restype = I32
    L.ntt_server_set_solo.argtypes = [VP, U32]
    L.ntt_server_set_solo.restype = I32
    L.ntt_server_destroy.argtypes = [VP]
    L.ntt_server_destroy.restype = None
    L.ntt_status_string.argtypes = [I32]
    L.ntt_status_string.restype = ctypes.c_char_p
    L.ntt_release_caches.argtypes = []
    L.ntt_release_caches.restype = None
    L.ntt_release_stream.argtypes = [VP]
    L.ntt_release_stream.restype = None
    L.ntt_launch_counts.argtypes = [ctypes.POINTER(U64), U32]
    L.ntt_launch_counts.restype = None
    return L


lib = _load()


def status_string(status: int) -> str:
    return lib.ntt_status_string(int(status)).decode()


def _check(status: int, where: str) -> None:
    if status != 0:
        raise NttError(status, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


_WORD = {torch.int32: 32, torch.uint32: 32, torch.int64: 64, torch.uint64: 64}


def _words(t: torch.Tensor, what: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % what)
    if t.dtype not in _WORD:
        raise TypeError("%s must be int32/uint32 (or int64/uint64)" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return _WORD[t.dtype]


def _log2(n: int) -> int:
    if n <= 0 or n & (n - 1):
        raise ValueError("length %d is not a power of two" % n)
    return n.bit_length() - 1


def default_root(m: int, log2n: int) -> int:
    """2^(nu/N) mod m: the harmonic of exact order N = 2^log2n (Eq. 5)."""
    r = ctypes.c_uint64(0)
    _check(lib.ntt_default_root(int(m), int(log2n), ctypes.byref(r)), "ntt_default_root")
    return int(r.value)


def modulus_order(m: int) -> int:
    """log2 of the order of 2 modulo m (Prop. 2)."""
    r = ctypes.c_uint32(0)
    _check(lib.ntt_modulus_order(int(m), ctypes.byref(r)), "ntt_modulus_order")
    return int(r.value)


def max_log2n(m: int) -> int:
    """Euler form: the largest n with 2^n dividing m - 1 (m prime)."""
    r = ctypes.c_uint32(0)
    _check(lib.ntt_max_log2n(int(m), ctypes.byref(r)), "ntt_max_log2n")
    return int(r.value)


def euler_root(m: int, log2n: int) -> int:
    """Euler form: a root of exact order 2^log2n modulo the prime m."""
    r = ctypes.c_uint64(0)
    _check(lib.ntt_euler_root(int(m), int(log2n), ctypes.byref(r)), "ntt_euler_root")
    return int(r.value)


def _root(m, log2n, flags):
    return euler_root(m, log2n) if flags & FLAG_EULER else default_root(m, log2n)


def _ntt(fn, name, x, m, root, out, flags, stream):
    bits = _words(x, "x")
    N = x.shape[-1]
    log2n = _log2(N)
    batch = x.numel() // N if x.numel() else 0
    if root is None:
        root = _root(m, log2n, flags)
    if out is None:
        out = torch.empty_like(x)
    elif _words(out, "out") != bits or out.shape != x.shape:
        raise ValueError("out must match x in shape and word width")
    _check(fn(int(m), log2n, int(root), bits, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
              batch, int(flags), _stream(stream)), name)
    return out


def ntt_forward(x: torch.Tensor, m: int, root: int | None = None, out=None, flags: int = 0, stream=None):
    """Eq. 2 along the last dimension (a power of two), natural order."""
    return _ntt(lib.ntt_forward, "ntt_forward", x, m, root, out, flags, stream)


def ntt_inverse(X: torch.Tensor, m: int, root: int | None = None, out=None, flags: int = 0, stream=None):
    """Eq. 3 (including N^-1) along the last dimension."""
    return _ntt(lib.ntt_inverse, "ntt_inverse", X, m, root, out, flags, stream)


def conv_circular(f: torch.Tensor, g: torch.Tensor, m: int, root: int | None = None, out=None,
                  flags: int = 0, stream=None):
    """Circular convolution of Eq. 1 of two 1-D sequences of equal power-of-two length."""
    bits = _words(f, "f")
    if _words(g, "g") != bits or g.shape != f.shape or f.dim() != 1:
        raise ValueError("f and g must be 1-D with the same length and word width")
    log2n = _log2(f.numel())
    if root is None:
        root = _root(m, log2n, flags)
    if out is None:
        out = torch.empty_like(f)
    elif _words(out, "out") != bits or out.shape != f.shape:
        raise ValueError("out must match f")
    _check(lib.conv_circular(int(m), log2n, int(root), bits, ctypes.c_void_p(f.data_ptr()),
                             ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr()), int(flags),
                             _stream(stream)), "conv_circular")
    return out


def conv_circular_noalloc(f: torch.Tensor, g: torch.Tensor, m: int, root: int, out: torch.Tensor, flags: int = 0,
                          stream=None):
    """conv_circular through the entry point that allocates nothing (static
    device scratch; the plan of (m, N, root) must exist from an earlier call).
    The root and the output tensor are required, so this wrapper allocates
    nothing either."""
    bits = _words(f, "f")
    if _words(g, "g") != bits or g.shape != f.shape or f.dim() != 1:
        raise ValueError("f and g must be 1-D with the same length and word width")
    if _words(out, "out") != bits or out.shape != f.shape:
        raise ValueError("out must match f")
    log2n = _log2(f.numel())
    _check(lib.conv_circular_noalloc(int(m), log2n, int(root), bits, ctypes.c_void_p(f.data_ptr()),
                                     ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr()), int(flags),
                                     _stream(stream)), "conv_circular_noalloc")
    return out


def deconvolve(f: torch.Tensor, h: torch.Tensor, m: int, root: int | None = None, out=None, flags: int = 0,
               stream=None):
    """Exact deconvolution: the g with f * g = h (Eq. 1) along the last
    dimension, g = inverse(forward(h) / forward(f)).  Raises NttError
    (NTT_E_SINGULAR) when a forward(f) coefficient is zero.  Synchronises."""
    bits = _words(f, "f")
    if _words(h, "h") != bits or h.shape != f.shape:
        raise ValueError("f and h must match in shape and word width")
    N = f.shape[-1]
    log2n = _log2(N)
    batch = f.numel() // N if f.numel() else 0
    if root is None:
        root = _root(m, log2n, flags)
    if out is None:
        out = torch.empty_like(f)
    elif _words(out, "out") != bits or out.shape != f.shape:
        raise ValueError("out must match f")
    _check(lib.conv_deconvolve(int(m), log2n, int(root), bits, ctypes.c_void_p(f.data_ptr()),
                               ctypes.c_void_p(h.data_ptr()), ctypes.c_void_p(out.data_ptr()), batch, int(flags),
                               _stream(stream)), "conv_deconvolve")
    return out


def conv_crt(f: torch.Tensor, g: torch.Tensor, out=None, stream=None):
    """Exact integer circular convolution along the last dimension (uint32
    operands, int64/uint64 result) from convolutions modulo 13631489 and
    7340033 combined by the Chinese remainder theorem; exact while every true
    value is below their product (about 1.0006e14)."""
    if _words(f, "f") != 32 or _words(g, "g") != 32 or g.shape != f.shape:
        raise ValueError("f and g must be 32-bit words of the same shape")
    N = f.shape[-1]
    log2n = _log2(N)
    batch = f.numel() // N if f.numel() else 0
    if out is None:
        out = torch.empty(f.shape, dtype=torch.int64, device=f.device)
    elif _words(out, "out") != 64 or out.shape != f.shape:
        raise ValueError("out must be 64-bit words of f's shape")
    _check(lib.conv_crt(log2n, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                        ctypes.c_void_p(out.data_ptr()), batch, 0, _stream(stream)), "conv_crt")
    return out


def conv2d(f: torch.Tensor, g: torch.Tensor, m: int, root_r: int | None = None, root_c: int | None = None,
           out=None, flags: int = 0, stream=None):
    """Two-dimensional circular convolution of R x C arrays (powers of two)
    modulo m, each dimension transformed with its own root of exact order."""
    bits = _words(f, "f")
    if _words(g, "g") != bits or g.shape != f.shape or f.dim() != 2:
        raise ValueError("f and g must be 2-D with the same shape and word width")
    log2r, log2c = _log2(f.shape[0]), _log2(f.shape[1])
    if root_r is None:
        root_r = _root(m, log2r, flags)
    if root_c is None:
        root_c = _root(m, log2c, flags)
    if out is None:
        out = torch.empty_like(f)
    elif _words(out, "out") != bits or out.shape != f.shape:
        raise ValueError("out must match f")
    _check(lib.conv2d_circular(int(m), log2r, log2c, int(root_r), int(root_c), bits, ctypes.c_void_p(f.data_ptr()),
                               ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr()), int(flags),
                               _stream(stream)), "conv2d_circular")
    return out


class BatchDesc:
    """Host-side batch descriptor kept alive between calls (log2n and offsets arrays)."""

    def __init__(self, log2n, offsets):
        import numpy as np
        n = np.asarray(log2n)
        if n.size and (n.min() < 0 or n.max() > 255):
            raise ValueError("log2n values must lie in [0, 255]")
        o = np.asarray(offsets)
        if o.size and o.dtype.kind == "i" and o.min() < 0:
            raise ValueError("offsets must be non-negative")
        self.log2n = np.ascontiguousarray(n.astype(np.uint8))
        self.offset = np.ascontiguousarray(o.astype(np.uint64))
        if self.log2n.shape != self.offset.shape:
            raise ValueError("log2n and offsets must have the same length")
        # one past the last element any item touches (the C ABI is not given
        # the buffer sizes, so the wrapper checks them against this)
        if self.log2n.size and int(self.log2n.max()) < 64:
            ends = self.offset + np.left_shift(np.uint64(1), self.log2n.astype(np.uint64))
            self.extent = int(ends.max()) if int(ends.min()) >= int(self.offset.min()) else 1 << 64
        else:
            self.extent = 0 if not self.log2n.size else 1 << 64
        self.c = _BatchDesc(len(self.log2n),
                            self.log2n.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            self.offset.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))


def copy_batch(dst, src, nbytes, stream=None) -> None:
    """Enqueues the copies dst[i] <- src[i] of nbytes[i] bytes on ``stream`` in
    one library call (device or pinned host addresses, as integers)."""
    d = np.ascontiguousarray(dst, dtype=np.uint64)
    s_ = np.ascontiguousarray(src, dtype=np.uint64)
    b = np.ascontiguousarray(nbytes, dtype=np.uint64)
    if not (d.ndim == s_.ndim == b.ndim == 1) or not (d.size == s_.size == b.size):
        raise ValueError("dst, src and nbytes must be 1-D of one length")
    _check(lib.ntt_copy_batch(d.ctypes.data, s_.ctypes.data, b.ctypes.data, d.size, _stream(stream)), "ntt_copy_batch")


def conv_batched(f: torch.Tensor, g: torch.Tensor, desc, m: int, root: int = 2, root_log2order: int | None = None,
                 out=None, flags: int = 0, stream=None):
    """A batch of independent circular convolutions of uneven power-of-two lengths.

    ``desc`` is a BatchDesc (or a (log2n, offsets) pair).  Item i uses
    root^(2^(root_log2order - log2n[i])); by default root = 2 with its full order.
    """
    if not isinstance(desc, BatchDesc):
        desc = BatchDesc(*desc)
    bits = _words(f, "f")
    if _words(g, "g") != bits or g.shape != f.shape:
        raise ValueError("f and g must match")
    if root_log2order is None:
        root_log2order = modulus_order(m) if root == 2 else None
        if root_log2order is None:
            raise ValueError("root_log2order is required when root != 2")
    if out is None:
        out = torch.empty_like(f)
    elif _words(out, "out") != bits or out.shape != f.shape:
        raise ValueError("out must match f")
    if desc.extent > f.numel():
        raise ValueError("the batch reaches element %d, beyond the %d elements of f, g and out"
                         % (desc.extent, f.numel()))
    _check(lib.conv_batched(int(m), int(root), int(root_log2order), bits, ctypes.byref(desc.c),
                            ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), int(flags), _stream(stream)), "conv_batched")
    return out


COUNT_NAMES = ("small", "fourstep", "fused", "multi", "transform", "desc_cached", "desc_ring", "desc_evicted",
               "queue_created")


def launch_counts() -> dict:
    """Cumulative launch and descriptor-upload counts of the library by form
    (diagnostics: read before and after a call to see which form it took)."""
    buf = (ctypes.c_uint64 * len(COUNT_NAMES))()
    lib.ntt_launch_counts(buf, len(COUNT_NAMES))
    return dict(zip(COUNT_NAMES, (int(v) for v in buf)))


def release_caches() -> None:
    lib.ntt_release_caches()


def release_stream(stream) -> None:
    """Frees the library's workspaces for `stream` (a torch stream), after
    waiting for it; call before the stream is dropped."""
    lib.ntt_release_stream(_stream(stream))
