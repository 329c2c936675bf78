"""The entry point that allocates nothing, conv_circular_noalloc, called
through the C ABI: bit-identical to conv_circular (the allocating entry point
it mirrors) on two calls in a row, the second shorter, for both word widths,
on the LDS path and the four-step path whose scratch is the library's static
device array; its refusals leave nothing enqueued."""
import ctypes
import os

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1005_1497_amd", "libnttmi.so")
M = 13631489
M64 = si.M_U64
OK, E_UNSUPPORTED, E_NOPLAN = 0, 8, 11


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    L = ctypes.CDLL(LIB)
    U64, U32, I32, VP = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
    for name in ("conv_circular", "conv_circular_noalloc"):
        fn = getattr(L, name)
        fn.argtypes = [U64, U32, U64, U32, VP, VP, VP, U32, VP]
        fn.restype = I32
    L.ntt_release_caches.argtypes = []
    L.ntt_release_caches.restype = None
    return L


def _dev(a):
    t = torch.from_numpy(a.view(np.int32 if a.dtype == np.uint32 else np.int64)).cuda()
    return t


def _host(t, dtype):
    return t.cpu().numpy().view(dtype)


def _call(lib, name, m, n, root, bits, f, g, h, stream, flags=0):
    return getattr(lib, name)(m, n, root, bits, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                              ctypes.c_void_p(h.data_ptr()), flags, ctypes.c_void_p(stream.cuda_stream))


@pytest.mark.parametrize("m,lognu,bits,sizes", [
    (M, 19, 32, (19, 13)),        # the longest four-step length, then a shorter one
    (M, 19, 32, (16, 10)),        # four-step, then the LDS path
    (M64, 18, 64, (18, 14)),      # 64-bit words at their longest
])
def test_noalloc_equals_conv_circular(lib, m, lognu, bits, sizes):
    dt = np.uint32 if bits == 32 else np.uint64
    s = torch.cuda.Stream()
    cases = []
    for k, n in enumerate(sizes):
        N = 1 << n
        root = pow(2, 1 << (lognu - n), m)
        rng = np.random.default_rng(1000 + 7 * n + bits)
        f, g = rng.integers(0, m, N, dtype=dt), rng.integers(0, m, N, dtype=dt)
        fd, gd = _dev(f), _dev(g)
        ref, out = torch.empty_like(fd), torch.full_like(fd, -1)
        # the allocating entry point builds the plan and gives the reference
        assert _call(lib, "conv_circular", m, n, root, bits, fd, gd, ref, s) == OK
        cases.append((n, root, f, g, fd, gd, ref, out))
    # set-up: the first call on the device looks up the static array's device
    # address, which makes the HIP runtime load the code object that holds it
    # (once per device); from then on no call changes the device's free memory
    n, root, f, g, fd, gd, ref, out = cases[0]
    assert _call(lib, "conv_circular_noalloc", m, n, root, bits, fd, gd, out, s) == OK
    out.fill_(-1)
    s.synchronize()
    free_before = torch.cuda.mem_get_info()[0]
    # two calls in a row on one stream, the second shorter
    for n, root, f, g, fd, gd, ref, out in cases:
        assert _call(lib, "conv_circular_noalloc", m, n, root, bits, fd, gd, out, s) == OK
    s.synchronize()
    assert torch.cuda.mem_get_info()[0] == free_before
    for n, root, f, g, fd, gd, ref, out in cases:
        got, want = _host(out, dt), _host(ref, dt)
        assert np.array_equal(got, want), n
        N = 1 << n
        idx = np.array([0, 1, N // 2, N - 1], np.uint64)
        assert np.array_equal(got[idx.astype(int)].astype(np.uint64), oracle.conv_entries(f, g, m, idx)), n
    # the same pair once more, in the other order (the scratch keeps the last
    # call's contents; every call writes its scratch before reading it)
    for n, root, f, g, fd, gd, ref, out in reversed(cases):
        out.fill_(-1)
        assert _call(lib, "conv_circular_noalloc", m, n, root, bits, fd, gd, out, s) == OK
    s.synchronize()
    for n, root, f, g, fd, gd, ref, out in cases:
        assert np.array_equal(_host(out, dt), _host(ref, dt)), n


def test_noalloc_refusals(lib):
    lib.ntt_release_caches()            # no plan on the device from here on
    s = torch.cuda.Stream()
    # scratch beyond the static array: 2^20 64-bit words of the Euler-form
    # prime 998244353 (2 N 8 bytes = 16 MiB > 4 MiB)
    me, n = 998244353, 20
    N = 1 << n
    root = pow(3, (me - 1) >> n, me)
    a = torch.zeros(N, dtype=torch.int64, device="cuda")
    out = torch.full_like(a, 5)
    assert lib.conv_circular(me, n, root, 64, a.data_ptr(), a.data_ptr(), out.data_ptr(), 0x10, s.cuda_stream) == OK
    out.fill_(5)
    s.synchronize()
    assert _call(lib, "conv_circular_noalloc", me, n, root, 64, a, a, out, s, flags=0x10) == E_UNSUPPORTED
    # the range check reads back: refused
    x = torch.zeros(1 << 10, dtype=torch.int32, device="cuda")
    y = torch.full_like(x, 5)
    root10 = pow(2, 1 << 9, M)
    assert _call(lib, "conv_circular", M, 10, root10, 32, x, x, y, s) == OK
    s.synchronize()
    y.fill_(5)
    assert _call(lib, "conv_circular_noalloc", M, 10, root10, 32, x, x, y, s, flags=0x1) == E_UNSUPPORTED
    # no plan for this root yet (a root of order 2^12 no call has used)
    root12 = pow(2, (1 << 7) * 13, M)
    z = torch.zeros(1 << 12, dtype=torch.int32, device="cuda")
    w = torch.full_like(z, 5)
    assert _call(lib, "conv_circular_noalloc", M, 12, root12, 32, z, z, w, s) == E_NOPLAN
    s.synchronize()
    assert bool((out == 5).all()) and bool((y == 5).all()) and bool((w == 5).all())
