"""The C-ABI library: it loads, exports every symbol the header declares, and
validates arguments on the host (these calls return before touching a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nttmi.h")
LIB = os.path.join(ROOT, "paper_1005_1497_amd", "libnttmi.so")

M = 13631489
BAD = ctypes.c_void_p(0x100000)   # never dereferenced: every call below fails validation first


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)) - {"defined"})


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnttmi.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    U64, U32, I32, VP = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
    L.conv_circular.argtypes = [U64, U32, U64, U32, VP, VP, VP, U32, VP]
    L.conv_circular.restype = I32
    L.conv_deconvolve.argtypes = [U64, U32, U64, U32, VP, VP, VP, U32, U32, VP]
    L.conv_deconvolve.restype = I32
    L.conv_crt.argtypes = [U32, VP, VP, VP, U32, U32, VP]
    L.conv_crt.restype = I32
    L.conv2d_circular.argtypes = [U64, U32, U32, U64, U64, U32, VP, VP, VP, U32, VP]
    L.conv2d_circular.restype = I32
    for n in ("ntt_forward", "ntt_inverse"):
        getattr(L, n).argtypes = [U64, U32, U64, U32, VP, VP, U32, U32, VP]
        getattr(L, n).restype = I32
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
    L.ntt_server_create.argtypes = [U64, U64, U32, U32, U32, U32, U32, U64, U32, ctypes.POINTER(VP)]
    L.ntt_server_create.restype = I32
    L.ntt_server_create_host.argtypes = [U64, U64, U32, U32, U32, U32, U32, U64, U32, ctypes.POINTER(VP)]
    L.ntt_server_create_host.restype = I32
    L.ntt_server_submit.argtypes = [VP, VP, VP, U32, ctypes.POINTER(U64)]
    L.ntt_server_submit.restype = I32
    L.ntt_server_stage.argtypes = [VP, U32, VP, VP, VP]
    L.ntt_server_stage.restype = I32
    L.ntt_server_submit_staged.argtypes = [VP, U64]
    L.ntt_server_submit_staged.restype = I32
    L.ntt_server_wait.argtypes = [VP, U64, VP, ctypes.c_double]
    L.ntt_server_wait.restype = I32
    L.ntt_server_stats.argtypes = [VP, VP, VP, VP, VP, U32]
    L.ntt_server_stats.restype = I32
    L.ntt_server_set_solo.argtypes = [VP, U32]
    L.ntt_server_set_solo.restype = I32
    L.ntt_server_destroy.argtypes = [VP]
    L.ntt_server_destroy.restype = None
    L.ntt_status_string.argtypes = [I32]
    L.ntt_status_string.restype = ctypes.c_char_p
    return L


def test_header_declares_the_four_calls():
    fns = header_functions()
    for name in ("ntt_forward", "ntt_inverse", "conv_circular", "conv_batched"):
        assert name in fns


def test_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for s in range(11):
        assert lib.ntt_status_string(s) and b"unknown" not in lib.ntt_status_string(s)
    assert b"unknown" in lib.ntt_status_string(99)


def test_modulus_order(lib):
    out = ctypes.c_uint32(0)
    for m, lognu in ((641, 6), (2424833, 10), (319489, 12), (13631489, 19), (31065037602817, 18)):
        assert lib.ntt_modulus_order(m, ctypes.byref(out)) == 0
        assert out.value == lognu
    assert lib.ntt_modulus_order(341, ctypes.byref(out)) == 2        # composite (Sec. II)
    assert lib.ntt_modulus_order(2 ** 32 + 1, ctypes.byref(out)) == 2  # F_5 composite
    assert lib.ntt_modulus_order(7, ctypes.byref(out)) == 2          # order of 2 is 3


def test_default_root_closed_forms(lib):
    r = ctypes.c_uint64(0)
    assert lib.ntt_default_root(M, 10, ctypes.byref(r)) == 0 and r.value == pow(2, 512, M)
    assert lib.ntt_default_root(M, 16, ctypes.byref(r)) == 0 and r.value == 256
    assert lib.ntt_default_root(M, 19, ctypes.byref(r)) == 0 and r.value == 2
    assert lib.ntt_default_root(M, 0, ctypes.byref(r)) == 0 and r.value == 1
    assert lib.ntt_default_root(M, 20, ctypes.byref(r)) == 3          # NTT_E_LENGTH


def test_conv_validation_errors(lib):
    c = lib.conv_circular
    assert c(341, 2, 4, 32, BAD, BAD, ctypes.c_void_p(0x200000), 0, None) == 2          # modulus composite
    assert c(M, 20, 2, 32, BAD, BAD, ctypes.c_void_p(0x200000), 0, None) == 3           # N does not divide nu
    assert c(M, 10, 2, 32, BAD, BAD, ctypes.c_void_p(0x200000), 0, None) == 4           # 2 has order 2^19
    assert c(M, 10, pow(2, 1024, M), 32, BAD, BAD, ctypes.c_void_p(0x200000), 0, None) == 4  # order 512
    assert c(M, 10, pow(2, 512, M), 16, BAD, BAD, ctypes.c_void_p(0x200000), 0, None) == 1   # elem_bits
    assert c(M, 10, pow(2, 512, M), 32, None, BAD, ctypes.c_void_p(0x200000), 0, None) == 1  # null
    # partial overlap of h with f
    assert c(M, 10, pow(2, 512, M), 32, BAD, ctypes.c_void_p(0x900000), ctypes.c_void_p(0x100000 + 64),
             0, None) == 1
    # a 32-bit word cannot carry a 45-bit modulus
    assert c(31065037602817, 10, pow(2, 256, 31065037602817), 32, BAD, BAD, ctypes.c_void_p(0x200000),
             0, None) == 2


def test_ntt_validation_errors(lib):
    for fn in (lib.ntt_forward, lib.ntt_inverse):
        assert fn(641, 7, 2, 32, BAD, BAD, 1, 0, None) == 3          # 641 allows N <= 64
        assert fn(641, 6, 3, 32, BAD, BAD, 1, 0, None) == 4
        assert fn(M, 4, pow(2, 2 ** 15, M), 32, BAD, BAD, 0, 0, None) == 0  # empty batch: nothing to do
        assert fn(M, 4, pow(2, 2 ** 15, M), 32, None, BAD, 1, 0, None) == 1


def test_u64_validation(lib):
    m = 31065037602817
    c = lib.conv_circular
    # root of the wrong order for 64-bit words
    assert c(m, 10, 2, 64, BAD, BAD, ctypes.c_void_p(0x200000), 0, None) == 4
    # 2^19 does not divide nu = 2^18
    assert c(m, 19, 2, 64, BAD, BAD, ctypes.c_void_p(0x200000), 0, None) == 3
    # a 58-bit Rader prime (order of 2 is 2^28) is valid but beyond exact fp64 residues
    m58 = 231292694251438081
    assert c(m58, 10, pow(2, 2 ** 18, m58), 64, BAD, BAD, ctypes.c_void_p(0x200000), 0, None) == 8


def test_flag_values_match_header():
    import paper_1005_1497_amd as nt
    text = open(HEADER).read()
    flags = dict(re.findall(r"#define\s+NTT_FLAG_(\w+)\s+(0x[0-9a-fA-F]+)u", text))
    assert flags, "no flags in the header"
    for name, val in flags.items():
        assert getattr(nt, "FLAG_" + name) == int(val, 16), name


def test_euler_form_queries_and_validation(lib):
    import paper_1005_1497_amd as nt
    out = ctypes.c_uint32(0)
    for m, v2 in ((7340033, 20), (13631489, 20), (998244353, 23), (31065037602817, 19)):
        assert lib.ntt_max_log2n(m, ctypes.byref(out)) == 0 and out.value == v2
    assert lib.ntt_max_log2n(341, ctypes.byref(out)) == 2
    r = ctypes.c_uint64(0)
    for m, n in ((7340033, 20), (7340033, 7), (13631489, 20), (998244353, 22)):
        assert lib.ntt_euler_root(m, n, ctypes.byref(r)) == 0
        assert pow(r.value, 1 << n, m) == 1 and pow(r.value, 1 << (n - 1), m) == m - 1
    assert lib.ntt_euler_root(7340033, 21, ctypes.byref(r)) == 3
    c = lib.conv_circular
    E = nt.FLAG_EULER
    w10 = pow(3, (7340033 - 1) >> 10, 7340033)   # 3 generates Z_7340033^*
    assert pow(w10, 512, 7340033) == 7340033 - 1
    assert c(7340033, 10, w10, 32, BAD, BAD, ctypes.c_void_p(0x200000), 0, None) == 2   # not a Rader prime
    assert c(7340033, 10, pow(w10, 2, 7340033), 32, BAD, BAD, ctypes.c_void_p(0x200000), E, None) == 4
    assert c(7340033, 21, w10, 32, BAD, BAD, ctypes.c_void_p(0x200000), E, None) == 3   # 2^21 does not divide m - 1
    assert c(341, 2, 4, 32, BAD, BAD, ctypes.c_void_p(0x200000), E, None) == 2           # composite



def test_deconvolve_validation(lib):
    d = lib.conv_deconvolve
    G = ctypes.c_void_p(0x200000)
    assert d(341, 2, 4, 32, BAD, BAD, G, 1, 0, None) == 2                       # composite modulus
    assert d(M, 20, 2, 32, BAD, BAD, G, 1, 0, None) == 3                        # N does not divide nu
    assert d(M, 10, 2, 32, BAD, BAD, G, 1, 0, None) == 4                        # root of the wrong order
    assert d(M, 10, pow(2, 512, M), 32, BAD, BAD, G, 0, 0, None) == 0           # empty batch
    assert d(M, 10, pow(2, 512, M), 32, None, BAD, G, 1, 0, None) == 1          # null
    assert d(M, 10, pow(2, 512, M), 32, BAD, BAD, ctypes.c_void_p(0x100000 + 64), 1, 0, None) == 1  # overlap



def test_crt_validation(lib):
    c = lib.conv_crt
    H = ctypes.c_void_p(0x4000000)
    assert c(20, BAD, BAD, H, 1, 0, None) == 3                                  # beyond 2^19
    assert c(10, BAD, BAD, H, 0, 0, None) == 0                                  # empty batch
    assert c(10, None, BAD, H, 1, 0, None) == 1                                 # null
    assert c(10, BAD, BAD, ctypes.c_void_p(0x100000 + 1024), 1, 0, None) == 1   # h overlaps f



def test_conv2d_validation(lib):
    c = lib.conv2d_circular
    H = ctypes.c_void_p(0x4000000)
    r10, r4 = pow(2, 512, M), pow(2, 1 << 15, M)
    assert c(M, 20, 4, 2, r4, 32, BAD, BAD, H, 0, None) == 3                  # rows beyond nu
    assert c(M, 10, 4, r4, r4, 32, BAD, BAD, H, 0, None) == 4                 # row root of the wrong order
    assert c(M, 10, 4, r10, r10, 32, BAD, BAD, H, 0, None) == 4               # column root of the wrong order
    assert c(M, 10, 4, r10, r4, 32, None, BAD, H, 0, None) == 1               # null
    assert c(M, 10, 4, r10, r4, 32, BAD, BAD, ctypes.c_void_p(0x100000 + 64), 0, None) == 1   # overlap


def test_copy_batch_validation(lib):
    # host-side checks only: nothing reaches the runtime
    import numpy as np
    z = np.zeros(2, np.uint64)
    assert lib.ntt_copy_batch(None, None, None, 0, None) == 0          # nothing to copy
    assert lib.ntt_copy_batch(None, z.ctypes.data, z.ctypes.data, 2, None) == 1
    dst = np.array([0x1000, 0], np.uint64)
    src = np.array([0x2000, 0x3000], np.uint64)
    nb = np.array([8, 8], np.uint64)                                      # entry 1 has a null dst
    assert lib.ntt_copy_batch(dst.ctypes.data, src.ctypes.data, nb.ctypes.data, 2, None) == 1


def test_server_argument_validation(lib):
    # host-side checks before any device work
    h = ctypes.c_void_p()
    M = 13631489
    assert lib.ntt_server_create(M, 2, 19, 32, 20, 4, 512, 0, 4, None) == 1            # no out pointer
    assert lib.ntt_server_create(M, 2, 19, 32, 29, 4, 512, 0, 4, ctypes.byref(h)) == 1  # arena too large
    assert lib.ntt_server_create(M, 2, 19, 32, 20, 0, 512, 0, 4, ctypes.byref(h)) == 1  # no stream
    assert lib.ntt_server_create(M, 2, 19, 32, 20, 17, 512, 0, 4, ctypes.byref(h)) == 1  # too many streams
    assert lib.ntt_server_create(M, 2, 19, 32, 20, 4, 0, 0, 4, ctypes.byref(h)) == 1    # empty batches
    assert lib.ntt_server_create(M, 2, 19, 32, 20, 4, 512, 0, 0, ctypes.byref(h)) == 1  # nothing in flight
    assert lib.ntt_server_create_host(M, 2, 19, 32, 20, 4, 512, 0, 4, None) == 1       # no out pointer
    assert lib.ntt_server_create_host(M, 2, 19, 32, 29, 4, 512, 0, 4, ctypes.byref(h)) == 1  # arena too large
    assert lib.ntt_server_create_host(M, 2, 19, 32, 20, 0, 512, 0, 4, ctypes.byref(h)) == 1  # no stream
    assert lib.ntt_server_create(M + 2, 2, 19, 32, 20, 4, 512, 0, 4, ctypes.byref(h)) == 2  # not a valid modulus
    assert lib.ntt_server_create(M, 3, 19, 32, 20, 4, 512, 0, 4, ctypes.byref(h)) == 4  # 3 has not order 2^19
    t = ctypes.c_uint64()
    assert lib.ntt_server_submit(None, None, None, 4, ctypes.byref(t)) == 1
    assert lib.ntt_server_wait(None, 1, None, 0.0) == 1
    assert lib.ntt_server_stage(None, 4, None, None, None) == 1
    assert lib.ntt_server_set_solo(None, 16) == 1
    assert lib.ntt_server_submit_staged(None, 1) == 1
    assert lib.ntt_server_stats(None, None, None, None, None, 0) == 1
    lib.ntt_server_destroy(None)
