"""GPU parity of the exact deconvolution (division filtering, Sec. III-A):
bit-exact against the oracle's deconvolution where the oracle's O(N^2)
transforms finish quickly, and at every size through the recovery property
deconvolve(f, f * g) = g with f * g from the parity-tested convolution.  A zero
spectral coefficient of the divisor is reported as NTT_E_SINGULAR."""
import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from tests.gpu_util import dev, host, root_of_order

pytestmark = pytest.mark.gpu

M = 13631489


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def _draw(seed, shape, m, bits=32):
    dtype = np.uint32 if bits == 32 else np.uint64
    return np.random.default_rng(seed).integers(0, m, shape, dtype=dtype)


@pytest.mark.parametrize("n", [0, 1, 2, 5, 8, 10, 12])
def test_deconv_matches_oracle(nt, n):
    N = 1 << n
    root = root_of_order(M, 19, n)
    f, h = _draw(300 + n, N, M), _draw(400 + n, N, M)
    try:
        ref = oracle.deconv_via_ntt(f, h, M, root)
    except oracle.Singular:
        pytest.skip("drawn divisor is singular")
    g = host(nt.deconvolve(dev(f), dev(h), M, root=root))
    assert np.array_equal(g, ref.astype(np.uint32))


# divisor seeds 1500 + n draw spectra without a zero coefficient (checked with
# an independent CPU transform when the test was written)
@pytest.mark.parametrize("n,rows", [(4, 300), (11, 5), (13, 3), (16, 2), (19, 1)])
def test_deconv_recovers_at_size(nt, n, rows):
    N = 1 << n
    f, g0 = _draw(1500 + n, (rows, N), M), _draw(600 + n, (rows, N), M)
    hs = []
    for r in range(rows):
        hs.append(nt.conv_circular(dev(f[r]), dev(g0[r]), M))
    h = torch.stack(hs)
    g = host(nt.deconvolve(dev(f), h, M))
    assert np.array_equal(g, g0)


def test_deconv_in_place_and_singular(nt):
    n, N = 13, 1 << 13
    f, g0 = _draw(700, N, M), _draw(701, N, M)
    h = nt.conv_circular(dev(f), dev(g0), M)
    nt.deconvolve(dev(f), h, M, out=h)                       # g written over h
    assert np.array_equal(host(h), g0)
    for bad in (np.ones(N, np.uint32), np.zeros(N, np.uint32)):
        with pytest.raises(nt.NttError) as e:
            nt.deconvolve(dev(bad), dev(g0), M)
        assert e.value.name == "NTT_E_SINGULAR"
    # one singular row among invertible ones
    rows = np.stack([f, np.ones(N, np.uint32), f])
    with pytest.raises(nt.NttError) as e:
        nt.deconvolve(dev(rows), dev(np.stack([g0, g0, g0])), M)
    assert e.value.name == "NTT_E_SINGULAR"


@pytest.mark.parametrize("n", [4, 12, 14])
def test_deconv_u64(nt, n):
    m = si.M_U64
    N = 1 << n
    f, g0 = _draw(800 + n, N, m, 64), _draw(900 + n, N, m, 64)
    h = nt.conv_circular(dev(f), dev(g0), m)
    g = host(nt.deconvolve(dev(f), h, m))
    assert np.array_equal(g, g0)
    if n <= 12:
        ref = oracle.deconv_via_ntt(f, host(h), m, root_of_order(m, 18, n))
        assert np.array_equal(g, ref)


def test_deconv_euler_form(nt):
    m, n = 7340033, 15
    N = 1 << n
    w = nt.euler_root(m, n)
    f, g0 = _draw(1000, N, m), _draw(1001, N, m)
    h = nt.conv_circular(dev(f), dev(g0), m, root=w, flags=nt.FLAG_EULER)
    g = host(nt.deconvolve(dev(f), h, m, root=w, flags=nt.FLAG_EULER))
    assert np.array_equal(g, g0)


def test_deconv_detects_one_zero_bin(nt):
    # this N = 2^19 divisor has exactly one zero spectral coefficient, at
    # u = 413618 (the oracle confirms it below); the GPU must report it
    n, N = 19, 1 << 19
    f = _draw(519, (1, N), M)[0]
    assert oracle.ntt_bins(f, M, 2, np.array([413618]))[0] == 0
    with pytest.raises(nt.NttError) as e:
        nt.deconvolve(dev(f), dev(_draw(1, N, M)), M)
    assert e.value.name == "NTT_E_SINGULAR"


def test_deconv_many_rows_through_the_work_queue(nt):
    # more rows than resident workgroups: the persistent kernel's queue hands
    # them out; every row recovers its g.  Random divisors of this length are
    # singular with probability about N/m per row, so each divisor is made as
    # the inverse transform of a spectrum drawn from [1, m): invertible.
    n, rows = 14, 700
    N = 1 << n
    spec = np.random.default_rng(1700).integers(1, M, (rows, N), dtype=np.uint32)
    f = host(nt.ntt_inverse(dev(spec), M))
    g0 = _draw(1701, (rows, N), M)
    lens = [n] * rows
    offs = [r * N for r in range(rows)]
    h = nt.conv_batched(dev(f.reshape(-1)), dev(g0.reshape(-1)), nt.BatchDesc(lens, offs), M)
    g = host(nt.deconvolve(dev(f), h.reshape(rows, N), M))
    assert np.array_equal(g, g0)


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_deconv_refuses_a_capturing_stream(nt):
    # the quotient's singular flag is read back with a synchronisation, so a
    # call on a stream under graph capture is refused before anything is
    # enqueued (torch reports the captured graph as empty); the stream stays
    # usable and the eager call still recovers g
    n, N = 10, 1 << 10
    f, g0 = _draw(1500 + n, N, M), _draw(610, N, M)
    fd = dev(f)
    h = nt.conv_circular(fd, dev(g0), M)
    out = torch.empty_like(fd)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        nt.deconvolve(fd, h, M, out=out, stream=s)       # plans and workspaces in place
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with pytest.raises(nt.NttError) as e:
        with torch.cuda.graph(graph, stream=s):
            nt.deconvolve(fd, h, M, out=out, stream=s)
    assert e.value.name == "NTT_E_UNSUPPORTED"
    torch.cuda.synchronize()
    out.zero_()
    with torch.cuda.stream(s):
        nt.deconvolve(fd, h, M, out=out, stream=s)
    s.synchronize()
    assert np.array_equal(host(out), g0)
