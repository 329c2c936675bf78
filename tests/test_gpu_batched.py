"""GPU parity of the batched forms: the fused batch equals the same items run
one by one, and the oracle on sampled items."""
import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

M = 13631489


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def _item_root(n):
    return pow(2, 1 << (19 - n), M)


@pytest.mark.parametrize("n,count", [(4, 300), (8, 70), (12, 5), (13, 9), (16, 6), (16, 700)])
def test_uniform_batch_matches_oracle(nt, n, count):
    w = si.Workload("t", M, (n,) * count, 32, M, 11 + n)
    f, g = si.operands(w)
    desc = nt.BatchDesc([n] * count, si.offsets([n] * count))
    h = host(nt.conv_batched(dev(f), dev(g), desc, M))
    N = 1 << n
    rng = np.random.default_rng(n)
    items = sorted(set([0, count - 1] + list(rng.integers(0, count, 3))))
    for i in items:
        fi, gi = f[i * N:(i + 1) * N], g[i * N:(i + 1) * N]
        if n <= 13:
            assert np.array_equal(h[i * N:(i + 1) * N], oracle.conv_direct(fi, gi, M).astype(np.uint32)), i
        else:
            idx = rng.integers(0, N, 24)
            assert np.array_equal(h[i * N + idx], oracle.conv_entries(fi, gi, M, idx).astype(np.uint32)), i
    # the same batch, one item per launch sequence
    h1 = host(nt.conv_batched(dev(f), dev(g), desc, M, flags=nt.FLAG_PER_ITEM))
    assert np.array_equal(h, h1)


def test_uneven_batch_matches_per_item(nt):
    w = si.uneven_batch(count=60, seed=4)
    f, g = si.operands(w)
    offs = si.offsets(w.log2n)
    desc = nt.BatchDesc(w.log2n, offs)
    h = host(nt.conv_batched(dev(f), dev(g), desc, M))
    h1 = host(nt.conv_batched(dev(f), dev(g), desc, M, flags=nt.FLAG_PER_ITEM))
    assert np.array_equal(h, h1)
    for i, n in enumerate(w.log2n):
        N = 1 << n
        o = int(offs[i])
        fi, gi, hi = f[o:o + N], g[o:o + N], h[o:o + N]
        if n <= 10:
            assert np.array_equal(hi, oracle.conv_direct(fi, gi, M).astype(np.uint32)), (i, n)
        else:
            idx = np.array([0, N - 1, N // 3])
            assert np.array_equal(hi[idx], oracle.conv_entries(fi, gi, M, idx).astype(np.uint32)), (i, n)


def test_gapped_offsets_and_empty(nt):
    # items out of order with gaps between them
    log2n = [5, 9, 3, 9, 13]
    offs = [9000, 0, 700, 20000, 40000]
    total = 40000 + (1 << 13) + 5
    f = si.uniform(1, total, M)
    g = si.uniform(2, total, M)
    out = dev(np.zeros(total, np.uint32))
    nt.conv_batched(dev(f), dev(g), nt.BatchDesc(log2n, offs), M, out=out)
    h = host(out)
    for n, o in zip(log2n, offs):
        N = 1 << n
        assert np.array_equal(h[o:o + N], oracle.conv_direct(f[o:o + N], g[o:o + N], M).astype(np.uint32))
    assert h[600] == 0 and h[total - 1] == 0        # gaps untouched
    nt.conv_batched(dev(f), dev(g), nt.BatchDesc([], []), M)  # empty batch


def test_overlapping_items_rejected(nt):
    f = dev(np.zeros(4096, np.uint32))
    with pytest.raises(nt.NttError) as e:
        nt.conv_batched(f, f, nt.BatchDesc([10, 10], [0, 512]), M)
    assert e.value.name == "NTT_E_ARG"


def _forms_agree(nt, lengths, seed, m=M, words=32):
    offs = si.offsets(lengths)
    w = si.Workload("forms", m, tuple(lengths), words, m, seed)
    f, g = si.operands(w)
    desc = nt.BatchDesc(lengths, offs)
    one = host(nt.conv_batched(dev(f), dev(g), desc, m))                       # one launch
    per_class = host(nt.conv_batched(dev(f), dev(g), desc, m, flags=nt.FLAG_PER_CLASS))
    per_item = host(nt.conv_batched(dev(f), dev(g), desc, m, flags=nt.FLAG_PER_ITEM))
    assert np.array_equal(one, per_class)
    assert np.array_equal(one, per_item)
    return f, g, offs, one


def test_single_launch_every_length(nt):
    # every length 2^0 .. 2^19 once, some twice, ragged tiles of the short
    # lengths; the single persistent launch equals the per-class and per-item
    # forms, and the oracle on each item (direct sum up to 2^10, sampled above)
    lengths = list(range(20)) + [19, 13, 12, 12, 12, 7, 0] + [6] * 130
    f, g, offs, h = _forms_agree(nt, lengths, 31)
    rng = np.random.default_rng(5)
    for n, o in zip(lengths, offs):
        N, o = 1 << n, int(o)
        fi, gi = f[o:o + N], g[o:o + N]
        if n <= 10:
            assert np.array_equal(h[o:o + N], oracle.conv_direct(fi, gi, M).astype(np.uint32)), n
        else:
            idx = rng.integers(0, N, 6)
            assert np.array_equal(h[o + idx], oracle.conv_entries(fi, gi, M, idx).astype(np.uint32)), n


def test_single_launch_reused_and_reordered(nt):
    # the same lengths in another order, twice in a row on one stream (the
    # work queue re-arms itself), and a batch whose longest item is short
    lengths = [12, 16, 3, 16, 14, 9, 15, 13, 12, 3]
    for _ in range(2):
        _forms_agree(nt, lengths, 32)
    _forms_agree(nt, [12, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2, 1, 0] * 3, 33)


@pytest.mark.parametrize("lengths", [
    [16] * 40,                                     # one length, many items
    [16] * 3,                                      # one length, few items
    [5] * 50 + [10] * 9 + [12] * 3,                # short lengths only
    list(range(6, 20)) * 3,                        # the uneven mix
])
def test_autotuned_form_matches(nt, lengths):
    offs = si.offsets(lengths)
    w = si.Workload("tune", M, tuple(lengths), 32, M, 51)
    f, g = si.operands(w)
    desc = nt.BatchDesc(lengths, offs)
    ref = host(nt.conv_batched(dev(f), dev(g), desc, M, flags=nt.FLAG_PER_ITEM))
    tuned = host(nt.conv_batched(dev(f), dev(g), desc, M, flags=nt.FLAG_AUTOTUNE))
    assert np.array_equal(tuned, ref)
    again = host(nt.conv_batched(dev(f), dev(g), desc, M))        # the cached form
    assert np.array_equal(again, ref)
    # in place (h is f), tuned afresh: the trial runs must not clobber the operands
    nt.release_caches()
    fd = dev(f)
    nt.conv_batched(fd, dev(g), desc, M, out=fd, flags=nt.FLAG_AUTOTUNE)
    assert np.array_equal(host(fd), ref)


def test_full_size_batch_in_bench_configuration(nt):
    # the timed workload itself: 4096 x N = 2^16 through the persistent fused
    # launch (the bench's launch configuration).  Every item is checked by the
    # convolution theorem (Sec. I) at four random bins, H(u) = F(u) G(u) with
    # the oracle's O(N) transform sums (Eq. 2), and through its values at
    # x = 1 and x = -1; eight whole items equal the oracle's direct sum (Eq. 1).
    w = si.batch_n65536(4096)
    n, count, N = 16, 4096, 1 << 16
    f, g = si.operands(w)
    desc = nt.BatchDesc([n] * count, si.offsets([n] * count))
    before = nt.launch_counts()
    hd = host(nt.conv_batched(dev(f), dev(g), desc, M))
    assert nt.launch_counts()["fused"] == before["fused"] + 1
    assert hd.max() < M
    h = hd.reshape(count, N)
    F, G = f.reshape(count, N), g.reshape(count, N)
    root = 256                                          # 2^8, of exact order 2^16
    rng = np.random.default_rng(99)
    bins = rng.integers(0, N, (count, 4)).astype(np.uint64)
    bins[:, 0] = rng.integers(1, N // 2, count)        # at least one bin away from 0 and N/2
    Fb = oracle.ntt_bins_rows(F, M, root, bins)
    Gb = oracle.ntt_bins_rows(G, M, root, bins)
    Hb = oracle.ntt_bins_rows(h, M, root, bins)
    prod = (Fb.astype(object) * Gb.astype(object)) % M
    bad = np.nonzero(prod.astype(np.uint64) != Hb)
    assert bad[0].size == 0, ("item", int(bad[0][0]), "bin", int(bins[bad[0][0], bad[1][0]]))
    Fi, Gi, Hi = F.astype(np.int64), G.astype(np.int64), h.astype(np.int64)
    at_one = lambda x: x.sum(axis=1) % M
    at_minus_one = lambda x: (x[:, 0::2].sum(axis=1) - x[:, 1::2].sum(axis=1)) % M
    assert np.array_equal(at_one(Hi), at_one(Fi) * at_one(Gi) % M)
    assert np.array_equal(at_minus_one(Hi), at_minus_one(Fi) * at_minus_one(Gi) % M)
    for i in (0, 1, 2, 1000, 2047, 3000, 4094, count - 1):
        assert np.array_equal(h[i], oracle.conv_direct(F[i], G[i], M).astype(np.uint32)), i


def test_transient_descriptors_many_batches_in_flight(nt):
    # 40 distinct batches (single- and multi-length, items in shuffled 2^16
    # blocks, so every batch needs a descriptor) issued back to back on two
    # streams with FLAG_TRANSIENT, more uploads in flight per stream than the
    # staging ring has slots; each output equals the cached-descriptor form
    S, BLK = 1 << 20, 1 << 16
    rng = np.random.default_rng(31)
    f = dev(rng.integers(0, M, S, dtype=np.uint32))
    g = dev(rng.integers(0, M, S, dtype=np.uint32))
    batches = []
    for b in range(40):
        k = int(rng.integers(2, 12))
        blocks = rng.permutation(S // BLK)[:k]
        if b % 3 == 0:
            lens = [int(rng.integers(4, 17))] * k
        else:
            lens = [int(v) for v in rng.integers(4, 17, k)]
        batches.append(nt.BatchDesc(lens, [int(x) * BLK for x in blocks]))
    refs = []
    for d in batches:
        refs.append(host(nt.conv_batched(f, g, d, M)))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.zeros_like(f) for _ in batches]
    torch.cuda.synchronize()
    for i, d in enumerate(batches):
        s = streams[i % 2]
        with torch.cuda.stream(s):
            nt.conv_batched(f, g, d, M, out=outs[i], flags=nt.FLAG_TRANSIENT, stream=s)
    torch.cuda.synchronize()
    fh, gh = host(f), host(g)
    for i, d in enumerate(batches):
        o = host(outs[i])
        for n, off in zip(d.log2n, d.offset):
            a, z = int(off), int(off) + (1 << int(n))
            if not np.array_equal(o[a:z], refs[i][a:z]):
                idx = np.array([0, (z - a) // 2, z - a - 1])
                orc = oracle.conv_entries(fh[a:z], gh[a:z], M, idx).astype(np.uint32)
                pytest.fail("batch %d item 2^%d at %d: transient zero=%s, transient==oracle %s, cached==oracle %s"
                            % (i, int(n), a, bool((o[a:z] == 0).all()), bool(np.array_equal(o[a:z][idx], orc)),
                               bool(np.array_equal(refs[i][a:z][idx], orc))))


def test_first_call_on_fresh_streams_after_release(nt):
    # regression: a stream's work queue is created (zeroed) at its first call;
    # the zeroing must be ordered before that call's persistent kernel on the
    # caller's non-blocking stream, also while another stream keeps the GPU busy
    # two items of 2^14 and of 2^16 that are not back to back: the batch keeps
    # the single multi-length launch (a persistent kernel on the work queue)
    lengths = [14, 6, 15, 14, 7, 5, 12, 16, 9, 16]
    offs = [int(i) << 16 for i in range(len(lengths))]
    rng = np.random.default_rng(41)
    S = len(lengths) << 16
    f = dev(rng.integers(0, M, S, dtype=np.uint32))
    g = dev(rng.integers(0, M, S, dtype=np.uint32))
    desc = nt.BatchDesc(lengths, offs)
    ref = host(nt.conv_batched(f, g, desc, M))
    busy_n = 64 << 16
    busy = dev(rng.integers(0, M, busy_n, dtype=np.uint32))
    busy_desc = nt.BatchDesc([16] * 64, si.offsets([16] * 64))
    for rep in range(3):
        nt.release_caches()
        a, b = torch.cuda.Stream(), torch.cuda.Stream()
        out = torch.zeros_like(f)
        busy_out = torch.zeros_like(busy)
        torch.cuda.synchronize()
        before = nt.launch_counts()
        with torch.cuda.stream(a):
            nt.conv_batched(busy, busy, busy_desc, M, out=busy_out, stream=a)
        with torch.cuda.stream(b):
            nt.conv_batched(f, g, desc, M, out=out, stream=b)
        torch.cuda.synchronize()
        after = nt.launch_counts()
        # the second call created its stream's work queue and ran the
        # multi-length kernel on it
        assert after["multi"] == before["multi"] + 1 and after["queue_created"] >= before["queue_created"] + 1
        o = host(out)
        for n, off in zip(lengths, offs):
            assert np.array_equal(o[off:off + (1 << n)], ref[off:off + (1 << n)]), (rep, n)


def test_release_stream_then_reuse(nt):
    # ntt_release_stream frees a stream's workspaces and work queue; the next
    # call on that stream creates them again and gives the same results (also
    # a stream the library never used may be released)
    # items of 2^16 and 2^13 not back to back: the multi-length launch, which
    # needs the stream's work queue
    lengths = [16, 16, 13, 16, 7, 16, 13, 15, 16, 16]
    offs = si.offsets(lengths)
    rng = np.random.default_rng(43)
    S = int(offs[-1]) + (1 << lengths[-1])
    f = dev(rng.integers(0, M, S, dtype=np.uint32))
    g = dev(rng.integers(0, M, S, dtype=np.uint32))
    desc = nt.BatchDesc(lengths, offs)
    ref = host(nt.conv_batched(f, g, desc, M))
    fh, gh = host(f), host(g)
    for k, idx in ((4, np.arange(1 << 7)), (6, np.array([0, 1, 4095, 8191]))):
        o, n = int(offs[k]), 1 << lengths[k]
        got = ref[o:o + n][idx]
        assert np.array_equal(got, oracle.conv_entries(fh[o:o + n], gh[o:o + n], M, idx).astype(got.dtype)), k
    nt.release_stream(torch.cuda.Stream())
    s = torch.cuda.Stream()
    for rep in range(3):
        out = torch.zeros_like(f)
        torch.cuda.synchronize()
        before = nt.launch_counts()
        with torch.cuda.stream(s):
            nt.conv_batched(f, g, desc, M, out=out, stream=s)
        nt.release_stream(s)
        after = nt.launch_counts()
        assert after["multi"] == before["multi"] + 1 and after["queue_created"] == before["queue_created"] + 1, rep
        assert np.array_equal(host(out), ref), rep


@pytest.mark.parametrize("n", [8, 12, 16])
def test_packed_one_length_batch_from_an_offset(nt, n):
    # one length, items back to back from a non-zero first offset (the packed
    # launch path), plain and after NTT_FLAG_AUTOTUNE stored a form for the
    # shape; the words before the first item stay untouched
    count, first = 37, 3 << n
    lengths = [n] * count
    offs = [first + (i << n) for i in range(count)]
    S = first + (count << n)
    rng = np.random.default_rng(44 + n)
    fh = rng.integers(0, M, S, dtype=np.uint32)
    gh = rng.integers(0, M, S, dtype=np.uint32)
    f, g = dev(fh), dev(gh)
    desc = nt.BatchDesc(lengths, offs)
    for flags in (0, nt.FLAG_AUTOTUNE, 0):
        out = torch.full_like(f, 7)
        o = host(nt.conv_batched(f, g, desc, M, out=out, flags=flags))
        assert np.all(o[:first] == 7)
        for k in (0, 17, count - 1):
            a = offs[k]
            idx = np.array([0, 1, (1 << n) - 1]) if n > 12 else np.arange(1 << n)
            got = o[a:a + (1 << n)][idx]
            want = oracle.conv_entries(fh[a:a + (1 << n)], gh[a:a + (1 << n)], M, idx).astype(got.dtype)
            assert np.array_equal(got, want), (flags, k)


@pytest.mark.parametrize("n,count", [(13, 180), (15, 350), (18, 180)])
def test_fused_form_at_full_occupancy(nt, n, count):
    # enough items to fill the resident workgroups, so the default form is the
    # persistent fused kernel (fewer items take the four-step form); sampled
    # outputs of the first, a middle and the last item against the oracle, and
    # the whole output against the four-step form's
    rng = np.random.default_rng(45 + n)
    N = 1 << n
    S = count * N
    fh = rng.integers(0, M, S, dtype=np.uint32)
    gh = rng.integers(0, M, S, dtype=np.uint32)
    f, g = dev(fh), dev(gh)
    desc = nt.BatchDesc([n] * count, si.offsets([n] * count))
    o = host(nt.conv_batched(f, g, desc, M))
    idx = np.concatenate([[0, 1, N - 1], rng.integers(0, N, 5)])
    for k in (0, count // 2, count - 1):
        a = k * N
        assert np.array_equal(o[a:a + N][idx], oracle.conv_entries(fh[a:a + N], gh[a:a + N], M, idx).astype(o.dtype)), k
    # two halves of the batch, each small enough for the four-step form
    half = count // 3
    d2 = nt.BatchDesc([n] * half, si.offsets([n] * half))
    o2 = host(nt.conv_batched(f[:half * N], g[:half * N], d2, M))
    assert np.array_equal(o2, o[:half * N])


def test_multi_length_launch_with_enough_tasks(nt):
    # several lengths, the items of each long length back to back, and more
    # tasks than two thirds of the resident workgroups: the default form is the
    # single multi-length launch because of the task count (with fewer tasks
    # these lengths would take one launch per length); against the per-length
    # form and sampled oracle entries
    rng = np.random.default_rng(46)
    long_ = sorted(int(x) for x in rng.integers(13, 17, 300))
    short = [int(x) for x in rng.integers(6, 13, 200)]
    lengths = short[:100] + long_ + short[100:]
    offs = si.offsets(lengths)
    S = int(offs[-1]) + (1 << lengths[-1])
    fh = rng.integers(0, M, S, dtype=np.uint32)
    gh = rng.integers(0, M, S, dtype=np.uint32)
    f, g = dev(fh), dev(gh)
    desc = nt.BatchDesc(lengths, offs)
    before = nt.launch_counts()
    o = host(nt.conv_batched(f, g, desc, M))
    assert nt.launch_counts()["multi"] == before["multi"] + 1
    per_class = host(nt.conv_batched(f, g, desc, M, flags=nt.FLAG_PER_CLASS))
    assert np.array_equal(o, per_class)
    for k in (0, 123, 499):
        a, N = int(offs[k]), 1 << lengths[k]
        idx = np.array([0, 1, N - 1])
        assert np.array_equal(o[a:a + N][idx], oracle.conv_entries(fh[a:a + N], gh[a:a + N], M, idx).astype(o.dtype)), k


def _few_task_batch(lengths, offs, seed):
    S = max(int(o) + (1 << n) for n, o in zip(lengths, offs))
    rng = np.random.default_rng(seed)
    return rng.integers(0, M, S, dtype=np.uint32), rng.integers(0, M, S, dtype=np.uint32)


def _check_items(o, fh, gh, lengths, offs):
    for n, a in zip(lengths, offs):
        N, a = 1 << n, int(a)
        idx = np.arange(N) if n <= 9 else np.array([0, 1, N // 2, N - 1])
        want = oracle.conv_entries(fh[a:a + N], gh[a:a + N], M, idx).astype(o.dtype)
        assert np.array_equal(o[a:a + N][idx], want), (n, a)


def test_few_tasks_contiguous_long_lengths_take_one_launch_per_length(nt):
    # fewer tasks than two thirds of the multi-length kernel's resident
    # workgroups, and every length above 2^12 one back-to-back run: one launch
    # per length, the long ones in the four-step form that spreads over the chip
    lengths = [8, 9, 15, 15, 15, 17, 17, 6]
    offs = si.offsets(lengths)
    fh, gh = _few_task_batch(lengths, offs, 47)
    f, g = dev(fh), dev(gh)
    desc = nt.BatchDesc(lengths, offs)
    before = nt.launch_counts()
    o = host(nt.conv_batched(f, g, desc, M))
    after = nt.launch_counts()
    assert after["multi"] == before["multi"]
    assert after["fourstep"] == before["fourstep"] + 2        # 2^15 and 2^17
    assert after["small"] == before["small"] + 3              # 2^6, 2^8, 2^9
    assert np.array_equal(o, host(nt.conv_batched(f, g, desc, M, flags=nt.FLAG_PER_CLASS)))
    _check_items(o, fh, gh, lengths, offs)


def test_few_tasks_scattered_long_lengths_keep_the_single_launch(nt):
    # the same lengths with the items of 2^15 apart: the four-step form needs a
    # uniform stride, so the batch keeps the single multi-length launch
    lengths = [15, 8, 15, 9, 15, 17, 17, 6]
    offs = si.offsets(lengths)
    fh, gh = _few_task_batch(lengths, offs, 48)
    f, g = dev(fh), dev(gh)
    desc = nt.BatchDesc(lengths, offs)
    before = nt.launch_counts()
    o = host(nt.conv_batched(f, g, desc, M))
    after = nt.launch_counts()
    assert after["multi"] == before["multi"] + 1
    assert after["fourstep"] == before["fourstep"]
    assert np.array_equal(o, host(nt.conv_batched(f, g, desc, M, flags=nt.FLAG_PER_CLASS)))
    _check_items(o, fh, gh, lengths, offs)


def test_descriptor_cache_eviction_keeps_descriptors_in_use(nt):
    # regression: the content-addressed descriptor cache frees its entries when
    # it is full (256).  Fill it to 255 entries, then run a multi-length batch
    # whose descriptor is new (the call that fills the cache and evicts); the
    # result equals the per-length form, and a second round of distinct
    # descriptors leaves it unchanged
    nt.release_caches()
    small = torch.zeros(1 << 16, dtype=torch.int32, device="cuda")
    before = nt.launch_counts()
    for i in range(255):
        # one length, two items apart: a descriptor of its own in the cache
        nt.conv_batched(small, small, nt.BatchDesc([5, 5], [0, 64 + 32 * i]), M, out=small.clone())
    mid = nt.launch_counts()
    assert mid["desc_cached"] - before["desc_cached"] == 255
    lengths = [16, 9, 16, 13, 5, 13, 12, 16]
    offs = si.offsets(lengths)
    fh, gh = _few_task_batch(lengths, offs, 49)
    f, g = dev(fh), dev(gh)
    desc = nt.BatchDesc(lengths, offs)
    o = host(nt.conv_batched(f, g, desc, M))
    after = nt.launch_counts()
    assert after["multi"] == mid["multi"] + 1
    assert after["desc_evicted"] == mid["desc_evicted"]      # 256 entries now: full, nothing freed yet
    for i in range(40):
        # offset lists not used above (the cache is keyed by content)
        nt.conv_batched(small, small, nt.BatchDesc([6, 6], [0, 40000 + 64 * i]), M, out=small.clone())
    assert nt.launch_counts()["desc_evicted"] > after["desc_evicted"]
    o2 = host(nt.conv_batched(f, g, desc, M))
    ref = host(nt.conv_batched(f, g, desc, M, flags=nt.FLAG_PER_CLASS))
    assert np.array_equal(o, ref) and np.array_equal(o2, ref)
    _check_items(o, fh, gh, lengths, offs)


def test_pinned_host_operands(nt):
    # f, g and h in pinned host memory, passed at the addresses the device
    # sees: the kernels load and store them over the host link, with no copies,
    # and the result equals the batch on device operands (tiles, four-step and
    # per-length forms, transient descriptors in pinned slots as well)
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")     # the runtime the process has loaded
    lengths = [6, 9, 12, 13, 15, 16, 13, 8]
    offs = si.offsets(lengths)
    total = int(offs[-1]) + (1 << lengths[-1])
    rng = np.random.default_rng(61)
    fh = rng.integers(0, M, total, dtype=np.uint32)
    gh = rng.integers(0, M, total, dtype=np.uint32)
    desc = nt.BatchDesc(lengths, offs)
    ref = host(nt.conv_batched(dev(fh), dev(gh), desc, M))
    pf = torch.from_numpy(fh.view(np.int32)).pin_memory()
    pg = torch.from_numpy(gh.view(np.int32)).pin_memory()
    ph = torch.zeros(total, dtype=torch.int32).pin_memory()

    def device_view(t):
        p = ctypes.c_void_p()
        assert hip.hipHostGetDevicePointer(ctypes.byref(p), ctypes.c_void_p(t.data_ptr()), 0) == 0
        return p

    for flags in (0, nt.FLAG_TRANSIENT):
        ph.zero_()
        st = nt.lib.conv_batched(M, 2, 19, 32, ctypes.byref(desc.c), device_view(pf), device_view(pg),
                                 device_view(ph), flags, None)
        assert st == 0
        torch.cuda.synchronize()
        assert np.array_equal(ph.numpy().view(np.uint32), ref), flags
    _check_items(ph.numpy().view(np.uint32), fh, gh, lengths, offs)
