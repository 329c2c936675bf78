"""GPU parity over seeded random batch shapes: item counts, uneven lengths
2^0..2^19 (2^18 for 64-bit words), gaps between items, items listed out of
address order, and the three launch forms (default, one launch per length,
one launch sequence per item).  Every form must give the same words, and
sampled items must equal the oracle's Eq. 1 sums at sampled indices (all of
an item's outputs when it is short)."""
import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

CASES = 24


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def _shape(rng, nmax):
    """log2 lengths and element offsets of one random batch (at most about
    2^23 elements in all)."""
    count = int(rng.choice([1, 2, 3, 7, 20, 64, 150, 400]))
    budget = 1 << 23
    lens = []
    for _ in range(count):
        # mostly short items, now and then a long one
        n = int(rng.integers(0, nmax + 1)) if rng.random() < 0.3 else int(rng.integers(0, 13))
        if sum(1 << k for k in lens) + (1 << n) > budget:
            break
        lens.append(n)
    if not lens:
        lens = [int(rng.integers(0, 10))]
    offs, pos = [], 0
    for n in lens:
        pos += int(rng.integers(0, 3)) * int(rng.integers(0, 64))   # optional gap
        offs.append(pos)
        pos += 1 << n
    order = np.arange(len(lens))
    if rng.random() < 0.3:
        rng.shuffle(order)                                            # listed out of address order
    return [lens[i] for i in order], [offs[i] for i in order], pos


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("case", range(CASES))
def test_random_batch_shape(nt, case, bits):
    rng = np.random.default_rng(1000 + case + (0 if bits == 32 else 500))
    wide = bits == 64
    m = si.M_U64 if wide else si.M_13631489
    nmax = 18 if wide else 19
    dt = np.uint64 if wide else np.uint32
    lens, offs, total = _shape(rng, nmax)
    f = rng.integers(0, m, total, dtype=dt)
    g = rng.integers(0, m, total, dtype=dt)
    desc = nt.BatchDesc(lens, offs)
    fd, gd = dev(f), dev(g)
    outs = []
    for flags in (0, nt.FLAG_PER_CLASS, nt.FLAG_PER_ITEM):
        h = torch.zeros_like(fd)
        nt.conv_batched(fd, gd, desc, m, out=h, flags=flags)
        outs.append(host(h))
    print("case %d: %d items, lengths %s, %d words%s" % (case, len(lens), sorted(set(lens)), total,
                                                         " (64-bit)" if wide else ""), flush=True)
    assert np.array_equal(outs[0], outs[1]), "one launch per length differs"
    assert np.array_equal(outs[0], outs[2]), "one launch sequence per item differs"
    h = outs[0]
    picks = sorted(set([0, len(lens) - 1] + list(rng.integers(0, len(lens), 3))))
    for i in picks:
        N, o = 1 << lens[i], offs[i]
        fi, gi = f[o:o + N], g[o:o + N]
        if N <= 256:
            ref = oracle.conv_direct(fi, gi, m).astype(np.uint64)
            assert np.array_equal(h[o:o + N].astype(np.uint64), ref), (case, i)
        else:
            idx = np.unique(np.concatenate([[0, N - 1], rng.integers(0, N, 6)])).astype(np.uint64)
            ref = oracle.conv_entries(fi, gi, m, idx)
            assert np.array_equal(h[o + idx.astype(np.int64)].astype(np.uint64), ref), (case, i)
    # words outside every item stay as they were (zero)
    mask = np.zeros(total, dtype=bool)
    for n, o in zip(lens, offs):
        mask[o:o + (1 << n)] = True
    assert not np.any(h[~mask]), "a gap was written"
