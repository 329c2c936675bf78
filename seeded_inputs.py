"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds only data and random draws: the moduli and sizes of the
workloads and numpy PCG64 generators for lengths and operands.  It contains none
of the method's arithmetic (no transform, no reduction, no root computation), so
both the oracle side and the GPU side can use it without sharing code.

Recipe (the same for every workload): ``numpy.random.default_rng(seed)``; draw
the lengths first (if the workload has several), then f, then g, item by item in
index order; operands are ``rng.integers(0, hi, size, dtype)`` with ``hi = m``
unless the workload restricts the values (the N = 2^19 exactness case uses
{0, 1, 2, 3}).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Table 1: the Rader primes and their maximum transform lengths.
M_641 = 641
M_2424833 = 2424833
M_319489 = 319489
M_13631489 = 13631489          # 13 * 2^20 + 1, the 32-bit-word prime with N_Max = 2^19
TABLE1 = {641: 64, 2424833: 1024, 319489: 4096, 13631489: 524288}

# A Rader prime that needs a 64-bit word (Table 1 has no 64-bit row): a factor
# of F_17, 59251857 * 2^19 + 1, 45 bits, order of 2 equal to 2^18.
M_U64 = 31065037602817
M_U64_NMAX = 1 << 18


@dataclass(frozen=True)
class Workload:
    name: str
    m: int
    log2n: tuple            # per-item log2 lengths
    elem_bits: int
    hi: int                 # operands drawn uniformly from [0, hi)
    seed: int
    drawn_lengths: tuple = ()   # (lo, hi) when the lengths were drawn from the seed

    @property
    def count(self) -> int:
        return len(self.log2n)

    @property
    def lengths(self) -> np.ndarray:
        return np.left_shift(np.ones(len(self.log2n), dtype=np.int64), np.array(self.log2n, dtype=np.int64))

    @property
    def total_elems(self) -> int:
        return int(self.lengths.sum())


def single_n1024(seed: int = 1) -> Workload:
    """One convolution, N = 1024, m = 13631489, operands uniform in [0, m)."""
    return Workload("single_n1024_m13631489", M_13631489, (10,), 32, M_13631489, seed)


def batch_n65536(count: int = 4096, seed: int = 2) -> Workload:
    """A batch of independent convolutions of N = 2^16, m = 13631489."""
    return Workload("batch%d_n65536_m13631489" % count, M_13631489, (16,) * count, 32, M_13631489, seed)


def single_n524288_small(seed: int = 3) -> Workload:
    """One convolution at N = 2^19 with operands in {0,1,2,3}: N*9 < m, so the
    residue result equals the true integer circular convolution."""
    return Workload("single_n524288_vals0to3_m13631489", M_13631489, (19,), 32, 4, seed)


def uneven_lengths(count: int = 10000, lo: int = 6, hi: int = 19, seed: int = 4) -> np.ndarray:
    """log2 lengths n uniform in [lo, hi] (inclusive), drawn first from the seed."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count)


def uneven_batch(count: int = 10000, seed: int = 4) -> Workload:
    """Uneven batch: lengths 2^n, n uniform in [6, 19], m = 13631489."""
    n = uneven_lengths(count, 6, 19, seed)
    return Workload("uneven%d_n2^6to2^19_m13631489" % count, M_13631489, tuple(int(v) for v in n), 32,
                    M_13631489, seed, (6, 19))


def served_lengths(count: int, seed: int = 5) -> np.ndarray:
    """log2 lengths of served requests, n uniform in [8, 18]."""
    rng = np.random.default_rng(seed)
    return rng.integers(8, 19, size=count)


def operands(w: Workload, rng_offset: int = 0):
    """Draw f and g for every item of w, item by item (f then g), after the
    lengths.  Returns two flat arrays with the items packed back to back."""
    rng = np.random.default_rng(w.seed + rng_offset)
    if w.drawn_lengths:
        # the lengths were drawn first from the same generator; replay that draw
        lo, hi = w.drawn_lengths
        rng.integers(lo, hi + 1, size=w.count)
    dtype = np.uint32 if w.elem_bits == 32 else np.uint64
    total = w.total_elems
    f = np.empty(total, dtype=dtype)
    g = np.empty(total, dtype=dtype)
    off = 0
    for n in w.log2n:
        size = 1 << n
        f[off:off + size] = rng.integers(0, w.hi, size=size, dtype=dtype)
        g[off:off + size] = rng.integers(0, w.hi, size=size, dtype=dtype)
        off += size
    return f, g


def uniform(seed: int, size: int, hi: int, dtype=np.uint32) -> np.ndarray:
    """size values uniform in [0, hi) from PCG64(seed)."""
    return np.random.default_rng(seed).integers(0, hi, size=size, dtype=dtype)


def offsets(log2n) -> np.ndarray:
    """Element offsets of items packed back to back."""
    sizes = np.left_shift(np.ones(len(log2n), dtype=np.uint64), np.asarray(log2n, dtype=np.uint64))
    off = np.zeros(len(log2n), dtype=np.uint64)
    if len(log2n) > 1:
        off[1:] = np.cumsum(sizes)[:-1]
    return off
