// Length-L transforms of a block of S sequences, one workgroup, on gfx950.
//
// The fast algorithm is the Cooley-Tukey factorisation of Eq. 2 with the
// complex root replaced by the integer root of unity (Sec. I), organised as
// Stockham autosort passes so that input and output are both in natural order:
//   pass p (radix R, Ns = product of the earlier radices), virtual item jv:
//     load  x[jv + r*L/R], r < R
//     scale x_r *= w_{Ns R}^(r * (jv mod Ns))            (inter-pass twiddle)
//     X = DFT_R(x)                                         (in registers)
//     store y[(jv / Ns) * Ns * R + (jv mod Ns) + r * Ns]
// Each work item holds E = min(16, L) residues in fp64 registers; the first
// pass takes radix R0 = 2^(log2 L mod 4) (when that is not 0) so that every
// later pass is radix 16.  Passes exchange data through LDS.
//
// Range: later passes take reduced inputs (|x| <= m/2 + 2), from the
// inter-pass twiddle product, which is applied even when the twiddle is 1;
// pass 0 takes the caller's, reduced or (32-bit words) canonical, |x| < m.
// Inside DFT_R only the non-trivial twiddles multiply, so a pass output is at
// most R (m/2 + 2) <= 8m + 32 in magnitude, the first pass's at most 16 m:
// inside the 48m limit of the product.
#pragma once
#include "arith.hpp"

namespace nttmi {

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }
constexpr int brevc(int i, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}

// In-register DFT of radix R on a[0..R), natural order in and out:
//   a[o] <- sum_i a[i] w_R^(i o).
// Radix-2 decimation in time on bit-reversed registers.  tw[e * ts] = w_R^e
// for e < R/2 as (w, w/m).
template <class W, int R>
__device__ __forceinline__ void dft_reg(double* a, const double2* tw, int ts, const ModC& M) {
    constexpr int LB = ilog2c(R);
    double t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[i] = a[brevc(i, LB)];
#pragma unroll
    for (int span = 1; span < R; span <<= 1) {
#pragma unroll
        for (int g = 0; g < R; g += 2 * span) {
#pragma unroll
            for (int k = 0; k < span; ++k) {
                double x = t[g + k];
                double y = t[g + k + span];
                if (k != 0) {
                    y = W::mul_tw(y, tw[k * (R / (2 * span)) * ts], M);
                }
                t[g + k] = x + y;
                t[g + k + span] = x - y;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = t[i];
}

enum { SEQ_FAST = 0, POS_FAST = 1 };

// Orders the LDS writes of an exchange before its reads.  When every sequence
// lives in one wave, the wave's own LDS accesses complete in issue order, so
// only the compiler must be kept from moving accesses across the point;
// otherwise the whole workgroup waits.
template <bool WAVE_LOCAL>
__device__ __forceinline__ void xch_sync() {
    if constexpr (WAVE_LOCAL) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Wave-uniform table read through the constant address space, so that it is
// issued as a scalar load into SGPRs (the tables are never written by kernels).
typedef __attribute__((address_space(4))) const double cdouble;
__device__ __forceinline__ double2 ld_uniform(const double2* P, int idx) {
    const cdouble* q = (const cdouble*)(const void*)P;
    double2 r;
    r.x = q[2 * idx];
    r.y = q[2 * idx + 1];
    return r;
}

// Geometry of a block: S sequences of length L, ORD = which index the thread
// id runs over fastest (SEQ_FAST: sequences, for strided sequences in global
// memory; POS_FAST: positions, for contiguous sequences).
template <int L, int S, int ORD>
struct Blk {
    static constexpr int l = ilog2c(L);
    static constexpr int E = L < 16 ? L : 16;          // residues per work item
    static constexpr int W = L / E;                    // work items per sequence
    static constexpr int T = S * W;                    // threads
    static constexpr int R0 = (L < 16) ? L : ((l % 4) ? (1 << (l % 4)) : 16);
    static constexpr int NP = (L < 16) ? 1 : (l / 4 + ((l % 4) ? 1 : 0));
    static constexpr int RL = (NP > 1) ? 16 : R0;      // radix of the last pass
    static constexpr int V0 = E / R0;                  // virtual items in pass 0
    static constexpr int VL = E / RL;                  // virtual items in the last pass
    // LDS rows of POS_FAST blocks.  Up to 256 positions a row is padded by
    // one double per 16 (the two sequences of a 32-lane group then sit 272
    // doubles apart).  From 512 on a sequence spans 32 lanes or more, and that
    // padding wraps a 32-lane access of consecutive positions onto one bank
    // twice; instead the low five bits of the position are XORed with bits
    // 4..8 and with bits 5..7 (a permutation of every aligned 512 positions,
    // no padding).  On 64 banks of 4 bytes, 32 lanes of 8-byte accesses per
    // cycle, every exchange of the passes (the stride-R0 store after a
    // radix-2/4/8 first pass included) and the reorder between forward and
    // inverse then touch 32 distinct bank pairs per 32 lanes.  Applied to the
    // 512-thread blocks (four-step rows, the multi-length kernel's tiles):
    // measured 2% faster there.  The 256-thread product tiles keep the padding:
    // with the swizzle their LDS instructions no longer pair up (28% more of
    // them) and the tile of 1024 measured 30% slower.
    static constexpr bool SWZ = (ORD == POS_FAST) && L >= 512 && S * L == 8192;
    static constexpr int ROWP = (ORD == POS_FAST) ? (SWZ ? L : L + L / 16) : L;
    static constexpr int LDS_DOUBLES = (NP > 1) ? S * ROWP : 1;
    // every sequence's W work items are lanes of one wave (POS_FAST, W | 64):
    // its exchanges need no workgroup barrier
    static constexpr bool WAVE_LOCAL = (ORD == POS_FAST) && (W <= 64) && (64 % W == 0);

    __device__ static __forceinline__ void item(int tid, int& s, int& j) {
        if (ORD == SEQ_FAST) { s = tid % S; j = tid / S; }
        else { j = tid % W; s = tid / W; }
    }
    __device__ static __forceinline__ int lds(int s, int pos) {
        if (ORD == SEQ_FAST) return pos * S + s;
        if constexpr (SWZ) return s * ROWP + (pos ^ ((pos >> 4) & 31) ^ ((pos >> 5) & 7));
        else return s * ROWP + pos + (pos >> 4);
    }
    // position of register i at the input of pass 0
    __device__ static __forceinline__ int pos0(int j, int i) {
        return j + (i / R0) * W + (i % R0) * (L / R0);
    }
    // position of register i at the output of the last pass
    __device__ static __forceinline__ int posL(int j, int i) {
        return j + (i / RL) * W + (i % RL) * (L / RL);
    }
};

// v[r] *= tw(r) mod m for r < R, with the table loads software-pipelined in
// groups of four (at most eight 16-byte twiddles in flight per lane), so that
// the loads do not all sit in VGPRs at once.
template <class W, int R, class TW>
__device__ __forceinline__ void mul_twiddles(double* v, const ModC& M, TW tw) {
    constexpr int G = R < 4 ? R : 4;
    double2 w0[G], w1[G];
#pragma unroll
    for (int q = 0; q < G; ++q) w0[q] = tw(q);
#pragma unroll
    for (int g = 0; g < R / G; ++g) {
        __builtin_amdgcn_sched_barrier(0);
        if (g + 1 < R / G) {
#pragma unroll
            for (int q = 0; q < G; ++q) w1[q] = tw((g + 1) * G + q);
        }
#pragma unroll
        for (int q = 0; q < G; ++q) v[g * G + q] = W::mul_tw(v[g * G + q], w0[q], M);
#pragma unroll
        for (int q = 0; q < G; ++q) w0[q] = w1[q];
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Index of w^e (e taken modulo N) in a table of powers P[e] = w^e, e < N,
// for the sub-transform root w_L = w^(N/L); INV selects w^-1.
template <bool INV>
__device__ __forceinline__ int tw_index(int eL, int lshift, int nmask) {
    int idx = eL << lshift;
    return INV ? ((-idx) & nmask) : idx;
}

// Full length-L transform of the block.  `twf(v, p, Ns, k)` multiplies v[r]
// by w_{16 Ns}^(r k) (or its inverse) for r < 16: the inter-pass twiddles of
// pass p.  On entry v[i] holds the pass-0 input
// at position Blk::pos0(j, i) of sequence s (reduced); on exit v[i] holds the
// output at Blk::posL(j, i).  `ldsbuf` must be free on entry and is free on
// exit.  P is the power table of the item's N-th root (N = L << lshift).
// REVS (SEQ_FAST only): the last exchange hands sequence S - 1 - s to work
// item s, so on exit v holds the transform of sequence S - 1 - s (the
// twiddles depend on positions only).
template <class W, int L, int S, int ORD, bool INV, bool REVS = false, class TWF>
__device__ __forceinline__ void block_dft_tw(double* v, double* ldsbuf, int s, int j,
                                             const double2* __restrict__ P, int lshift, int nmask,
                                             const ModC& M, TWF twf) {
    using B = Blk<L, S, ORD>;
    static_assert(!REVS || (ORD == SEQ_FAST && B::NP > 1), "sequence reversal: SEQ_FAST blocks with an exchange");
    constexpr int E = B::E;
    // keep the uniform twiddle loads inside this transform (not hoisted into
    // the caller's loops, where several transforms' tables would pile up)
    asm volatile("" ::: "memory");
    double2 twE[E / 2 > 0 ? E / 2 : 1];
#pragma unroll
    for (int e = 0; e < E / 2; ++e) twE[e] = ld_uniform(P, tw_index<INV>(e * (L / E), lshift, nmask));

    // pass 0: V0 independent DFTs of radix R0, no inter-pass twiddle
#pragma unroll
    for (int vv = 0; vv < B::V0; ++vv) dft_reg<W, B::R0>(v + vv * B::R0, twE, E / B::R0, M);

    int Ns = B::R0;
#pragma unroll
    for (int p = 1; p < B::NP; ++p) {
        const int Rp = (p == 1) ? B::R0 : 16;   // radix of the pass that produced v
        const int Vp = E / Rp;
        const int NsP = Ns / Rp;                // its stride
        // write outputs of the previous pass
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int vv = i / Rp, r = i % Rp;
            const int jv = j + vv * B::W;
            const int pos = (jv / NsP) * NsP * Rp + (jv % NsP) + r * NsP;
            ldsbuf[B::lds(s, pos)] = v[i];
        }
        (void)Vp;
        xch_sync<B::WAVE_LOCAL>();
        // read inputs of this pass (radix 16, one virtual item jv = j)
        const int sr = (REVS && p == B::NP - 1) ? S - 1 - s : s;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = ldsbuf[B::lds(sr, j + r * (L / 16))];
        xch_sync<B::WAVE_LOCAL>();
        // inter-pass twiddles w_{16 Ns}^(r k) = w_L^((L/(16 Ns)) r k), k = j mod Ns
        twf(v, p, Ns, j & (Ns - 1));
        dft_reg<W, 16>(v, twE, 1, M);
        Ns *= 16;
    }
}

// Two independent length-L transforms of the same block geometry, pass by
// pass in lockstep (va, vb as in block_dft_tw): the two register sets give the
// scheduler independent work around each exchange, and the uniform twiddles
// are loaded once.  The exchanges of va and vb take turns in `ldsbuf`.
template <class W, int L, int S, int ORD, bool INV, class TWF>
__device__ __forceinline__ void block_dft2_tw(double* va, double* vb, double* ldsbuf, int s, int j,
                                              const double2* __restrict__ P, int lshift, int nmask,
                                              const ModC& M, TWF twf) {
    using B = Blk<L, S, ORD>;
    constexpr int E = B::E;
    asm volatile("" ::: "memory");
    double2 twE[E / 2 > 0 ? E / 2 : 1];
#pragma unroll
    for (int e = 0; e < E / 2; ++e) twE[e] = ld_uniform(P, tw_index<INV>(e * (L / E), lshift, nmask));
#pragma unroll
    for (int vv = 0; vv < B::V0; ++vv) {
        dft_reg<W, B::R0>(va + vv * B::R0, twE, E / B::R0, M);
        dft_reg<W, B::R0>(vb + vv * B::R0, twE, E / B::R0, M);
    }
    int Ns = B::R0;
#pragma unroll
    for (int p = 1; p < B::NP; ++p) {
        const int Rp = (p == 1) ? B::R0 : 16;
        const int NsP = Ns / Rp;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            double* v = half ? vb : va;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int vv = i / Rp, r = i % Rp;
                const int jv = j + vv * B::W;
                const int pos = (jv / NsP) * NsP * Rp + (jv % NsP) + r * NsP;
                ldsbuf[B::lds(s, pos)] = v[i];
            }
            xch_sync<B::WAVE_LOCAL>();
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = ldsbuf[B::lds(s, j + r * (L / 16))];
            xch_sync<B::WAVE_LOCAL>();
        }
        twf(va, p, Ns, j & (Ns - 1));
        twf(vb, p, Ns, j & (Ns - 1));
        dft_reg<W, 16>(va, twE, 1, M);
        dft_reg<W, 16>(vb, twE, 1, M);
        Ns *= 16;
    }
}

// Per-pass twiddle tables of a length-L transform, laid out [pass][k][r] with
// entry w_{16 Ns}^(r k) (k < Ns, r < 16), so that one work item's sixteen
// twiddles are contiguous.  Rows are padded to 17 entries so that lanes with
// consecutive k read different LDS banks.  Pass p >= 1 has Ns = R0 16^(p-1).
template <int L>
struct PassTab {
    using B = Blk<L, 1, SEQ_FAST>;
    static constexpr int ROW = 17;
    static constexpr int ns(int p) { return p <= 0 ? 1 : (p == 1 ? B::R0 : 16 * ns(p - 1)); }
    static constexpr int off(int p) { return p <= 1 ? 0 : off(p - 1) + ROW * ns(p - 1); }
    static constexpr int SIZE = B::NP > 1 ? off(B::NP) : 1;   // entries of all passes
    // exponent of w_L of entry (p, k, r)
    __device__ static __forceinline__ int expo(int p, int k, int r) { return (L / (16 * ns(p))) * r * k; }
};

// block_dft_tw with the inter-pass twiddles read from the global power table
// (software-pipelined loads).
template <class W, int L, int S, int ORD, bool INV>
__device__ __forceinline__ void block_dft(double* v, double* ldsbuf, int s, int j,
                                          const double2* __restrict__ P, int lshift, int nmask,
                                          const ModC& M) {
    block_dft_tw<W, L, S, ORD, INV>(v, ldsbuf, s, j, P, lshift, nmask, M, [&](double* vv, int, int Ns, int k) {
        const int step = (L / (16 * Ns)) * k;
        mul_twiddles<W, 16>(vv, M, [&](int r) { return P[tw_index<INV>(step * r, lshift, nmask)]; });
    });
}

}  // namespace nttmi
