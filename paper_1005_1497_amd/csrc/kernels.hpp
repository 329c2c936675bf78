// Device code of the library (gfx950): the kernels as templates, shared by
// the launcher translation units (launch_*.hip).
//
// Small lengths (N <= 2^SMALL_MAX_LOG2N): one workgroup transforms whole
// sequences in LDS; the fused convolution kernel runs forward(f), forward(g),
// the pointwise product, inverse and the N^-1 scaling in one launch (Sec. I,
// convolution theorem; Eqs. 1-3).
//
// Large lengths: the four-step factorisation N = A * B (the multi-dimensional
// technique mentioned in Sec. I): length-B transforms down the A columns, the
// twiddle w^(t1 u2), length-A transforms along the B rows.  For a convolution
// the frequency-domain order is internal, so no transpose is needed: the row
// phase runs forward(f), forward(g), product, inverse and the inverse twiddle
// on each row, and the last phase runs the inverse column transforms.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <type_traits>

#include "blockdft.hpp"
#include "launch.hpp"

namespace nttmi {

// Length cases of the launchers: log2 N handled in LDS, and by the four-step path.
#define NTT_SMALL_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)
#define NTT_LARGE_CASES(X) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22)

// Pass-0 inputs of a transform of two or more passes from E operand words.
// Such a transform takes pass-0 inputs of magnitude up to m as well as reduced
// ones: the first pass's outputs are then at most 16 m, inside the 48 m limit
// of the inter-pass twiddle product that reduces them.  So 32-bit words that
// are all below m in the wave (canonical operands, the usual case) enter as
// they are, and the E reductions are replaced by one maximum; a wave with any
// word at or above m reduces them all.  64-bit words are always reduced: their
// product limit is 12 m.  (Used by the four-step column phase; in the LDS
// tiles the extra live values cost a wave of occupancy.)
template <class W, int E>
__device__ __forceinline__ void load_pass0(double* v, const typename W::word* w, const ModC& M) {
    if constexpr (W::WB == 4) {
        // each word is converted as it arrives (no word stays live)
        uint32_t mx = 0;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            v[i] = (double)w[i];
            mx = w[i] > mx ? w[i] : mx;
        }
        if (__builtin_amdgcn_ballot_w64((double)mx >= M.m) != 0) {
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = reduce(v[i], M);
        }
    } else {
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = W::load_reduce(w[i], M);
    }
}

// ------------------------------------------------------------------ small N
// Convolutions per workgroup of the LDS kernels: 256 threads (small_s), or one
// wave per tile up to L = 1024 (small_s_wave), which spreads a short batch over
// more CUs.
constexpr int small_s(int L) { return L < 16 ? 256 : 4096 / L; }
constexpr int small_s_wave(int L) { return L < 16 ? 64 : (L <= 1024 ? 1024 / L : 1); }
constexpr int small_threads(int L, int S) { return L < 16 ? S : S * (L / 16); }

// Pointwise step between the forward and inverse transforms.  OP_MUL, the
// convolution (Eq. 1 by the convolution theorem, Sec. I): F * (G N^-1).
// OP_DIV, the deconvolution (division filtering; the prime modulus makes every
// nonzero coefficient invertible, Sec. III-A): (G N^-1) / F, with F reduced and
// inverted as F^(m-2) (Fermat); a zero F sets *singular (the quotient is then
// meaningless, and the caller reports it).  F and G are forward outputs
// (|.| <= 8m + 32 for 32-bit words, < 12 m for 64-bit words).
enum { OP_MUL = 0, OP_DIV = 1, OP_CRT = 2 };   // OP_CRT: OP_MUL with the two-prime final store
template <class W, int OP>
__device__ __forceinline__ double spectral(double F, double G, const DevPlan& p, const ModC& M,
                                           uint32_t* singular) {
    const double gs = W::mul_tw(G, make_double2(p.ninv, p.ninvq), M);
    if constexpr (OP == OP_MUL) {
        return W::mul_var(F, gs, M);
    } else {
        const double fr = W::reduce_s(F, M);
        if (fr == 0.0) atomicOr(singular, 1u);
        const uint64_t e = (uint64_t)M.m - 2;
        const int top = 63 - __builtin_clzll(e);
        return W::mul_var(pow_mod<W>(fr, e, top, M), gs, M);
    }
}

template <class W, class FT>
__device__ __forceinline__ double spec_in(FT x) {
    if constexpr (std::is_same<FT, double>::value) return x;
    else return W::from_s(x);
}

// The pointwise step over the E values of a work item: v[i] <- spectral(F[i],
// v[i]).  OP_DIV inverts the E divisor values together (Montgomery's
// simultaneous inversion): one Fermat power of the product of all E, then each
// inverse from the prefix products while the running inverse is peeled back
// factor by factor; 3 (E - 1) products and one power in place of E powers.  A
// zero divisor value sets *singular and enters the products as 1.
template <class W, int OP, int E, class FT>
__device__ __forceinline__ void spectral_block(const FT* F, double* v, const DevPlan& p, const ModC& M,
                                               uint32_t* singular) {
    if constexpr (OP == OP_MUL || E == 1) {
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = spectral<W, OP>(spec_in<W>(F[i]), v[i], p, M, singular);
    } else {
        const double2 ni = make_double2(p.ninv, p.ninvq);
        double c[E];   // c[i] = r_0 r_1 ... r_i
        bool zero = false;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            double r = W::reduce_s(spec_in<W>(F[i]), M);
            zero |= (r == 0.0);
            r = (r == 0.0) ? 1.0 : r;
            c[i] = (i == 0) ? r : W::mul_var(c[i - 1], r, M);
        }
        if (zero) atomicOr(singular, 1u);
        const uint64_t e = (uint64_t)M.m - 2;
        const int top = 63 - __builtin_clzll(e);
        double inv = pow_mod<W>(c[E - 1], e, top, M);   // (r_0 ... r_{E-1})^-1
#pragma unroll
        for (int i = E - 1; i >= 1; --i) {
            // r_i is formed again rather than kept (registers)
            double r = W::reduce_s(spec_in<W>(F[i]), M);
            r = (r == 0.0) ? 1.0 : r;
            const double ri = W::mul_var(inv, c[i - 1], M);   // r_i^-1
            inv = W::mul_var(inv, r, M);                       // (r_0 ... r_{i-1})^-1
            v[i] = W::mul_var(ri, W::mul_tw(v[i], ni, M), M);
        }
        v[0] = W::mul_var(inv, W::mul_tw(v[0], ni, M), M);
    }
}

// Inter-pass twiddle table of a length-L transform (PassTab layout: pass,
// k, 17 entries per row; INV: of the inverse transform), filled cooperatively
// by the workgroup; the caller synchronises before use.
template <int L, class T, bool INV = false>
__device__ __forceinline__ void fill_pass_tab(T* t, const DevPlan& p, int logn) {
    using PT = PassTab<L>;
    using B = Blk<L, 1, SEQ_FAST>;
    const int lshift = logn - B::l;
    const int nmask = (1 << logn) - 1;
#pragma unroll
    for (int q = 1; q < B::NP; ++q) {
        const int cnt = 16 * PT::ns(q);
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            const int k = e >> 4, r = e & 15;
            const double2 w = p.P[tw_index<INV>(PT::expo(q, k, r), lshift, nmask)];
            if constexpr (std::is_same<T, double2>::value) t[PT::off(q) + k * PT::ROW + r] = w;
            else t[PT::off(q) + k * PT::ROW + r] = w.x;
        }
    }
}

// Inter-pass twiddles of a length-L transform from its shared pass table.
template <class W, int L, class T>
struct TwTab {
    const T* t;
    ModC M;
    __device__ __forceinline__ void operator()(double* v, int p, int, int k) const {
        const T* b = t + PassTab<L>::off(p) + PassTab<L>::ROW * k;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if constexpr (std::is_same<T, double2>::value) v[r] = W::mul_tw(v[r], b[r], M);
            else v[r] = W::mul_w(v[r], b[r], M);
        }
    }
};
template <class W, int L, class T>
__device__ __forceinline__ TwTab<W, L, T> twtab(const T* t, const ModC& M) {
    return TwTab<W, L, T>{t, M};
}

// Tiles whose inter-pass twiddles sit in an LDS table (PassTab<L>) beside the
// exchange buffer: (w, w/m) pairs while both fit half a CU's LDS, else w alone
// (w/m formed at use).
constexpr bool small_tab(int L) { return L >= 32 && L <= (1 << SMALL_MAX_LOG2N); }
// 256-thread tiles whose table is split (SplitTab): the full table keeps them at
// two workgroups per CU (72 KB), the split one at three (41-44 KB).  Measured
// on 2^26-element batches: convolutions at 2048 and 4096 0.427 -> 0.369 ms (64-bit
// words 0.322 -> 0.297), transforms 0.220-0.239 -> 0.182-0.184 ms forward; at 1024
// the split table gained nothing (its full table already leaves three per CU).
constexpr bool small_split(int L) { return L >= 2048 && L <= (1 << SMALL_MAX_LOG2N); }

// Split twiddle table of a length-L transform with three passes (L >= 512):
// pass 1's table as in PassTab, then for the last pass (Ns = ns(2)) a 16 x 17
// table of w_{16 Ns}^(r kl), kl < 16, instead of its Ns x 17 one.  The last
// pass's twiddle for k = 16 kh + kl is pass 1's entry (kh, r) = w_Ns^(r kh)
// times the small table's (kl, r): one product more per twiddle, and a table of
// 544 instead of 4624 entries at 4096 (8.7 instead of 74 KB of pairs).
template <int L>
struct SplitTab {
    using PT = PassTab<L>;
    static constexpr int LAST = Blk<L, 1, SEQ_FAST>::NP - 1;
    static_assert(LAST == 2, "split table: transforms of three passes");
    static constexpr int LO = PT::off(LAST);   // where the small table starts
    static constexpr int SIZE = LO + PT::ROW * 16;
};

template <int L, class T, bool INV = false>
__device__ __forceinline__ void fill_split_tab(T* t, const DevPlan& p, int logn) {
    using PT = PassTab<L>;
    using ST = SplitTab<L>;
    const int lshift = logn - Blk<L, 1, SEQ_FAST>::l;
    const int nmask = (1 << logn) - 1;
    for (int e = threadIdx.x; e < 16 * PT::ns(1) + 256; e += blockDim.x) {
        const bool lo = e >= 16 * PT::ns(1);
        const int f = lo ? e - 16 * PT::ns(1) : e;
        const int k = f >> 4, r = f & 15;
        const double2 w = p.P[tw_index<INV>(PT::expo(lo ? ST::LAST : 1, k, r), lshift, nmask)];
        T* d = t + (lo ? ST::LO : PT::off(1)) + k * PT::ROW + r;
        if constexpr (std::is_same<T, double2>::value) *d = w;
        else *d = w.x;
    }
}

template <class W, int L, class T>
struct TwSplit {
    const T* t;
    ModC M;
    __device__ __forceinline__ void operator()(double* v, int p, int, int k) const {
        using PT = PassTab<L>;
        using ST = SplitTab<L>;
        if (p < ST::LAST) {
            const T* b = t + PT::off(p) + PT::ROW * k;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if constexpr (std::is_same<T, double2>::value) v[r] = W::mul_tw(v[r], b[r], M);
                else v[r] = W::mul_w(v[r], b[r], M);
            }
        } else {
            const T* bh = t + PT::off(ST::LAST - 1) + PT::ROW * (k >> 4);
            const T* bl = t + ST::LO + PT::ROW * (k & 15);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                double w;
                if constexpr (std::is_same<T, double2>::value) w = W::mul_tw(bh[r].x, bl[r], M);
                else w = W::mul_w(bh[r], bl[r], M);
                v[r] = W::mul_w(v[r], w, M);
            }
        }
    }
};

// One tile of S convolutions of length L <= 2^12, entirely in the LDS of one
// workgroup of S * max(1, L/16) threads: forward(f), forward(g), the product
// with N^-1 folded in, inverse and the canonical store.  Item s of the tile
// starts at offs[s] (offs != null) or at base + s L; items s >= cnt are
// computed on item 0's data and not stored.
//
// TAB: the inter-pass twiddles come from `tab`, the workgroup's LDS table of
// the forward transform (filled by the caller), and the inverse runs as the
// forward transform of the spectrum with its index negated (x(t) = N^-1
// F(X)(-t) = N^-1 F(X(-.))(t), Eq. 3 through Eq. 2), so one table serves all
// three transforms.  Otherwise they are read from the global power table.
template <class W, int L, int S, int OP = OP_MUL, bool TAB = false, class TE = double2>
__device__ __forceinline__ void small_conv_tile(const typename W::word* f, const typename W::word* g,
                                                typename W::word* h, const uint64_t* offs, uint64_t base,
                                                uint32_t cnt, const DevPlan& p, double* lds, int tid,
                                                uint32_t* singular = nullptr, const TE* tab = nullptr) {
    using B = Blk<L, S, POS_FAST>;
    static_assert(!TAB || B::NP > 1, "twiddle table: transforms with more than one pass");
    int s, j;
    B::item(tid, s, j);
    const bool valid = (uint32_t)s < cnt;
    const uint32_t si = valid ? (uint32_t)s : 0u;
    const uint64_t off = offs ? offs[si] : base + (uint64_t)si * L;
    const ModC M = p.M;
    const int lshift = p.logn - B::l;
    // the forward transform of f waits in scratch words (|F| <= 8m + 32 fits
    // an int32 for 32-bit words), which halves its registers
    typename W::sword F[B::E];
    double v[B::E];
    // At L = 4096 g's words are loaded before f is transformed, so that their
    // latency overlaps f's transform (measured 4.5% there; at shorter lengths
    // the extra registers cost a wave of occupancy or spill)
    constexpr bool PRE_G = L >= 4096;
    typename W::word gw[PRE_G ? B::E : 1];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = W::load_reduce(f[off + B::pos0(j, i)], M);
    if constexpr (PRE_G) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) gw[i] = g[off + B::pos0(j, i)];
    }
    auto forward = [&](double* vv) {
        if constexpr (TAB && small_split(L))
            block_dft_tw<W, L, S, POS_FAST, false>(vv, lds, s, j, p.P, lshift, p.nmask, M, TwSplit<W, L, TE>{tab, M});
        else if constexpr (TAB)
            block_dft_tw<W, L, S, POS_FAST, false>(vv, lds, s, j, p.P, lshift, p.nmask, M, twtab<W, L>(tab, M));
        else
            block_dft<W, L, S, POS_FAST, false>(vv, lds, s, j, p.P, lshift, p.nmask, M);
    };
    forward(v);
#pragma unroll
    for (int i = 0; i < B::E; ++i) F[i] = W::to_s(v[i]);
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = W::load_reduce(PRE_G ? gw[PRE_G ? i : 0] : g[off + B::pos0(j, i)], M);
    forward(v);
    // pointwise step with N^-1 folded in
    if constexpr (OP == OP_MUL) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = spectral<W, OP_MUL>(W::from_s(F[i]), v[i], p, M, singular);
    } else {
        spectral_block<W, OP, B::E>(F, v, p, M, singular);
    }
    if (TAB || B::R0 != B::RL) {
        // output positions of the forward transform differ from the input
        // positions of the inverse (or, TAB, the spectrum is read at negated
        // frequencies): reorder through LDS
#pragma unroll
        for (int i = 0; i < B::E; ++i) {
            const int k = B::posL(j, i);
            lds[B::lds(s, TAB ? ((L - k) & (L - 1)) : k)] = v[i];
        }
        xch_sync<B::WAVE_LOCAL>();
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = lds[B::lds(s, B::pos0(j, i))];
        xch_sync<B::WAVE_LOCAL>();
    }
    if constexpr (TAB) forward(v);
    else block_dft<W, L, S, POS_FAST, true>(v, lds, s, j, p.P, lshift, p.nmask, M);
    if (valid) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) h[off + B::posL(j, i)] = W::canon(v[i], M);
    }
}

// The product kernels of 32-bit words up to 1024 fit three waves per SIMD
// (<= 168 VGPRs) without spilling: measured 13% faster at 1024 than the
// unconstrained allocation (two waves).  Longer tiles, 64-bit words and the
// quotient (more registers) would spill there.

template <int L, int S>
constexpr bool small_tab_pairs() {
    return 8 * Blk<L, S, POS_FAST>::LDS_DOUBLES + 16 * PassTab<L>::SIZE <= 80 * 1024;
}

constexpr int small_waves_per_eu(int L, int op, int wb) { return (L <= 1024 && op == OP_MUL && wb == 4) ? 3 : 1; }

template <class W, int L, int S, int OP>
__global__ __launch_bounds__(256, (small_waves_per_eu(L, OP, W::WB))) void k_conv_small(const typename W::word* f,
                                                                               const typename W::word* g,
                                                    typename W::word* h, const uint64_t* __restrict__ offs,
                                                    uint32_t count, DevPlan p, uint32_t* singular) {
    __shared__ double lds[Blk<L, S, POS_FAST>::LDS_DOUBLES];
    const uint64_t first = (uint64_t)blockIdx.x * S;
    const uint32_t cnt = (uint32_t)(count - first < (uint64_t)S ? count - first : (uint64_t)S);
    // (the one-wave tiles keep the global table: a table per 64 threads would
    // cost more LDS, and more loads to fill, than it saves)
    if constexpr (small_tab(L) && S == small_s(L) && small_split(L)) {
        __shared__ double2 tab[SplitTab<L>::SIZE];
        fill_split_tab<L>(tab, p, p.logn);
        __syncthreads();
        small_conv_tile<W, L, S, OP, true, double2>(f, g, h, offs ? offs + first : nullptr, first * L, cnt, p, lds,
                                                    threadIdx.x, singular, tab);
    } else if constexpr (small_tab(L) && S == small_s(L)) {
        using TE = typename std::conditional<small_tab_pairs<L, S>(), double2, double>::type;
        __shared__ TE tab[PassTab<L>::SIZE];
        fill_pass_tab<L>(tab, p, p.logn);
        __syncthreads();
        small_conv_tile<W, L, S, OP, true, TE>(f, g, h, offs ? offs + first : nullptr, first * L, cnt, p, lds,
                                               threadIdx.x, singular, tab);
    } else {
        small_conv_tile<W, L, S, OP>(f, g, h, offs ? offs + first : nullptr, first * L, cnt, p, lds, threadIdx.x,
                                     singular);
    }
}

// MULIN (inverse only): the input is the pointwise product x y mod m, formed
// on load (the 2-D convolution's product step fused into its first inverse pass).
template <class W, int L, bool INV, bool MULIN = false>
__global__ __launch_bounds__(256) void k_ntt_small(const typename W::word* x, typename W::word* X, uint32_t batch,
                                                   DevPlan p, const typename W::word* y) {
    constexpr int S = small_s(L);
    using B = Blk<L, S, POS_FAST>;
    __shared__ double lds[B::LDS_DOUBLES];
    int s, j;
    B::item(threadIdx.x, s, j);
    const uint64_t row = (uint64_t)blockIdx.x * S + s;
    const bool valid = row < batch;
    const uint64_t off = valid ? row * (uint64_t)L : 0;
    const ModC M = p.M;
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = W::load_reduce(x[off + B::pos0(j, i)], M);
    if constexpr (MULIN) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = W::mul_var(v[i], W::load_reduce(y[off + B::pos0(j, i)], M), M);
    }
    // (one transform per tile: the table pays where it keeps three or more
    // workgroups per CU; at 2048 and 4096 the full table measured even and
    // 6-13% slower than the global power table, the split one 17-26% faster)
    if constexpr (small_split(L)) {
        __shared__ double2 tab[SplitTab<L>::SIZE];
        fill_split_tab<L, double2, INV>(tab, p, p.logn);
        __syncthreads();
        block_dft_tw<W, L, S, POS_FAST, INV>(v, lds, s, j, p.P, p.logn - B::l, p.nmask, M,
                                             TwSplit<W, L, double2>{tab, M});
    } else if constexpr (small_tab(L) && L <= 1024) {
        using TE = typename std::conditional<small_tab_pairs<L, S>(), double2, double>::type;
        __shared__ TE tab[PassTab<L>::SIZE];
        fill_pass_tab<L, TE, INV>(tab, p, p.logn);
        __syncthreads();
        block_dft_tw<W, L, S, POS_FAST, INV>(v, lds, s, j, p.P, p.logn - B::l, p.nmask, M, twtab<W, L>(tab, M));
    } else {
        block_dft<W, L, S, POS_FAST, INV>(v, lds, s, j, p.P, p.logn - B::l, p.nmask, M);
    }
    if (valid) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) {
            const double y = INV ? W::mul_tw(v[i], make_double2(p.ninv, p.ninvq), M) : v[i];
            X[off + B::posL(j, i)] = W::canon(y, M);
        }
    }
}

// ------------------------------------------------------------------ four-step
// Geometry for N = 2^LOGN = A * B, A = 2^fs_la(LOGN) (row length),
// B = N / A (column length).  Element t = t1 + A t2 (t1 < A, t2 < B),
// frequency u = u2 + B u1.  Scratch rows: Y[u2 * A + t1].
template <int LOGN, int TT = 512>
struct FS {
    static constexpr int la = fs_la(LOGN), lb = LOGN - fs_la(LOGN);
    static constexpr int A = 1 << la, Bn = 1 << lb, N = 1 << LOGN;
    // threads per workgroup: 512, so that a column block of B = 256 spans 32
    // columns (128-byte rows of a block: whole cache lines); 256 for the
    // multi-launch kernels of batches too short to fill the chip with
    // 512-thread blocks (half the columns and rows per block, twice the
    // workgroups)
    static constexpr int T = TT;
    static constexpr int SC = 16 * T / Bn; // columns per block
    static constexpr int SR = 16 * T / A;  // rows per block
    using BC = Blk<Bn, SC, SEQ_FAST>;
    using BR = Blk<A, SR, POS_FAST>;
    using BRS = Blk<A, SR, SEQ_FAST>;      // rows read/written at stride B (natural-order NTT)
    static constexpr int mx(int a, int b) { return a > b ? a : b; }
    static constexpr int XCH = mx(mx(BC::LDS_DOUBLES, BR::LDS_DOUBLES), BRS::LDS_DOUBLES);
};

// Buffer resource over [p, p + bytes) (raw, untyped; out-of-range reads
// return 0 and out-of-range writes are dropped).  Accesses take a per-lane
// byte offset and a wave-uniform byte offset, so that the strided accesses of
// a work item cost no per-element address arithmetic.
#ifndef NTT_STREAM_AUX
#define NTT_STREAM_AUX 2   // cache policy of streamed operands: non-temporal
#endif
struct Buf {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ Buf(const void* p, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000)) {}
    __device__ __forceinline__ uint32_t ld32(uint32_t v, uint32_t s) const {
        return __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0);
    }
    __device__ __forceinline__ int32_t ldi32(uint32_t v, uint32_t s) const {
        return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0);
    }
    __device__ __forceinline__ double ld64f(uint32_t v, uint32_t s) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
    }
    __device__ __forceinline__ void st32(uint32_t x, uint32_t v, uint32_t s) const {
        __builtin_amdgcn_raw_buffer_store_b32(x, r, v, s, 0);
    }
    // streaming (non-temporal) variants for operands read or written once
    __device__ __forceinline__ uint32_t ld32s(uint32_t v, uint32_t s) const {
        return __builtin_amdgcn_raw_buffer_load_b32(r, v, s, NTT_STREAM_AUX);
    }
    __device__ __forceinline__ void st32s(uint32_t x, uint32_t v, uint32_t s) const {
        __builtin_amdgcn_raw_buffer_store_b32(x, r, v, s, NTT_STREAM_AUX);
    }
    __device__ __forceinline__ uint64_t ld64(uint32_t v, uint32_t s) const {
        return __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
    }
    __device__ __forceinline__ void st64(uint64_t x, uint32_t v, uint32_t s) const {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, x),
                                              r, v, s, 0);
    }
};

// Four-step twiddle w^(t1 u2) from the plan's table (the inverse transforms
// use it too): 32-bit words when the modulus fits (half the bytes and
// registers of the fp64 table).
template <class W>
struct Tw4 {
    using T = typename std::conditional<W::WB == 4, uint32_t, double>::type;
    __device__ static __forceinline__ Buf buf(const DevPlan& p, uint32_t n) {
        if constexpr (W::WB == 4) return Buf(p.TT32, n * 4u);
        else return Buf(p.TT, n * 8u);
    }
    __device__ static __forceinline__ T ld(const Buf& b, uint32_t ve, uint32_t se) {
        if constexpr (W::WB == 4) return b.ld32(ve * 4u, se * 4u);
        else return b.ld64f(ve * 8u, se * 8u);
    }
};

// Word accesses of streamed operands (read or written once per launch).
template <class W>
__device__ __forceinline__ typename W::word ld_word_s(const Buf& b, uint32_t ve, uint32_t se) {
    if constexpr (W::WB == 4) return b.ld32s(ve * 4u, se * 4u);
    else return b.ld64(ve * 8u, se * 8u);
}
template <class W>
__device__ __forceinline__ void st_word_s(const Buf& b, typename W::word x, uint32_t ve, uint32_t se) {
    if constexpr (W::WB == 4) b.st32s(x, ve * 4u, se * 4u);
    else b.st64(x, ve * 8u, se * 8u);
}

// Word and scratch accesses by element offsets (per-lane, uniform).
template <class W>
__device__ __forceinline__ typename W::word ld_word(const Buf& b, uint32_t ve, uint32_t se) {
    if constexpr (W::WB == 4) return b.ld32(ve * 4u, se * 4u);
    else return b.ld64(ve * 8u, se * 8u);
}
template <class W>
__device__ __forceinline__ void st_word(const Buf& b, typename W::word x, uint32_t ve, uint32_t se) {
    if constexpr (W::WB == 4) b.st32(x, ve * 4u, se * 4u);
    else b.st64(x, ve * 8u, se * 8u);
}
template <class W>
__device__ __forceinline__ double ld_scr(const Buf& b, uint32_t ve, uint32_t se) {
    if constexpr (W::SB == 4) return W::from_s(b.ldi32(ve * 4u, se * 4u));
    else return b.ld64f(ve * 8u, se * 8u);
}
template <class W>
__device__ __forceinline__ typename W::sword ld_scr_raw(const Buf& b, uint32_t ve, uint32_t se) {
    if constexpr (W::SB == 4) return b.ldi32(ve * 4u, se * 4u);
    else return b.ld64f(ve * 8u, se * 8u);
}
template <class W>
__device__ __forceinline__ void st_scr(const Buf& b, double y, uint32_t ve, uint32_t se) {
    if constexpr (W::SB == 4) b.st32((uint32_t)W::to_s(y), ve * 4u, se * 4u);
    else b.st64(__builtin_bit_cast(uint64_t, y), ve * 8u, se * 8u);
}

// Shared-memory layout of a four-step workgroup: the pass exchange buffer and
// the per-pass twiddle tables of the column (length B) and row (length A)
// transforms.  Only forward tables: every inverse transform runs as the
// forward transform with its output index negated (x(t) = N^-1 F(X)(-t) for
// the forward transform F of Eq. 2, which is Eq. 3).  Table entries are
// (w, w/m) pairs, which save the quotient multiply of every inter-pass
// twiddle, unless the pairs would push the workgroup out of two-per-CU
// residency or out of LDS; then they hold w alone and w/m is formed at use.
//
// PART selects what a kernel holds: FS_ALL (the fused kernels: both phases),
// FS_COL (the column kernels of the multi-launch four-step: the column
// exchange and table only) or FS_ROW (its row kernels: the row exchange and
// table only), so that the column kernels of the long lengths fit two
// workgroups per CU and no kernel fills a table it does not read.
constexpr int LDS_HALF_CU = 80 * 1024;
enum { FS_ALL = 0, FS_COL = 1, FS_ROW = 2 };
template <int LOGN, int PART = FS_ALL, int TT = 512>
struct FSLds {
    using G = FS<LOGN, TT>;
    static constexpr bool SAME = (G::A == G::Bn);
    static constexpr int TC = PassTab<G::Bn>::SIZE;   // entries per column table
    static constexpr int TR = PassTab<G::A>::SIZE;    // entries per row table
    static constexpr int XCHP = PART == FS_COL   ? G::BC::LDS_DOUBLES
                                : PART == FS_ROW ? G::mx(G::BR::LDS_DOUBLES, G::BRS::LDS_DOUBLES)
                                                 : G::XCH;
    static constexpr int XCH2 = (XCHP + 1) & ~1;       // tables start 16-byte aligned
    static constexpr bool HASC = PART != FS_ROW, HASR = PART != FS_COL && (PART == FS_ROW || !SAME);
    static constexpr int ENTRIES = (HASC ? TC : 0) + (HASR ? TR : 0);
    static constexpr int BYTES1 = 8 * (XCH2 + ENTRIES);
    static constexpr int BYTES2 = 8 * (XCH2 + 2 * ENTRIES);
    static constexpr bool PAIRS = BYTES2 <= LDS_HALF_CU || (BYTES1 > LDS_HALF_CU && BYTES2 <= 150 * 1024);
    using Entry = typename std::conditional<PAIRS, double2, double>::type;
    static constexpr int WORDS = PAIRS ? BYTES2 / 8 : BYTES1 / 8;
    double* xch;
    const Entry* colf;
    const Entry* rowf;
};


// Where the exchange buffer and the twiddle tables sit in `lds`.
template <int LOGN, int PART = FS_ALL, int TT = 512>
__device__ __forceinline__ FSLds<LOGN, PART, TT> fs_lds_layout(double* lds) {
    using FL = FSLds<LOGN, PART, TT>;
    FL L;
    L.xch = lds;
    typename FL::Entry* t = reinterpret_cast<typename FL::Entry*>(lds + FL::XCH2);
    L.colf = FL::HASC ? t : nullptr;
    L.rowf = PART == FS_ROW ? t : (PART == FS_COL ? nullptr : (FL::SAME ? t : t + FL::TC));
    return L;
}

// Fills the twiddle tables of plan p; ends with a barrier.
template <int LOGN, int PART, int TT>
__device__ __forceinline__ void fs_lds_fill(const FSLds<LOGN, PART, TT>& L, const DevPlan& p) {
    using G = FS<LOGN, TT>;
    using FL = FSLds<LOGN, PART, TT>;
    using E = typename FL::Entry;
    if constexpr (FL::HASC) fill_pass_tab<G::Bn>(const_cast<E*>(L.colf), p, LOGN);
    if constexpr (FL::HASR) fill_pass_tab<G::A>(const_cast<E*>(L.rowf), p, LOGN);
    __syncthreads();
}

template <int LOGN, int PART = FS_ALL, int TT = 512>
__device__ __forceinline__ FSLds<LOGN, PART, TT> fs_lds_init(double* lds, const DevPlan& p) {
    const FSLds<LOGN, PART, TT> L = fs_lds_layout<LOGN, PART, TT>(lds);
    fs_lds_fill<LOGN>(L, p);
    return L;
}


// Column phase, forward: length-B transforms of columns c0..c0+SC of x
// (natural order, any 32-bit values), times w^(t1 u2), into scratch rows.
// Positions of a work item are j + const(i), so every access is a buffer
// access with one per-lane offset and a compile-time uniform offset.
template <class W, int LOGN, int TT = 512>
struct ColIn {
    typename W::word w[FS<LOGN, TT>::BC::E];
};

// Raw loads of a forward column block (issued ahead of its transform).
// Positions of a work item are j + const(i), so every access is a buffer
// access with one per-lane offset and a compile-time uniform offset.
template <class W, int LOGN, int TT = 512>
__device__ __forceinline__ ColIn<W, LOGN, TT> col_fwd_load(const typename W::word* x, int c0) {
    using G = FS<LOGN, TT>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const Buf bx(x, G::N * W::WB);
    ColIn<W, LOGN, TT> in;
#pragma unroll
    for (int i = 0; i < B::E; ++i) in.w[i] = ld_word_s<W>(bx, c0 + s + G::A * j, G::A * B::pos0(0, i));
    return in;
}

// Column phase, forward: length-B transforms of columns c0..c0+SC of x
// (natural order), times w^(t1 u2), into scratch rows Y[u2 * A + t1].
template <class W, int LOGN, int PART, int TT>
__device__ __forceinline__ void col_fwd_compute(const ColIn<W, LOGN, TT>& in, typename W::sword* Y, int c0,
                                                const DevPlan& p, const FSLds<LOGN, PART, TT>& L) {
    using G = FS<LOGN, TT>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int t1 = c0 + s;
    const Buf by(Y, G::N * W::SB), bt = Tw4<W>::buf(p, G::N);
    double v[B::E];
    // four-step twiddles, loaded ahead of the transform
    typename Tw4<W>::T tw4[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) tw4[i] = Tw4<W>::ld(bt, j * G::A + t1, B::posL(0, i) * G::A);
    load_pass0<W, B::E>(v, in.w, M);
    block_dft_tw<W, G::Bn, G::SC, SEQ_FAST, false>(v, L.xch, s, j, p.P, G::la, G::N - 1, M,
                                                   twtab<W, G::Bn>(L.colf, M));
#pragma unroll
    for (int i = 0; i < B::E; ++i)
        st_scr<W>(by, W::mul_w(v[i], (double)tw4[i], M), j * G::A + t1, B::posL(0, i) * G::A);
}

template <class W, int LOGN, int PART, int TT>
__device__ __forceinline__ void col_fwd_block(const typename W::word* x, typename W::sword* Y, int c0,
                                              const DevPlan& p, const FSLds<LOGN, PART, TT>& L) {
    col_fwd_compute<W, LOGN>(col_fwd_load<W, LOGN, TT>(x, c0), Y, c0, p, L);
}

// Where the row phases of the inverse store: row position s1 of row u2 goes to
// scratch column (s1 - 1) mod A, so that the inverse column phase, which needs
// column -d mod A for destination column d, finds it at A - 1 - d and reads
// whole cache lines (see col_inv_src).  Positions s1 = j + posL(0, i) with
// posL(0, i) = i A / 16: registers i >= 1 keep the per-lane offset u2 A + j and
// take the uniform offset posL(0, i) - 1; register 0 takes the per-lane offset
// below (lane j = 0, position 0, goes to the row's last column).  No offset is
// negative, so the buffer's range check drops nothing.
template <int LOGN>
__device__ __forceinline__ uint32_t scr_row_shift(int u2, int j) {
    using G = FS<LOGN>;
    return (uint32_t)(u2 * G::A + (j == 0 ? G::A : j) - 1);
}

// Row phase of a convolution: for rows r0..r0+SR, forward(f row), forward(g
// row), product with N^-1, then the first half of the inverse four-step as a
// forward one (row transforms, times w^(t1 u2)), back into Yf; the inverse
// column phase negates the output index.
template <class W, int LOGN, int TT = 512>
struct RowIn {
    typename W::sword f[FS<LOGN, TT>::BR::E];
    typename W::sword g[FS<LOGN, TT>::BR::E];
};

template <class W, int LOGN, int TT = 512>
__device__ __forceinline__ RowIn<W, LOGN, TT> row_conv_load(const typename W::sword* Yf, const typename W::sword* Yg,
                                                        int r0) {
    using G = FS<LOGN, TT>;
    using B = typename G::BR;
    int s, j;
    B::item(threadIdx.x, s, j);
    const Buf bf(Yf, G::N * W::SB), bg(Yg, G::N * W::SB);
    const uint32_t rowoff = (uint32_t)((r0 + s) * G::A + j);
    RowIn<W, LOGN, TT> in;
#pragma unroll
    for (int i = 0; i < B::E; ++i) in.f[i] = ld_scr_raw<W>(bf, rowoff, B::pos0(0, i));
#pragma unroll
    for (int i = 0; i < B::E; ++i) in.g[i] = ld_scr_raw<W>(bg, rowoff, B::pos0(0, i));
    return in;
}

// LOCKSTEP transforms the f and g rows pass by pass together (more
// independent work around each exchange, about 2% faster at 2^17..2^19, but
// about 32 more VGPRs); the kernels limited to 128 VGPRs take them one after
// the other.
template <class W, int LOGN, int OP = OP_MUL, bool LOCKSTEP = true, int PART = FS_ALL, int TT = 512>
__device__ __forceinline__ void row_conv_compute(const RowIn<W, LOGN, TT>& in, typename W::sword* Yf, int r0,
                                                 const DevPlan& p, const FSLds<LOGN, PART, TT>& L,
                                                 uint32_t* singular = nullptr) {
    using G = FS<LOGN, TT>;
    using B = typename G::BR;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int u2 = r0 + s;
    const Buf bf(Yf, G::N * W::SB), bt = Tw4<W>::buf(p, G::N);
    const uint32_t rowoff = (uint32_t)(u2 * G::A + j);
    double F[B::E], v[B::E];
    if constexpr (LOCKSTEP) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) F[i] = W::from_s(in.f[i]);
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = W::from_s(in.g[i]);
        block_dft2_tw<W, G::A, G::SR, POS_FAST, false>(F, v, L.xch, s, j, p.P, G::lb, G::N - 1, M,
                                                       twtab<W, G::A>(L.rowf, M));
    } else {
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = W::from_s(in.f[i]);
        block_dft_tw<W, G::A, G::SR, POS_FAST, false>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M,
                                                      twtab<W, G::A>(L.rowf, M));
#pragma unroll
        for (int i = 0; i < B::E; ++i) F[i] = v[i];
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = W::from_s(in.g[i]);
        block_dft_tw<W, G::A, G::SR, POS_FAST, false>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M,
                                                      twtab<W, G::A>(L.rowf, M));
    }
    if constexpr (OP == OP_MUL) {   // (kept inline: the product path's register allocation)
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = spectral<W, OP_MUL>(F[i], v[i], p, M, singular);
    } else {
        spectral_block<W, OP, B::E>(F, v, p, M, singular);
    }
    if (B::R0 != B::RL) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) L.xch[B::lds(s, B::posL(j, i))] = v[i];
        xch_sync<B::WAVE_LOCAL>();
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = L.xch[B::lds(s, B::pos0(j, i))];
        xch_sync<B::WAVE_LOCAL>();
    }
    typename Tw4<W>::T tw4[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) tw4[i] = Tw4<W>::ld(bt, rowoff, B::posL(0, i));
    // the inverse rows: forward transforms (the output index is negated by the
    // inverse column phase), then the twiddle w^(u2 s1) of the forward four-step
    block_dft_tw<W, G::A, G::SR, POS_FAST, false>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M,
                                                  twtab<W, G::A>(L.rowf, M));
    // scratch column (s1 - 1) mod A for row position s1 (scr_row_shift)
    st_scr<W>(bf, W::mul_w(v[0], (double)tw4[0], M), scr_row_shift<LOGN>(u2, j), 0u);
#pragma unroll
    for (int i = 1; i < B::E; ++i) st_scr<W>(bf, W::mul_w(v[i], (double)tw4[i], M), rowoff, B::posL(0, i) - 1);
}

template <class W, int LOGN, int OP = OP_MUL, bool LOCKSTEP = true, int PART = FS_ALL, int TT = 512>
__device__ __forceinline__ void row_conv_block(typename W::sword* Yf, const typename W::sword* Yg, int r0,
                                               const DevPlan& p, const FSLds<LOGN, PART, TT>& L,
                                               uint32_t* singular = nullptr) {
    row_conv_compute<W, LOGN, OP, LOCKSTEP>(row_conv_load<W, LOGN, TT>(Yf, Yg, r0), Yf, r0, p, L, singular);
}

// Column phase, inverse: length-B transforms of scratch columns, optional
// N^-1, canonical store.  Each transform is the forward one and its output
// index is negated (Eq. 3 as the forward transform of Eq. 2 read at -t), so
// the block that stores destination columns c0 .. c0 + SC - 1 transforms the
// columns t1 = -(c0 + s) mod A.  The row phases store column t1 at scratch
// position (t1 - 1) mod A (scr_row_shift), so those columns sit at positions
// A - 1 - (c0 + s): the SC positions ending at A - 1 - c0, one whole block of
// cache lines, read in ascending order.
template <class W, int LOGN, int TT = 512>
struct ColInvIn {
    typename W::sword w[FS<LOGN, TT>::BC::E];
};

template <int LOGN, int TT = 512>
__device__ __forceinline__ uint32_t col_inv_src(int c0, int s) {
    using G = FS<LOGN, TT>;
    return (uint32_t)(G::A - c0 - G::SC + s);
}

template <class W, int LOGN, int TT = 512>
__device__ __forceinline__ ColInvIn<W, LOGN, TT> col_inv_load(const typename W::sword* Y, int c0) {
    using G = FS<LOGN, TT>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const Buf by(Y, G::N * W::SB);
    const uint32_t off = (uint32_t)(j * G::A) + col_inv_src<LOGN, TT>(c0, s);
    ColInvIn<W, LOGN, TT> in;
#pragma unroll
    for (int i = 0; i < B::E; ++i) in.w[i] = ld_scr_raw<W>(by, off, B::pos0(0, i) * G::A);
    return in;
}

// Where the inverse column phase stores.  The transform of the block's last
// exchange reverses the sequences (block_dft_tw's REVS), so work item s ends
// with the transform of source column t1 = -(c0 + s) mod A, whose elements
// t = t1 + A t2 (t2 = j + posL(0, i)) belong at -t mod N: destination column
// c0 + s, ascending with s, so that every store of a block fills whole cache
// lines.  For t1 != 0 the destination row is B - 1 - t2; since posL(0, i) =
// i B / 16, that is (W - 1 - j) + posL(0, 15 - i): register i goes where
// register 15 - i of lane (c0 + s, W - 1 - j) would, so one per-lane offset and
// the reversed register order give every address.  Column 0 (c0 = s = 0) maps
// to rows B - t2 mod B, one row further; its element t = 0 stays at 0 (stored
// by the item with j = 0 on its own).
template <int LOGN>
struct NegStore {
    uint32_t lane;   // per-lane element offset
    bool zero;       // the lane holding t = 0 (its register 0)
    __device__ __forceinline__ NegStore(int c0, int s, int j) {
        using G = FS<LOGN>;
        using B = typename G::BC;
        static_assert(B::E == 16 && B::NP > 1, "negated store: radix-16 column passes");
        const uint32_t d = (uint32_t)(c0 + s);   // destination column
        const uint32_t jr = (uint32_t)(B::W - 1 - j) + (d == 0 ? 1u : 0u);
        lane = d + G::A * jr;
        zero = d == 0 && j == 0;
    }
    // uniform element offset of register i
    __device__ static constexpr uint32_t reg(int i) { return FS<LOGN>::A * FS<LOGN>::BC::posL(0, 15 - i); }
};

template <class W, int LOGN, bool SCALE, bool CRT = false, int PART = FS_ALL, int TT = 512>
__device__ __forceinline__ void col_inv_compute(const ColInvIn<W, LOGN, TT>& in, typename W::word* x, int c0,
                                                const DevPlan& p, const FSLds<LOGN, PART, TT>& L,
                                                const CrtStore& crt = CrtStore{}) {
    using G = FS<LOGN, TT>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const NegStore<LOGN> ns(c0, s, j);
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = W::from_s(in.w[i]);
    // the first residues (at the output positions), loaded ahead of the
    // transform that hides their latency; lane t = 0's register 0 (beyond the
    // buffer at the negated offset, so read as 0) reloaded from position 0
    uint32_t a1v[CRT ? B::E : 1];
    if constexpr (CRT) {
        const Buf ba(crt.a1, G::N * 4u);
#pragma unroll
        for (int i = 0; i < B::E; ++i) a1v[i] = ba.ld32s(ns.lane * 4u, NegStore<LOGN>::reg(i) * 4u);
        if (ns.zero) a1v[0] = ba.ld32s(0u, 0u);
    }
    block_dft_tw<W, G::Bn, G::SC, SEQ_FAST, false, true>(v, L.xch, s, j, p.P, G::la, G::N - 1, M,
                                                            twtab<W, G::Bn>(L.colf, M));
    if constexpr (!CRT) {
        const Buf bx(x, G::N * W::WB);
        typename W::word out[B::E];
#pragma unroll
        for (int i = 0; i < B::E; ++i) {
            const double y = SCALE ? W::mul_tw(v[i], make_double2(p.ninv, p.ninvq), M) : v[i];
            out[i] = W::canon(y, M);
            st_word_s<W>(bx, out[i], ns.lane, NegStore<LOGN>::reg(i));   // lane t = 0: dropped (beyond the buffer)
        }
        if (ns.zero) st_word_s<W>(bx, out[0], 0u, 0u);
    } else {
        // y is this element mod m2 (= M.m) and a1 its residue mod m1: the
        // integer in [0, m1 m2) with both residues is a1 + m1 t,
        // t = ((y - a1) m1^-1) mod m2 (every product below 2^47)
        const Buf bh(crt.h, G::N * 8u);
        const double c = (double)crt.c;
        uint64_t out[B::E];
#pragma unroll
        for (int i = 0; i < B::E; ++i) {
            const uint32_t a1 = a1v[i];
            const double y = SCALE ? W::mul_tw(v[i], make_double2(p.ninv, p.ninvq), M) : v[i];
            const double d = reduce(y - (double)a1, M);
            double t = mulmod_var(d, c, M);
            t = (t < 0.0) ? t + M.m : t;
            t = (t >= M.m) ? t - M.m : t;
            out[i] = (uint64_t)a1 + (uint64_t)crt.m1 * (uint64_t)t;
            bh.st64(out[i], ns.lane * 8u, NegStore<LOGN>::reg(i) * 8u);
        }
        if (ns.zero) bh.st64(out[0], 0u, 0u);
    }
}

template <class W, int LOGN, bool SCALE, int PART, int TT>
__device__ __forceinline__ void col_inv_block(const typename W::sword* Y, typename W::word* x, int c0,
                                              const DevPlan& p, const FSLds<LOGN, PART, TT>& L) {
    col_inv_compute<W, LOGN, SCALE>(col_inv_load<W, LOGN, TT>(Y, c0), x, c0, p, L);
}

// Row phase of the natural-order forward transform: X[u2 + B u1].
template <class W, int LOGN, int PART, int TT>
__device__ __forceinline__ void row_fwd_nat_block(const typename W::sword* Y, typename W::word* X, int r0,
                                                  const DevPlan& p, const FSLds<LOGN, PART, TT>& L) {
    using G = FS<LOGN, TT>;
    using B = typename G::BRS;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int u2 = r0 + s;
    const Buf by(Y, G::N * W::SB), bx(X, G::N * W::WB);
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = ld_scr<W>(by, u2 * G::A + j, B::pos0(0, i));
    block_dft_tw<W, G::A, G::SR, SEQ_FAST, false>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M,
                                                  twtab<W, G::A>(L.rowf, M));
#pragma unroll
    for (int i = 0; i < B::E; ++i) st_word<W>(bx, W::canon(v[i], M), u2 + G::Bn * j, G::Bn * B::posL(0, i));
}

// Row phase of the natural-order inverse transform: from X[u2 + B u1] to
// scratch rows: forward row transforms times w^(u2 s1) (the inverse column
// phase negates the output index).
template <class W, int LOGN, int PART, int TT>
__device__ __forceinline__ void row_inv_nat_block(const typename W::word* X, typename W::sword* Y, int r0,
                                                  const DevPlan& p, const FSLds<LOGN, PART, TT>& L) {
    using G = FS<LOGN, TT>;
    using B = typename G::BRS;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int u2 = r0 + s;
    const Buf bx(X, G::N * W::WB), by(Y, G::N * W::SB), bt = Tw4<W>::buf(p, G::N);
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = W::load_reduce(ld_word<W>(bx, u2 + G::Bn * j, G::Bn * B::pos0(0, i)), M);
    typename Tw4<W>::T tw4[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) tw4[i] = Tw4<W>::ld(bt, u2 * G::A + j, B::posL(0, i));
    block_dft_tw<W, G::A, G::SR, SEQ_FAST, false>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M,
                                                  twtab<W, G::A>(L.rowf, M));
    st_scr<W>(by, W::mul_w(v[0], (double)tw4[0], M), scr_row_shift<LOGN>(u2, j), 0u);
#pragma unroll
    for (int i = 1; i < B::E; ++i)
        st_scr<W>(by, W::mul_w(v[i], (double)tw4[i], M), u2 * G::A + j, B::posL(0, i) - 1);
}

// Kernels of the multi-launch four-step (grid.y = item / row of the batch).
// For rows of 2^FS_ROW_LOOP_CONV positions and more (the convolution's row
// kernel; 2^FS_ROW_LOOP_NAT for the natural-order transforms) the row kernels
// take row blocks blockIdx.x, blockIdx.x + gridDim.x, ... of their item, so
// that a grid narrower than the item's row blocks fills each workgroup's
// twiddle table once for several blocks.  Shorter rows take one block per
// workgroup, the loop's step then a compile-time constant.  Measured against
// one block per workgroup: convolution rows of 512, 1024, 2048 9%, 3%, 8%
// faster; transform rows of 2048 10-17% faster, of 512 and 1024 2-14% slower;
// a grid-strided loop at rows of 256 7% slower.
constexpr int FS_ROW_LOOP_CONV = 9, FS_ROW_LOOP_NAT = 11;
template <class W, int LOGN, int TT>
__global__ __launch_bounds__(TT) void k_fs_col_fwd(const typename W::word* x, typename W::sword* Y,
                                                    uint64_t item_stride, uint64_t ystride, DevPlan p) {
    __shared__ double lds[FSLds<LOGN, FS_COL, TT>::WORDS];
    const FSLds<LOGN, FS_COL, TT> L = fs_lds_init<LOGN, FS_COL, TT>(lds, p);
    col_fwd_block<W, LOGN>(x + blockIdx.y * item_stride, Y + blockIdx.y * ystride, blockIdx.x * FS<LOGN, TT>::SC, p, L);
}
// Column phase of both operands in one launch: grid.y = 2 * items, the first
// half f (into Y_f), the second g (into Y_g = Y_f + N).
template <class W, int LOGN, int TT>
__global__ __launch_bounds__(TT) void k_fs_col_fwd2(const typename W::word* f, const typename W::word* g,
                                                     typename W::sword* Y, uint64_t item_stride, uint64_t ystride,
                                                     uint32_t items, DevPlan p) {
    __shared__ double lds[FSLds<LOGN, FS_COL, TT>::WORDS];
    const FSLds<LOGN, FS_COL, TT> L = fs_lds_init<LOGN, FS_COL, TT>(lds, p);
    const uint32_t second = blockIdx.y >= items ? 1u : 0u;
    const uint32_t item = blockIdx.y - second * items;
    col_fwd_block<W, LOGN>((second ? g : f) + item * item_stride, Y + item * ystride + second * FS<LOGN, TT>::N,
                           blockIdx.x * FS<LOGN, TT>::SC, p, L);
}
template <class W, int LOGN, int OP, int TT>
__global__ __launch_bounds__(TT) void k_fs_row_conv(typename W::sword* Yf, const typename W::sword* Yg,
                                                     uint64_t ystride, DevPlan p, uint32_t* singular) {
    __shared__ double lds[FSLds<LOGN, FS_ROW, TT>::WORDS];
    const FSLds<LOGN, FS_ROW, TT> L = fs_lds_init<LOGN, FS_ROW, TT>(lds, p);
    const uint32_t bstep = FS<LOGN, TT>::la >= FS_ROW_LOOP_CONV ? gridDim.x : FS<LOGN, TT>::Bn / FS<LOGN, TT>::SR;
    for (uint32_t b = blockIdx.x; b < (uint32_t)(FS<LOGN, TT>::Bn / FS<LOGN, TT>::SR); b += bstep)
        row_conv_block<W, LOGN, OP>(Yf + blockIdx.y * ystride, Yg + blockIdx.y * ystride, (int)b * FS<LOGN, TT>::SR, p,
                                    L, singular);
}
template <class W, int LOGN, bool SCALE, int TT>
__global__ __launch_bounds__(TT) void k_fs_col_inv(const typename W::sword* Y, typename W::word* x,
                                                    uint64_t item_stride, uint64_t ystride, DevPlan p) {
    __shared__ double lds[FSLds<LOGN, FS_COL, TT>::WORDS];
    const FSLds<LOGN, FS_COL, TT> L = fs_lds_init<LOGN, FS_COL, TT>(lds, p);
    col_inv_block<W, LOGN, SCALE>(Y + blockIdx.y * ystride, x + blockIdx.y * item_stride, blockIdx.x * FS<LOGN, TT>::SC,
                                  p, L);
}
template <class W, int LOGN, int TT>
__global__ __launch_bounds__(TT) void k_fs_row_fwd_nat(const typename W::sword* Y, typename W::word* X,
                                                        uint64_t item_stride, uint64_t ystride, DevPlan p) {
    __shared__ double lds[FSLds<LOGN, FS_ROW, TT>::WORDS];
    const FSLds<LOGN, FS_ROW, TT> L = fs_lds_init<LOGN, FS_ROW, TT>(lds, p);
    const uint32_t bstep = FS<LOGN, TT>::la >= FS_ROW_LOOP_NAT ? gridDim.x : FS<LOGN, TT>::Bn / FS<LOGN, TT>::SR;
    for (uint32_t b = blockIdx.x; b < (uint32_t)(FS<LOGN, TT>::Bn / FS<LOGN, TT>::SR); b += bstep)
        row_fwd_nat_block<W, LOGN>(Y + blockIdx.y * ystride, X + blockIdx.y * item_stride, (int)b * FS<LOGN, TT>::SR, p,
                                   L);
}
template <class W, int LOGN, int TT>
__global__ __launch_bounds__(TT) void k_fs_row_inv_nat(const typename W::word* X, typename W::sword* Y,
                                                        uint64_t item_stride, uint64_t ystride, DevPlan p) {
    __shared__ double lds[FSLds<LOGN, FS_ROW, TT>::WORDS];
    const FSLds<LOGN, FS_ROW, TT> L = fs_lds_init<LOGN, FS_ROW, TT>(lds, p);
    const uint32_t bstep = FS<LOGN, TT>::la >= FS_ROW_LOOP_NAT ? gridDim.x : FS<LOGN, TT>::Bn / FS<LOGN, TT>::SR;
    for (uint32_t b = blockIdx.x; b < (uint32_t)(FS<LOGN, TT>::Bn / FS<LOGN, TT>::SR); b += bstep)
        row_inv_nat_block<W, LOGN>(X + blockIdx.y * item_stride, Y + blockIdx.y * ystride, (int)b * FS<LOGN, TT>::SR, p,
                                   L);
}

// Residency of the persistent fused kernel.  Where the LDS (<= 80 KB) and
// register (<= 128 VGPRs) budgets allow, two workgroups share a CU and hide
// each other's memory and barrier latency; otherwise one workgroup per CU
// issues the next block's loads before transforming the current block.
template <class W, int LOGN, int OP = OP_MUL>
struct FusedCfg {
    // (the deconvolution's simultaneous inversion needs more registers)
    static constexpr bool TWO = (W::WB == 4) && LOGN >= 13 && LOGN <= 16 && OP != OP_DIV;
    // minimum waves per SIMD (the second __launch_bounds__ argument): four
    // for two 512-thread workgroups per CU, i.e. at most 128 VGPRs
    static constexpr int WAVES_PER_EU = TWO ? 4 : 2;
    // phases with software prefetch (fused_conv_item): all of them at one
    // workgroup per CU
    static constexpr int PF = TWO ? 0 : 15;
};

// Work queue of a persistent launch: q[0] is the next item, q[1] counts the
// workgroups that have left.  Both are zero when a launch starts; the last
// workgroup to leave zeroes them again for the next launch on the stream.
__device__ __forceinline__ uint32_t queue_take(uint32_t* q, uint32_t* slot) {
    __syncthreads();   // every thread has read the previous ticket
    if (threadIdx.x == 0) *slot = atomicAdd(&q[0], 1u);
    __syncthreads();
    return *slot;
}
__device__ __forceinline__ void queue_leave(uint32_t* q) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&q[1], 1u) == gridDim.x - 1) {
            __threadfence();
            atomicExch(&q[0], 0u);
            atomicExch(&q[1], 0u);
        }
    }
}

// One convolution of length 2^LOGN by the four-step path, start to finish, in
// one workgroup: columns of f and of g into the scratch Yf, Yg (N words each),
// rows (forward f, forward g, product with N^-1, inverse) back into Yf, then
// the inverse columns into h.  PF selects the phases whose blocks issue their
// loads before the previous block is transformed (software prefetch into
// registers): bit 0 the forward columns, bit 1 the rows, bit 2 the inverse
// columns; bit 3 transforms the f and g rows pass by pass together
// (row_conv_compute's LOCKSTEP).  Ends with a barrier.
template <class W, int LOGN, int PF, int OP = OP_MUL, int PART = FS_ALL>
__device__ __forceinline__ void fused_conv_item(const typename W::word* fi, const typename W::word* gi,
                                                typename W::word* hi, typename W::sword* Yf,
                                                typename W::sword* Yg, const DevPlan& p, const FSLds<LOGN, PART>& L,
                                                uint32_t* singular = nullptr, const CrtStore& crt = CrtStore{}) {
    using G = FS<LOGN>;
    constexpr int CL = G::A - G::SC;
    constexpr int SOP = OP == OP_DIV ? OP_DIV : OP_MUL;   // the pointwise step
    constexpr bool CRT = OP == OP_CRT;                    // the final store
    if constexpr (!(PF & 1)) {
        for (int c0 = 0; c0 < G::A; c0 += G::SC) col_fwd_block<W, LOGN>(fi, Yf, c0, p, L);
        for (int c0 = 0; c0 < G::A; c0 += G::SC) col_fwd_block<W, LOGN>(gi, Yg, c0, p, L);
    } else {
        ColIn<W, LOGN> cin = col_fwd_load<W, LOGN>(fi, 0);
        for (int c0 = 0; c0 < CL; c0 += G::SC) {
            const ColIn<W, LOGN> nxt = col_fwd_load<W, LOGN>(fi, c0 + G::SC);
            col_fwd_compute<W, LOGN>(cin, Yf, c0, p, L);
            cin = nxt;
        }
        {
            const ColIn<W, LOGN> nxt = col_fwd_load<W, LOGN>(gi, 0);
            col_fwd_compute<W, LOGN>(cin, Yf, CL, p, L);
            cin = nxt;
        }
        for (int c0 = 0; c0 < CL; c0 += G::SC) {
            const ColIn<W, LOGN> nxt = col_fwd_load<W, LOGN>(gi, c0 + G::SC);
            col_fwd_compute<W, LOGN>(cin, Yg, c0, p, L);
            cin = nxt;
        }
        col_fwd_compute<W, LOGN>(cin, Yg, CL, p, L);
    }
    __syncthreads();
    if constexpr (!(PF & 2)) {
        for (int r0 = 0; r0 < G::Bn; r0 += G::SR)
            row_conv_block<W, LOGN, SOP, (PF & 8) != 0>(Yf, Yg, r0, p, L, singular);
    } else {
        RowIn<W, LOGN> rin = row_conv_load<W, LOGN>(Yf, Yg, 0);
        for (int r0 = 0; r0 < G::Bn - G::SR; r0 += G::SR) {
            const RowIn<W, LOGN> nxt = row_conv_load<W, LOGN>(Yf, Yg, r0 + G::SR);
            row_conv_compute<W, LOGN, SOP, (PF & 8) != 0>(rin, Yf, r0, p, L, singular);
            rin = nxt;
        }
        row_conv_compute<W, LOGN, SOP, (PF & 8) != 0>(rin, Yf, G::Bn - G::SR, p, L, singular);
    }
    __syncthreads();
    if constexpr (!(PF & 4)) {
        for (int c0 = 0; c0 < G::A; c0 += G::SC)
            col_inv_compute<W, LOGN, false, CRT>(col_inv_load<W, LOGN>(Yf, c0), hi, c0, p, L, crt);
    } else {
        ColInvIn<W, LOGN> iin = col_inv_load<W, LOGN>(Yf, 0);
        for (int c0 = 0; c0 < CL; c0 += G::SC) {
            const ColInvIn<W, LOGN> nxt = col_inv_load<W, LOGN>(Yf, c0 + G::SC);
            col_inv_compute<W, LOGN, false, CRT>(iin, hi, c0, p, L, crt);
            iin = nxt;
        }
        col_inv_compute<W, LOGN, false, CRT>(iin, hi, CL, p, L, crt);
    }
    __syncthreads();
}

// Persistent fused convolution of a uniform-length batch: one workgroup owns
// one convolution at a time, start to finish, with a private 2N-word scratch,
// and takes its next convolution from the work queue (workgroups that share a
// CU do not progress at the same rate).
template <class W, int LOGN, int OP = OP_MUL>
__global__ __launch_bounds__(512, (FusedCfg<W, LOGN, OP>::WAVES_PER_EU)) void k_conv_fused(
    const typename W::word* f, const typename W::word* g, typename W::word* h, const uint64_t* __restrict__ offs,
    uint32_t count, typename W::sword* scratch, uint32_t* queue, DevPlan p, uint32_t* singular, CrtStore crt) {
    using G = FS<LOGN>;
    __shared__ double lds[FSLds<LOGN>::WORDS];
    __shared__ uint32_t ticket;
    const FSLds<LOGN> L = fs_lds_init<LOGN>(lds, p);
    typename W::sword* Yf = scratch + (size_t)blockIdx.x * 2 * G::N;
    typename W::sword* Yg = Yf + G::N;
    for (;;) {
        const uint32_t item = queue_take(queue, &ticket);
        if (item >= count) break;
        const uint64_t off = offs ? offs[item] : (uint64_t)item * G::N;
        CrtStore ci = crt;
        if constexpr (OP == OP_CRT) {
            ci.a1 += off;
            ci.h += off;
        }
        fused_conv_item<W, LOGN, FusedCfg<W, LOGN, OP>::PF, OP>(f + off, g + off, h + off, Yf, Yg, p, L, singular,
                                                                ci);
    }
    queue_leave(queue);
}

// ------------------------------------------------------------------ one launch, many lengths
// Persistent convolution of a batch of uneven lengths 2^0 .. 2^NMAX in one
// launch.  The host lists tasks longest first: one task per convolution of
// length > 2^12 (the fused four-step path of fused_conv_item), one tile of up to
// multi_s(L) convolutions per task below (small_conv_tile).  Workgroups take
// tasks from the work queue, so the short tasks at the end of the list fill in
// behind the long ones.  plans[n] is the plan of length 2^n.
struct MultiTask {
    uint64_t first;   // index of the task's first item in the item-offset list
    uint32_t logn;
    uint32_t cnt;     // items in the task (1 above 2^12)
};
constexpr int multi_s(int L) { return L < 16 ? 512 : 8192 / L; }
template <class W>
struct MultiCfg {
    static constexpr int NMAX = (W::WB == 4) ? 19 : 18;
    static constexpr int mx(int a, int b) { return a > b ? a : b; }
    template <int N>
    static constexpr int large_words() {
        if constexpr (N < 13) return 1;
        else return mx(FSLds<N>::WORDS, large_words<N - 1>());
    }
    static constexpr int SMALL_WORDS = 8704;   // >= Blk<L, 8192/L, POS_FAST>::LDS_DOUBLES for 16 < L <= 4096
    static constexpr int WORDS = mx(large_words<NMAX>(), SMALL_WORDS);
};

// The LDS twiddle table of a small tile of the multi-length kernel, after the
// tile's exchange buffer in the space the long lengths size: (w, w/m) pairs
// (MODE 2) or w alone (MODE 1) as they fit, else none (MODE 0: twiddles from
// the global power table).
template <class W, int K>
struct MultiTab {
    static constexpr int L = 1 << K;
    static constexpr int OFF = (Blk<L, multi_s(L), POS_FAST>::LDS_DOUBLES + 1) & ~1;
    static constexpr int FREE = MultiCfg<W>::WORDS - OFF;
    static constexpr int TS = PassTab<L>::SIZE;
    static constexpr int MODE = !small_tab(L) ? 0 : (2 * TS <= FREE ? 2 : (TS <= FREE ? 1 : 0));
    using Entry = typename std::conditional<MODE == 2, double2, double>::type;
};

// Tasks of length 2^K, while the queue hands them out: the task list is
// sorted longest first and tickets only grow, so a workgroup meets every
// length at most once and in decreasing order.  Each length has its own loop
// (no loop around all of them), so what the compiler hoists out of one
// length's loop stays inside that length's code.  Returns the first ticket of
// a shorter length (or past the end).
template <class W, int K>
__device__ __forceinline__ uint32_t multi_run(uint32_t t, const typename W::word* f, const typename W::word* g,
                                              typename W::word* h, const MultiTask* __restrict__ tasks,
                                              uint32_t ntasks, const uint64_t* __restrict__ toffs,
                                              typename W::sword* Y, uint32_t* queue,
                                              const DevPlan* __restrict__ plans, double* lds, uint32_t* ticket) {
    if (t >= ntasks || tasks[t].logn != (uint32_t)K) return t;
    const DevPlan p = plans[K];
    if constexpr (K > SMALL_MAX_LOG2N) {
        const FSLds<K> L = fs_lds_layout<K>(lds);
        fs_lds_fill<K>(L, p);
        do {
            const uint64_t o = toffs[tasks[t].first];
            fused_conv_item<W, K, 15>(f + o, g + o, h + o, Y, Y + (1 << K), p, L);
            t = __builtin_amdgcn_readfirstlane(queue_take(queue, ticket));
        } while (t < ntasks && tasks[t].logn == (uint32_t)K);
    } else {
        constexpr int L = 1 << K, S = multi_s(L);
        using MT = MultiTab<W, K>;
        using TE = typename MT::Entry;
        TE* tab = reinterpret_cast<TE*>(lds + MT::OFF);
        if constexpr (MT::MODE != 0) {
            // the previous class's waves may still read the table region
            __syncthreads();
            fill_pass_tab<L>(tab, p, K);
            __syncthreads();
        }
        do {
            const MultiTask task = tasks[t];
            // the thread index, opaque to the compiler on every pass, so that the
            // tile's per-thread addressing is recomputed here instead of being
            // held in registers across the whole loop
            int tid = (int)threadIdx.x;
            asm volatile("" : "+v"(tid));
            small_conv_tile<W, L, S, OP_MUL, MT::MODE != 0, TE>(f, g, h, toffs + task.first, 0, task.cnt, p, lds,
                                                                tid, nullptr, tab);
            t = __builtin_amdgcn_readfirstlane(queue_take(queue, ticket));
        } while (t < ntasks && tasks[t].logn == (uint32_t)K);
    }
    return t;
}

template <class W, int K>
__device__ __forceinline__ uint32_t multi_from(uint32_t t, const typename W::word* f, const typename W::word* g,
                                               typename W::word* h, const MultiTask* __restrict__ tasks,
                                               uint32_t ntasks, const uint64_t* __restrict__ toffs,
                                               typename W::sword* Y, uint32_t* queue,
                                               const DevPlan* __restrict__ plans, double* lds, uint32_t* ticket) {
    t = multi_run<W, K>(t, f, g, h, tasks, ntasks, toffs, Y, queue, plans, lds, ticket);
    if constexpr (K > 0) return multi_from<W, K - 1>(t, f, g, h, tasks, ntasks, toffs, Y, queue, plans, lds, ticket);
    else return t;
}

template <class W>
__global__ __launch_bounds__(512, 2) void k_conv_multi(const typename W::word* f, const typename W::word* g,
                                                       typename W::word* h, const MultiTask* __restrict__ tasks,
                                                       uint32_t ntasks, const uint64_t* __restrict__ toffs,
                                                       typename W::sword* scratch, uint64_t scratch_words,
                                                       uint32_t* queue, const DevPlan* __restrict__ plans) {
    __shared__ double lds[MultiCfg<W>::WORDS];
    __shared__ uint32_t ticket;
    typename W::sword* Y = scratch + (size_t)blockIdx.x * scratch_words;
    const uint32_t t = __builtin_amdgcn_readfirstlane(queue_take(queue, &ticket));
    multi_from<W, MultiCfg<W>::NMAX>(t, f, g, h, tasks, ntasks, toffs, Y, queue, plans, lds, &ticket);
    queue_leave(queue);
}

}  // namespace nttmi
