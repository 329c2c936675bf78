// Device kernels and their launchers (gfx950).
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
#include <hip/hip_runtime.h>
#include "blockdft.hpp"
#include "launch.hpp"

namespace nttmi {

// Residency target: four waves per SIMD (<= 128 VGPRs per lane) keeps two or
// more workgroups per CU for latency hiding across barriers.
#define NTT_OCC __attribute__((amdgpu_waves_per_eu(4, 8)))

// ------------------------------------------------------------------ small N
constexpr int small_s(int L) { return L < 16 ? 256 : 4096 / L; }

template <int L>
__global__ __launch_bounds__(256) void k_conv_small(const uint32_t* f, const uint32_t* g, uint32_t* h,
                                                    const uint64_t* __restrict__ offs, uint32_t count,
                                                    DevPlan p) {
    constexpr int S = small_s(L);
    using B = Blk<L, S, POS_FAST>;
    __shared__ double lds[B::LDS_DOUBLES];
    int s, j;
    B::item(threadIdx.x, s, j);
    const uint64_t item = (uint64_t)blockIdx.x * S + s;
    const bool valid = item < count;
    const uint64_t off = valid ? (offs ? offs[item] : item * (uint64_t)L) : (offs ? offs[0] : 0);
    const ModC M = p.M;
    const int lshift = p.logn - B::l;
    double F[B::E], v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = reduce((double)f[off + B::pos0(j, i)], M);
    block_dft<L, S, POS_FAST, false>(v, lds, s, j, p.P, lshift, p.nmask, M);
#pragma unroll
    for (int i = 0; i < B::E; ++i) F[i] = v[i];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = reduce((double)g[off + B::pos0(j, i)], M);
    block_dft<L, S, POS_FAST, false>(v, lds, s, j, p.P, lshift, p.nmask, M);
    // pointwise product with N^-1 folded in: F * (G * N^-1)
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
        const double gs = mulmod(v[i], p.ninv, p.ninvq, M);
        v[i] = mulmod_var(F[i], gs, M);
    }
    if (B::R0 != B::RL) {
        // output positions of the forward transform differ from the input
        // positions of the inverse: reorder through LDS
#pragma unroll
        for (int i = 0; i < B::E; ++i) lds[B::lds(s, B::posL(j, i))] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = lds[B::lds(s, B::pos0(j, i))];
        __syncthreads();
    }
    block_dft<L, S, POS_FAST, true>(v, lds, s, j, p.P, lshift, p.nmask, M);
    if (valid) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) h[off + B::posL(j, i)] = canon_u32(v[i], M);
    }
}

template <int L, bool INV>
__global__ __launch_bounds__(256) void k_ntt_small(const uint32_t* x, uint32_t* X, uint32_t batch, DevPlan p) {
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
    for (int i = 0; i < B::E; ++i) v[i] = reduce((double)x[off + B::pos0(j, i)], M);
    block_dft<L, S, POS_FAST, INV>(v, lds, s, j, p.P, p.logn - B::l, p.nmask, M);
    if (valid) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) {
            const double y = INV ? mulmod(v[i], p.ninv, p.ninvq, M) : v[i];
            X[off + B::posL(j, i)] = canon_u32(y, M);
        }
    }
}

// ------------------------------------------------------------------ four-step
// Geometry for N = 2^LOGN = A * B, A = 2^ceil(LOGN/2) (row length),
// B = 2^floor(LOGN/2) (column length).  Element t = t1 + A t2 (t1 < A, t2 < B),
// frequency u = u2 + B u1.  Scratch rows: Y[u2 * A + t1].
template <int LOGN>
struct FS {
    static constexpr int la = (LOGN + 1) / 2, lb = LOGN / 2;
    static constexpr int A = 1 << la, Bn = 1 << lb, N = 1 << LOGN;
    // threads per workgroup: 512, so that a column block of B = 256 spans 32
    // columns (128-byte rows of a block: whole cache lines)
    static constexpr int T = 512;
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
};

// Shared-memory layout of a four-step workgroup: the pass exchange buffer and
// the per-pass twiddle tables of the column (length B) and row (length A)
// transforms, forward and inverse (w only; w/m is formed at use).
template <int LOGN>
struct FSLds {
    using G = FS<LOGN>;
    static constexpr bool SAME = (G::A == G::Bn);
    static constexpr int TC = PassTab<G::Bn>::SIZE;
    static constexpr int TR = PassTab<G::A>::SIZE;
    static constexpr int WORDS = G::XCH + 2 * TC + (SAME ? 0 : 2 * TR);
    double* xch;
    const double* colf;
    const double* coli;
    const double* rowf;
    const double* rowi;
};

template <int L, bool INV>
__device__ __forceinline__ void fill_pass_tab(double* t, const DevPlan& p, int logn) {
    using PT = PassTab<L>;
    using B = Blk<L, 1, SEQ_FAST>;
    const int lshift = logn - B::l;
    const int nmask = (1 << logn) - 1;
#pragma unroll
    for (int q = 1; q < B::NP; ++q) {
        const int cnt = 16 * PT::ns(q);
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            const int k = e >> 4, r = e & 15;
            t[PT::off(q) + k * PT::ROW + r] = p.P[tw_index<INV>(PT::expo(q, k, r), lshift, nmask)].x;
        }
    }
}

// Fills the twiddle tables; ends with a barrier.
template <int LOGN>
__device__ __forceinline__ FSLds<LOGN> fs_lds_init(double* lds, const DevPlan& p) {
    using G = FS<LOGN>;
    using FL = FSLds<LOGN>;
    FL L;
    L.xch = lds;
    double* t = lds + G::XCH;
    fill_pass_tab<G::Bn, false>(t, p, LOGN);
    fill_pass_tab<G::Bn, true>(t + FL::TC, p, LOGN);
    L.colf = t;
    L.coli = t + FL::TC;
    if (FL::SAME) {
        L.rowf = L.colf;
        L.rowi = L.coli;
    } else {
        fill_pass_tab<G::A, false>(t + 2 * FL::TC, p, LOGN);
        fill_pass_tab<G::A, true>(t + 2 * FL::TC + FL::TR, p, LOGN);
        L.rowf = t + 2 * FL::TC;
        L.rowi = t + 2 * FL::TC + FL::TR;
    }
    __syncthreads();
    return L;
}

// Inter-pass twiddles of a length-L transform from its shared pass table.
template <int L>
struct TwTab {
    const double* t;
    ModC M;
    __device__ __forceinline__ void operator()(double* v, int p, int, int k) const {
        const double* b = t + PassTab<L>::off(p) + PassTab<L>::ROW * k;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = mulmod_var(v[r], b[r], M);
    }
};

// Column phase, forward: length-B transforms of columns c0..c0+SC of x
// (natural order, any 32-bit values), times w^(t1 u2), into scratch rows.
// Positions of a work item are j + const(i), so every access is a buffer
// access with one per-lane offset and a compile-time uniform offset.
template <int LOGN>
struct ColIn {
    uint32_t w[FS<LOGN>::BC::E];
};

// Raw loads of a forward column block (issued ahead of its transform).
template <int LOGN>
__device__ __forceinline__ ColIn<LOGN> col_fwd_load(const uint32_t* x, int c0) {
    using G = FS<LOGN>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const Buf bx(x, G::N * 4u);
    ColIn<LOGN> in;
#pragma unroll
    for (int i = 0; i < B::E; ++i) in.w[i] = bx.ld32((c0 + s + G::A * j) * 4u, G::A * (B::pos0(0, i)) * 4u);
    return in;
}

template <int LOGN>
__device__ __forceinline__ void col_fwd_compute(const ColIn<LOGN>& in, int32_t* Y, int c0, const DevPlan& p,
                                                const FSLds<LOGN>& L) {
    using G = FS<LOGN>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int t1 = c0 + s;
    const Buf by(Y, G::N * 4u), bt(p.TT, G::N * 8u);
    double v[B::E];
    // four-step twiddles, loaded ahead of the transform
    double tw4[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) tw4[i] = bt.ld64f((j * G::A + t1) * 8u, B::posL(0, i) * G::A * 8u);
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = reduce((double)in.w[i], M);
    block_dft_tw<G::Bn, G::SC, SEQ_FAST, false>(v, L.xch, s, j, p.P, G::la, G::N - 1, M, TwTab<G::Bn>{L.colf, M});
#pragma unroll
    for (int i = 0; i < B::E; ++i)
        by.st32((uint32_t)to_i32(mulmod_var(v[i], tw4[i], M)), (j * G::A + t1) * 4u, B::posL(0, i) * G::A * 4u);
}

// Column phase, forward: length-B transforms of columns c0..c0+SC of x
// (natural order, any 32-bit values), times w^(t1 u2), into scratch rows.
// Positions of a work item are j + const(i), so every access is a buffer
// access with one per-lane offset and a compile-time uniform offset.
template <int LOGN>
__device__ __forceinline__ void col_fwd_block(const uint32_t* x, int32_t* Y, int c0, const DevPlan& p,
                                              const FSLds<LOGN>& L) {
    col_fwd_compute<LOGN>(col_fwd_load<LOGN>(x, c0), Y, c0, p, L);
}

// Row phase of a convolution: for rows r0..r0+SR, forward(f row), forward(g
// row), product with N^-1, inverse, times w^-(t1 u2), back into Yf.
template <int LOGN>
struct RowIn {
    int32_t f[FS<LOGN>::BR::E];
    int32_t g[FS<LOGN>::BR::E];
};

template <int LOGN>
__device__ __forceinline__ RowIn<LOGN> row_conv_load(const int32_t* Yf, const int32_t* Yg, int r0) {
    using G = FS<LOGN>;
    using B = typename G::BR;
    int s, j;
    B::item(threadIdx.x, s, j);
    const Buf bf(Yf, G::N * 4u), bg(Yg, G::N * 4u);
    const uint32_t rowoff = (uint32_t)((r0 + s) * G::A + j);
    RowIn<LOGN> in;
#pragma unroll
    for (int i = 0; i < B::E; ++i) in.f[i] = bf.ldi32(rowoff * 4u, B::pos0(0, i) * 4u);
#pragma unroll
    for (int i = 0; i < B::E; ++i) in.g[i] = bg.ldi32(rowoff * 4u, B::pos0(0, i) * 4u);
    return in;
}

template <int LOGN>
__device__ __forceinline__ void row_conv_compute(const RowIn<LOGN>& in, int32_t* Yf, int r0, const DevPlan& p,
                                                 const FSLds<LOGN>& L) {
    using G = FS<LOGN>;
    using B = typename G::BR;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int u2 = r0 + s;
    const Buf bf(Yf, G::N * 4u), bt(p.TTi, G::N * 8u);
    const uint32_t rowoff = (uint32_t)(u2 * G::A + j);
    double F[B::E], v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = from_i32(in.f[i]);
    block_dft_tw<G::A, G::SR, POS_FAST, false>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M, TwTab<G::A>{L.rowf, M});
#pragma unroll
    for (int i = 0; i < B::E; ++i) F[i] = v[i];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = from_i32(in.g[i]);
    block_dft_tw<G::A, G::SR, POS_FAST, false>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M, TwTab<G::A>{L.rowf, M});
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
        const double gs = mulmod(v[i], p.ninv, p.ninvq, M);
        v[i] = mulmod_var(F[i], gs, M);
    }
    if (B::R0 != B::RL) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) L.xch[B::lds(s, B::posL(j, i))] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = L.xch[B::lds(s, B::pos0(j, i))];
        __syncthreads();
    }
    double tw4[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) tw4[i] = bt.ld64f(rowoff * 8u, B::posL(0, i) * 8u);
    block_dft_tw<G::A, G::SR, POS_FAST, true>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M, TwTab<G::A>{L.rowi, M});
#pragma unroll
    for (int i = 0; i < B::E; ++i)
        bf.st32((uint32_t)to_i32(mulmod_var(v[i], tw4[i], M)), rowoff * 4u, B::posL(0, i) * 4u);
}

template <int LOGN>
__device__ __forceinline__ void row_conv_block(int32_t* Yf, const int32_t* Yg, int r0, const DevPlan& p,
                                               const FSLds<LOGN>& L) {
    row_conv_compute<LOGN>(row_conv_load<LOGN>(Yf, Yg, r0), Yf, r0, p, L);
}

// Column phase, inverse: length-B inverse transforms of scratch columns,
// optional N^-1, canonical store to x[t1 + A t2].
template <int LOGN>
struct ColInvIn {
    int32_t w[FS<LOGN>::BC::E];
};

template <int LOGN>
__device__ __forceinline__ ColInvIn<LOGN> col_inv_load(const int32_t* Y, int c0) {
    using G = FS<LOGN>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const Buf by(Y, G::N * 4u);
    ColInvIn<LOGN> in;
#pragma unroll
    for (int i = 0; i < B::E; ++i) in.w[i] = by.ldi32((j * G::A + c0 + s) * 4u, B::pos0(0, i) * G::A * 4u);
    return in;
}

template <int LOGN, bool SCALE>
__device__ __forceinline__ void col_inv_compute(const ColInvIn<LOGN>& in, uint32_t* x, int c0, const DevPlan& p,
                                                const FSLds<LOGN>& L) {
    using G = FS<LOGN>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const Buf bx(x, G::N * 4u);
    const uint32_t off = (uint32_t)(j * G::A + c0 + s);
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = from_i32(in.w[i]);
    block_dft_tw<G::Bn, G::SC, SEQ_FAST, true>(v, L.xch, s, j, p.P, G::la, G::N - 1, M, TwTab<G::Bn>{L.coli, M});
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
        const double y = SCALE ? mulmod(v[i], p.ninv, p.ninvq, M) : v[i];
        bx.st32(canon_u32(y, M), off * 4u, B::posL(0, i) * G::A * 4u);
    }
}

template <int LOGN, bool SCALE>
__device__ __forceinline__ void col_inv_block(const int32_t* Y, uint32_t* x, int c0, const DevPlan& p,
                                              const FSLds<LOGN>& L) {
    col_inv_compute<LOGN, SCALE>(col_inv_load<LOGN>(Y, c0), x, c0, p, L);
}

// Row phase of the natural-order forward transform: X[u2 + B u1].
template <int LOGN>
__device__ __forceinline__ void row_fwd_nat_block(const int32_t* Y, uint32_t* X, int r0, const DevPlan& p,
                                                  const FSLds<LOGN>& L) {
    using G = FS<LOGN>;
    using B = typename G::BRS;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int u2 = r0 + s;
    const Buf by(Y, G::N * 4u), bx(X, G::N * 4u);
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = from_i32(by.ldi32((u2 * G::A + j) * 4u, B::pos0(0, i) * 4u));
    block_dft_tw<G::A, G::SR, SEQ_FAST, false>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M, TwTab<G::A>{L.rowf, M});
#pragma unroll
    for (int i = 0; i < B::E; ++i) bx.st32(canon_u32(v[i], M), (u2 + G::Bn * j) * 4u, G::Bn * B::posL(0, i) * 4u);
}

// Row phase of the natural-order inverse transform: from X[u2 + B u1] to
// scratch rows, times w^-(t1 u2).
template <int LOGN>
__device__ __forceinline__ void row_inv_nat_block(const uint32_t* X, int32_t* Y, int r0, const DevPlan& p,
                                                  const FSLds<LOGN>& L) {
    using G = FS<LOGN>;
    using B = typename G::BRS;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int u2 = r0 + s;
    const Buf bx(X, G::N * 4u), by(Y, G::N * 4u), bt(p.TTi, G::N * 8u);
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = reduce((double)bx.ld32((u2 + G::Bn * j) * 4u, G::Bn * B::pos0(0, i) * 4u), M);
    double tw4[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) tw4[i] = bt.ld64f((u2 * G::A + j) * 8u, B::posL(0, i) * 8u);
    block_dft_tw<G::A, G::SR, SEQ_FAST, true>(v, L.xch, s, j, p.P, G::lb, G::N - 1, M, TwTab<G::A>{L.rowi, M});
#pragma unroll
    for (int i = 0; i < B::E; ++i)
        by.st32((uint32_t)to_i32(mulmod_var(v[i], tw4[i], M)), (u2 * G::A + j) * 4u, B::posL(0, i) * 4u);
}

// Kernels of the multi-launch four-step (grid.y = item / row of the batch).
template <int LOGN>
__global__ __launch_bounds__(512) void k_fs_col_fwd(const uint32_t* x, int32_t* Y, uint64_t item_stride,
                                                    uint64_t ystride, DevPlan p) {
    __shared__ double lds[FSLds<LOGN>::WORDS];
    const FSLds<LOGN> L = fs_lds_init<LOGN>(lds, p);
    col_fwd_block<LOGN>(x + blockIdx.y * item_stride, Y + blockIdx.y * ystride, blockIdx.x * FS<LOGN>::SC, p, L);
}
template <int LOGN>
__global__ __launch_bounds__(512) void k_fs_row_conv(int32_t* Yf, const int32_t* Yg, uint64_t ystride,
                                                     DevPlan p) {
    __shared__ double lds[FSLds<LOGN>::WORDS];
    const FSLds<LOGN> L = fs_lds_init<LOGN>(lds, p);
    row_conv_block<LOGN>(Yf + blockIdx.y * ystride, Yg + blockIdx.y * ystride, blockIdx.x * FS<LOGN>::SR, p, L);
}
template <int LOGN, bool SCALE>
__global__ __launch_bounds__(512) void k_fs_col_inv(const int32_t* Y, uint32_t* x, uint64_t item_stride,
                                                    uint64_t ystride, DevPlan p) {
    __shared__ double lds[FSLds<LOGN>::WORDS];
    const FSLds<LOGN> L = fs_lds_init<LOGN>(lds, p);
    col_inv_block<LOGN, SCALE>(Y + blockIdx.y * ystride, x + blockIdx.y * item_stride, blockIdx.x * FS<LOGN>::SC,
                               p, L);
}
template <int LOGN>
__global__ __launch_bounds__(512) void k_fs_row_fwd_nat(const int32_t* Y, uint32_t* X, uint64_t item_stride,
                                                        uint64_t ystride, DevPlan p) {
    __shared__ double lds[FSLds<LOGN>::WORDS];
    const FSLds<LOGN> L = fs_lds_init<LOGN>(lds, p);
    row_fwd_nat_block<LOGN>(Y + blockIdx.y * ystride, X + blockIdx.y * item_stride, blockIdx.x * FS<LOGN>::SR, p, L);
}
template <int LOGN>
__global__ __launch_bounds__(512) void k_fs_row_inv_nat(const uint32_t* X, int32_t* Y, uint64_t item_stride,
                                                        uint64_t ystride, DevPlan p) {
    __shared__ double lds[FSLds<LOGN>::WORDS];
    const FSLds<LOGN> L = fs_lds_init<LOGN>(lds, p);
    row_inv_nat_block<LOGN>(X + blockIdx.y * item_stride, Y + blockIdx.y * ystride, blockIdx.x * FS<LOGN>::SR, p, L);
}

// Persistent fused convolution of a uniform-length batch: one workgroup owns
// one convolution at a time, start to finish, with a private 2N-word scratch.
template <int LOGN>
__global__ __launch_bounds__(512) void k_conv_fused(const uint32_t* f, const uint32_t* g, uint32_t* h,
                                                    const uint64_t* __restrict__ offs, uint32_t count,
                                                    int32_t* scratch, DevPlan p) {
    using G = FS<LOGN>;
    __shared__ double lds[FSLds<LOGN>::WORDS];
    const FSLds<LOGN> L = fs_lds_init<LOGN>(lds, p);
    int32_t* Yf = scratch + (size_t)blockIdx.x * 2 * G::N;
    int32_t* Yg = Yf + G::N;
    for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
        const uint64_t off = offs ? offs[item] : (uint64_t)item * G::N;
        const uint32_t* fi = f + off;
        const uint32_t* gi = g + off;
        // columns of f then of g; the next block's loads are issued before
        // the current block is transformed
        constexpr int CL = G::A - G::SC;
        ColIn<LOGN> cin = col_fwd_load<LOGN>(fi, 0);
        for (int c0 = 0; c0 < CL; c0 += G::SC) {
            const ColIn<LOGN> nxt = col_fwd_load<LOGN>(fi, c0 + G::SC);
            col_fwd_compute<LOGN>(cin, Yf, c0, p, L);
            cin = nxt;
        }
        {
            const ColIn<LOGN> nxt = col_fwd_load<LOGN>(gi, 0);
            col_fwd_compute<LOGN>(cin, Yf, CL, p, L);
            cin = nxt;
        }
        for (int c0 = 0; c0 < CL; c0 += G::SC) {
            const ColIn<LOGN> nxt = col_fwd_load<LOGN>(gi, c0 + G::SC);
            col_fwd_compute<LOGN>(cin, Yg, c0, p, L);
            cin = nxt;
        }
        col_fwd_compute<LOGN>(cin, Yg, CL, p, L);
        __syncthreads();
        RowIn<LOGN> rin = row_conv_load<LOGN>(Yf, Yg, 0);
        for (int r0 = 0; r0 < G::Bn - G::SR; r0 += G::SR) {
            const RowIn<LOGN> nxt = row_conv_load<LOGN>(Yf, Yg, r0 + G::SR);
            row_conv_compute<LOGN>(rin, Yf, r0, p, L);
            rin = nxt;
        }
        row_conv_compute<LOGN>(rin, Yf, G::Bn - G::SR, p, L);
        __syncthreads();
        ColInvIn<LOGN> iin = col_inv_load<LOGN>(Yf, 0);
        for (int c0 = 0; c0 < CL; c0 += G::SC) {
            const ColInvIn<LOGN> nxt = col_inv_load<LOGN>(Yf, c0 + G::SC);
            col_inv_compute<LOGN, false>(iin, h + off, c0, p, L);
            iin = nxt;
        }
        col_inv_compute<LOGN, false>(iin, h + off, CL, p, L);
        __syncthreads();
    }
}

// Sets *flag when some x[i] >= m.
__global__ void k_range_check(const uint32_t* __restrict__ x, uint64_t n, uint32_t m, uint32_t* flag) {
    uint32_t bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        bad |= (x[i] >= m) ? 1u : 0u;
    if (bad) atomicOr(flag, 1u);
}

hipError_t launch_range_check(const uint32_t* x, uint64_t n, uint32_t m, uint32_t* flag, hipStream_t st) {
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(uint32_t), st);
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_range_check, dim3((uint32_t)blocks), dim3(256), 0, st, x, n, m, flag);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launchers
#define NTT_SMALL_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)
#define NTT_LARGE_CASES(X) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22)

hipError_t launch_conv_small(int logn, const uint32_t* f, const uint32_t* g, uint32_t* h, const uint64_t* offs,
                             uint32_t count, const DevPlan& p, hipStream_t st) {
    if (count == 0) return hipSuccess;
    switch (logn) {
#define CASE(n)                                                                                   \
    case n: {                                                                                     \
        const uint32_t S = small_s(1 << n);                                                       \
        hipLaunchKernelGGL(k_conv_small<1 << n>, dim3((count + S - 1) / S), dim3(256), 0, st, f, g, h, \
                           offs, count, p);                                                       \
        return hipGetLastError();                                                                 \
    }
        NTT_SMALL_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_ntt_small(int logn, bool inv, const uint32_t* x, uint32_t* X, uint32_t batch, const DevPlan& p,
                            hipStream_t st) {
    if (batch == 0) return hipSuccess;
    switch (logn) {
#define CASE(n)                                                                                          \
    case n: {                                                                                            \
        const uint32_t S = small_s(1 << n);                                                              \
        if (inv)                                                                                         \
            hipLaunchKernelGGL((k_ntt_small<1 << n, true>), dim3((batch + S - 1) / S), dim3(256), 0, st, x, X, \
                               batch, p);                                                                \
        else                                                                                             \
            hipLaunchKernelGGL((k_ntt_small<1 << n, false>), dim3((batch + S - 1) / S), dim3(256), 0, st, x, \
                               X, batch, p);                                                             \
        return hipGetLastError();                                                                        \
    }
        NTT_SMALL_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_conv_fourstep(int logn, const uint32_t* f, const uint32_t* g, uint32_t* h, uint32_t items,
                                uint64_t item_stride, int32_t* scratch, const DevPlan& p, hipStream_t st) {
    if (items == 0) return hipSuccess;
    switch (logn) {
#define CASE(n)                                                                                               \
    case n: {                                                                                                 \
        using G = FS<n>;                                                                                      \
        const uint64_t ys = 2ull * G::N;                                                                      \
        int32_t* Yf = scratch;                                                                                \
        int32_t* Yg = scratch + G::N;                                                                         \
        hipLaunchKernelGGL(k_fs_col_fwd<n>, dim3(G::A / G::SC, items), dim3(G::T), 0, st, f, Yf, item_stride, ys, p); \
        hipLaunchKernelGGL(k_fs_col_fwd<n>, dim3(G::A / G::SC, items), dim3(G::T), 0, st, g, Yg, item_stride, ys, p); \
        hipLaunchKernelGGL(k_fs_row_conv<n>, dim3(G::Bn / G::SR, items), dim3(G::T), 0, st, Yf, (const int32_t*)Yg, ys, p); \
        hipLaunchKernelGGL((k_fs_col_inv<n, false>), dim3(G::A / G::SC, items), dim3(G::T), 0, st,           \
                           (const int32_t*)Yf, h, item_stride, ys, p);                                        \
        return hipGetLastError();                                                                             \
    }
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_ntt_fourstep(int logn, bool inv, const uint32_t* x, uint32_t* X, uint32_t batch,
                               int32_t* scratch, const DevPlan& p, hipStream_t st) {
    if (batch == 0) return hipSuccess;
    switch (logn) {
#define CASE(n)                                                                                               \
    case n: {                                                                                                 \
        using G = FS<n>;                                                                                      \
        const uint64_t N = G::N;                                                                              \
        if (!inv) {                                                                                           \
            hipLaunchKernelGGL(k_fs_col_fwd<n>, dim3(G::A / G::SC, batch), dim3(G::T), 0, st, x, scratch, N, N, p); \
            hipLaunchKernelGGL(k_fs_row_fwd_nat<n>, dim3(G::Bn / G::SR, batch), dim3(G::T), 0, st,              \
                               (const int32_t*)scratch, X, N, N, p);                                          \
        } else {                                                                                              \
            hipLaunchKernelGGL(k_fs_row_inv_nat<n>, dim3(G::Bn / G::SR, batch), dim3(G::T), 0, st, x, scratch, N, N, p); \
            hipLaunchKernelGGL((k_fs_col_inv<n, true>), dim3(G::A / G::SC, batch), dim3(G::T), 0, st,          \
                               (const int32_t*)scratch, X, N, N, p);                                          \
        }                                                                                                     \
        return hipGetLastError();                                                                             \
    }
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_conv_fused(int logn, const uint32_t* f, const uint32_t* g, uint32_t* h, const uint64_t* offs,
                             uint32_t count, int32_t* scratch, uint32_t grid, const DevPlan& p, hipStream_t st) {
    if (count == 0) return hipSuccess;
    switch (logn) {
#define CASE(n)                                                                                             \
    case n:                                                                                                 \
        hipLaunchKernelGGL(k_conv_fused<n>, dim3(grid), dim3(FS<n>::T), 0, st, f, g, h, offs, count, scratch, p); \
        return hipGetLastError();
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

int fused_blocks_per_cu(int logn) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (logn) {
#define CASE(n) \
    case n: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_conv_fused<n>, FS<n>::T, 0); break;
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            break;
    }
    return e == hipSuccess ? nb : 0;
}

}  // namespace nttmi
