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
    static constexpr int SC = 4096 / Bn;   // columns per block (256 threads)
    static constexpr int SR = 4096 / A;    // rows per block
    using BC = Blk<Bn, SC, SEQ_FAST>;
    using BR = Blk<A, SR, POS_FAST>;
    using BRS = Blk<A, SR, SEQ_FAST>;      // rows read/written at stride B (natural-order NTT)
    static constexpr int LDS = (BC::LDS_DOUBLES > BR::LDS_DOUBLES ? BC::LDS_DOUBLES : BR::LDS_DOUBLES) >
                                       BRS::LDS_DOUBLES
                                   ? (BC::LDS_DOUBLES > BR::LDS_DOUBLES ? BC::LDS_DOUBLES : BR::LDS_DOUBLES)
                                   : BRS::LDS_DOUBLES;
};

// Column phase, forward: length-B transforms of columns c0..c0+SC of x
// (natural order, any 32-bit values), times w^(t1 u2), into scratch rows.
template <int LOGN>
__device__ __forceinline__ void col_fwd_block(const uint32_t* x, int32_t* Y, int c0, const DevPlan& p,
                                              double* lds) {
    using G = FS<LOGN>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int t1 = c0 + s;
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = reduce((double)x[t1 + (size_t)G::A * B::pos0(j, i)], M);
    block_dft<G::Bn, G::SC, SEQ_FAST, false>(v, lds, s, j, p.P, G::la, G::N - 1, M);
    mul_twiddles<B::E>(v, M, [&](int i) { return p.TT[(size_t)B::posL(j, i) * G::A + t1]; });
#pragma unroll
    for (int i = 0; i < B::E; ++i) Y[(size_t)B::posL(j, i) * G::A + t1] = to_i32(v[i]);
}

// Row phase of a convolution: for rows r0..r0+SR, forward(f row), forward(g
// row), product with N^-1, inverse, times w^-(t1 u2), back into Yf.
template <int LOGN>
__device__ __forceinline__ void row_conv_block(int32_t* Yf, const int32_t* Yg, int r0, const DevPlan& p,
                                               double* lds) {
    using G = FS<LOGN>;
    using B = typename G::BR;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int u2 = r0 + s;
    int32_t* rf = Yf + (size_t)u2 * G::A;
    const int32_t* rg = Yg + (size_t)u2 * G::A;
    double F[B::E], v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = from_i32(rf[B::pos0(j, i)]);
    block_dft<G::A, G::SR, POS_FAST, false>(v, lds, s, j, p.P, G::lb, G::N - 1, M);
#pragma unroll
    for (int i = 0; i < B::E; ++i) F[i] = v[i];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = from_i32(rg[B::pos0(j, i)]);
    block_dft<G::A, G::SR, POS_FAST, false>(v, lds, s, j, p.P, G::lb, G::N - 1, M);
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
        const double gs = mulmod(v[i], p.ninv, p.ninvq, M);
        v[i] = mulmod_var(F[i], gs, M);
    }
    if (B::R0 != B::RL) {
#pragma unroll
        for (int i = 0; i < B::E; ++i) lds[B::lds(s, B::posL(j, i))] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < B::E; ++i) v[i] = lds[B::lds(s, B::pos0(j, i))];
        __syncthreads();
    }
    block_dft<G::A, G::SR, POS_FAST, true>(v, lds, s, j, p.P, G::lb, G::N - 1, M);
    mul_twiddles<B::E>(v, M, [&](int i) { return p.TTi[(size_t)u2 * G::A + B::posL(j, i)]; });
#pragma unroll
    for (int i = 0; i < B::E; ++i) rf[B::posL(j, i)] = to_i32(v[i]);
}

// Column phase, inverse: length-B inverse transforms of scratch columns,
// optional N^-1, canonical store to x[t1 + A t2].
template <int LOGN, bool SCALE>
__device__ __forceinline__ void col_inv_block(const int32_t* Y, uint32_t* x, int c0, const DevPlan& p,
                                              double* lds) {
    using G = FS<LOGN>;
    using B = typename G::BC;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int t1 = c0 + s;
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = from_i32(Y[(size_t)B::pos0(j, i) * G::A + t1]);
    block_dft<G::Bn, G::SC, SEQ_FAST, true>(v, lds, s, j, p.P, G::la, G::N - 1, M);
#pragma unroll
    for (int i = 0; i < B::E; ++i) {
        const double y = SCALE ? mulmod(v[i], p.ninv, p.ninvq, M) : v[i];
        x[t1 + (size_t)G::A * B::posL(j, i)] = canon_u32(y, M);
    }
}

// Row phase of the natural-order forward transform: X[u2 + B u1].
template <int LOGN>
__device__ __forceinline__ void row_fwd_nat_block(const int32_t* Y, uint32_t* X, int r0, const DevPlan& p,
                                                  double* lds) {
    using G = FS<LOGN>;
    using B = typename G::BRS;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int u2 = r0 + s;
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = from_i32(Y[(size_t)u2 * G::A + B::pos0(j, i)]);
    block_dft<G::A, G::SR, SEQ_FAST, false>(v, lds, s, j, p.P, G::lb, G::N - 1, M);
#pragma unroll
    for (int i = 0; i < B::E; ++i) X[u2 + (size_t)G::Bn * B::posL(j, i)] = canon_u32(v[i], M);
}

// Row phase of the natural-order inverse transform: from X[u2 + B u1] to
// scratch rows, times w^-(t1 u2).
template <int LOGN>
__device__ __forceinline__ void row_inv_nat_block(const uint32_t* X, int32_t* Y, int r0, const DevPlan& p,
                                                  double* lds) {
    using G = FS<LOGN>;
    using B = typename G::BRS;
    int s, j;
    B::item(threadIdx.x, s, j);
    const ModC M = p.M;
    const int u2 = r0 + s;
    double v[B::E];
#pragma unroll
    for (int i = 0; i < B::E; ++i) v[i] = reduce((double)X[u2 + (size_t)G::Bn * B::pos0(j, i)], M);
    block_dft<G::A, G::SR, SEQ_FAST, true>(v, lds, s, j, p.P, G::lb, G::N - 1, M);
    mul_twiddles<B::E>(v, M, [&](int i) { return p.TTi[(size_t)u2 * G::A + B::posL(j, i)]; });
#pragma unroll
    for (int i = 0; i < B::E; ++i) Y[(size_t)u2 * G::A + B::posL(j, i)] = to_i32(v[i]);
}

// Kernels of the multi-launch four-step (grid.y = item / row of the batch).
template <int LOGN>
__global__ __launch_bounds__(256) void k_fs_col_fwd(const uint32_t* x, int32_t* Y, uint64_t item_stride,
                                                    uint64_t ystride, DevPlan p) {
    __shared__ double lds[FS<LOGN>::LDS];
    col_fwd_block<LOGN>(x + blockIdx.y * item_stride, Y + blockIdx.y * ystride, blockIdx.x * FS<LOGN>::SC, p,
                        lds);
}
template <int LOGN>
__global__ __launch_bounds__(256) void k_fs_row_conv(int32_t* Yf, const int32_t* Yg, uint64_t ystride,
                                                     DevPlan p) {
    __shared__ double lds[FS<LOGN>::LDS];
    row_conv_block<LOGN>(Yf + blockIdx.y * ystride, Yg + blockIdx.y * ystride, blockIdx.x * FS<LOGN>::SR, p,
                         lds);
}
template <int LOGN, bool SCALE>
__global__ __launch_bounds__(256) void k_fs_col_inv(const int32_t* Y, uint32_t* x, uint64_t item_stride,
                                                    uint64_t ystride, DevPlan p) {
    __shared__ double lds[FS<LOGN>::LDS];
    col_inv_block<LOGN, SCALE>(Y + blockIdx.y * ystride, x + blockIdx.y * item_stride, blockIdx.x * FS<LOGN>::SC,
                               p, lds);
}
template <int LOGN>
__global__ __launch_bounds__(256) void k_fs_row_fwd_nat(const int32_t* Y, uint32_t* X, uint64_t item_stride,
                                                        uint64_t ystride, DevPlan p) {
    __shared__ double lds[FS<LOGN>::LDS];
    row_fwd_nat_block<LOGN>(Y + blockIdx.y * ystride, X + blockIdx.y * item_stride, blockIdx.x * FS<LOGN>::SR, p,
                            lds);
}
template <int LOGN>
__global__ __launch_bounds__(256) void k_fs_row_inv_nat(const uint32_t* X, int32_t* Y, uint64_t item_stride,
                                                        uint64_t ystride, DevPlan p) {
    __shared__ double lds[FS<LOGN>::LDS];
    row_inv_nat_block<LOGN>(X + blockIdx.y * item_stride, Y + blockIdx.y * ystride, blockIdx.x * FS<LOGN>::SR, p,
                            lds);
}

// Persistent fused convolution of a uniform-length batch: one workgroup owns
// one convolution at a time, start to finish, with a private 2N-word scratch.
template <int LOGN>
__global__ __launch_bounds__(256) void k_conv_fused(const uint32_t* f, const uint32_t* g, uint32_t* h,
                                                    const uint64_t* __restrict__ offs, uint32_t count,
                                                    int32_t* scratch, DevPlan p) {
    using G = FS<LOGN>;
    __shared__ double lds[G::LDS];
    int32_t* Yf = scratch + (size_t)blockIdx.x * 2 * G::N;
    int32_t* Yg = Yf + G::N;
    for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
        const uint64_t off = offs ? offs[item] : (uint64_t)item * G::N;
        for (int c0 = 0; c0 < G::A; c0 += G::SC) col_fwd_block<LOGN>(f + off, Yf, c0, p, lds);
        for (int c0 = 0; c0 < G::A; c0 += G::SC) col_fwd_block<LOGN>(g + off, Yg, c0, p, lds);
        __syncthreads();
        for (int r0 = 0; r0 < G::Bn; r0 += G::SR) row_conv_block<LOGN>(Yf, Yg, r0, p, lds);
        __syncthreads();
        for (int c0 = 0; c0 < G::A; c0 += G::SC) col_inv_block<LOGN, false>(Yf, h + off, c0, p, lds);
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
#define NTT_LARGE_CASES(X) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24)

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
        hipLaunchKernelGGL(k_fs_col_fwd<n>, dim3(G::A / G::SC, items), dim3(256), 0, st, f, Yf, item_stride, ys, p); \
        hipLaunchKernelGGL(k_fs_col_fwd<n>, dim3(G::A / G::SC, items), dim3(256), 0, st, g, Yg, item_stride, ys, p); \
        hipLaunchKernelGGL(k_fs_row_conv<n>, dim3(G::Bn / G::SR, items), dim3(256), 0, st, Yf, (const int32_t*)Yg, ys, p); \
        hipLaunchKernelGGL((k_fs_col_inv<n, false>), dim3(G::A / G::SC, items), dim3(256), 0, st,           \
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
            hipLaunchKernelGGL(k_fs_col_fwd<n>, dim3(G::A / G::SC, batch), dim3(256), 0, st, x, scratch, N, N, p); \
            hipLaunchKernelGGL(k_fs_row_fwd_nat<n>, dim3(G::Bn / G::SR, batch), dim3(256), 0, st,              \
                               (const int32_t*)scratch, X, N, N, p);                                          \
        } else {                                                                                              \
            hipLaunchKernelGGL(k_fs_row_inv_nat<n>, dim3(G::Bn / G::SR, batch), dim3(256), 0, st, x, scratch, N, N, p); \
            hipLaunchKernelGGL((k_fs_col_inv<n, true>), dim3(G::A / G::SC, batch), dim3(256), 0, st,          \
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
        hipLaunchKernelGGL(k_conv_fused<n>, dim3(grid), dim3(256), 0, st, f, g, h, offs, count, scratch, p); \
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
    case n: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_conv_fused<n>, 256, 0); break;
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            break;
    }
    return e == hipSuccess ? nb : 0;
}

}  // namespace nttmi
