// Launchers of the multi-launch four-step kernels (lengths above 2^12).
#include "kernels.hpp"

namespace nttmi {

// Workgroups per item of a row kernel.  Rows of 2^loop_la positions and more
// (the kernel's threshold, FS_ROW_LOOP_*): fewer workgroups than row blocks
// once the batch has many, each taking several blocks and filling its twiddle
// table once for them, with at least about 1024 workgroups in the launch.
// Shorter rows keep a workgroup per block.
static uint32_t fs_row_grid(int la, int loop_la, uint32_t rblocks, uint32_t items) {
    if (la < loop_la) return rblocks;
    const uint64_t total = (uint64_t)rblocks * items;
    uint32_t per = (uint32_t)(total / 1024);   // blocks per workgroup
    if (per < 1) per = 1;
    if (per > rblocks) per = rblocks;
    return (rblocks + per - 1) / per;
}

// Whether a multi-launch four-step launch of `blocks512` column blocks of
// 512-thread workgroups (over all operands and items) takes 256-thread
// workgroups instead: where the 512-thread blocks would not give every CU
// one, halving the blocks doubles their number (measured for one item: 2^16
// 18.5 -> 15.6 us, 2^18 23.0 -> 19.8 us, 2^19 28.3 -> 22.9 us; for 8 items of
// 2^18, 1024 blocks of 256 threads, 38.1 -> 42.4 us, so larger batches keep
// 512).  Lengths up to 2^19 only: their columns have at most 256 positions,
// so that a 256-thread block still spans 16 columns or more (row segments of
// 64 bytes or more).
static bool fs_narrow(int logn, uint64_t blocks512, uint32_t cus) {
    return logn <= FOURSTEP_256_MAX_LOG2N && blocks512 < (uint64_t)cus;
}

template <class W, int n, int TT>
static hipError_t conv_fourstep_g(const void* f, const void* g, void* h, uint32_t items, uint64_t item_stride,
                                  void* scratch, const DevPlan& p, hipStream_t st, uint32_t* singular) {
    using T = typename W::word;
    using SW = typename W::sword;
    using G = FS<n, TT>;
    const uint64_t ys = 2ull * G::N;
    SW* Yf = (SW*)scratch;
    SW* Yg = Yf + G::N;
    if (2ull * items <= 65535) {
        hipLaunchKernelGGL((k_fs_col_fwd2<W, n, TT>), dim3(G::A / G::SC, 2 * items), dim3(G::T), 0, st, (const T*)f,
                           (const T*)g, Yf, item_stride, ys, items, p);
    } else {
        hipLaunchKernelGGL((k_fs_col_fwd<W, n, TT>), dim3(G::A / G::SC, items), dim3(G::T), 0, st, (const T*)f, Yf,
                           item_stride, ys, p);
        hipLaunchKernelGGL((k_fs_col_fwd<W, n, TT>), dim3(G::A / G::SC, items), dim3(G::T), 0, st, (const T*)g, Yg,
                           item_stride, ys, p);
    }
    const dim3 rgrid(fs_row_grid(G::la, FS_ROW_LOOP_CONV, G::Bn / G::SR, items), items);
    if (singular)
        hipLaunchKernelGGL((k_fs_row_conv<W, n, OP_DIV, TT>), rgrid, dim3(G::T), 0, st, Yf, (const SW*)Yg, ys, p,
                           singular);
    else
        hipLaunchKernelGGL((k_fs_row_conv<W, n, OP_MUL, TT>), rgrid, dim3(G::T), 0, st, Yf, (const SW*)Yg, ys, p,
                           singular);
    hipLaunchKernelGGL((k_fs_col_inv<W, n, false, TT>), dim3(G::A / G::SC, items), dim3(G::T), 0, st, (const SW*)Yf,
                       (T*)h, item_stride, ys, p);
    return hipGetLastError();
}

template <class W, int n>
static hipError_t conv_fourstep_n(const void* f, const void* g, void* h, uint32_t items, uint64_t item_stride,
                                  void* scratch, const DevPlan& p, hipStream_t st, uint32_t* singular, uint32_t cus,
                                  int tt) {
    using G = FS<n>;
    if constexpr (n <= FOURSTEP_256_MAX_LOG2N) {
        if (tt == 256 || (tt == 0 && fs_narrow(n, 2ull * items * (G::A / G::SC), cus)))
            return conv_fourstep_g<W, n, 256>(f, g, h, items, item_stride, scratch, p, st, singular);
    }
    return conv_fourstep_g<W, n, 512>(f, g, h, items, item_stride, scratch, p, st, singular);
}

template <class W>
static hipError_t conv_fourstep_t(int logn, const void* f, const void* g, void* h, uint32_t items,
                                  uint64_t item_stride, void* scratch, const DevPlan& p, hipStream_t st,
                                  uint32_t* singular, uint32_t cus, int tt) {
    switch (logn) {
#define CASE(n) \
    case n: return conv_fourstep_n<W, n>(f, g, h, items, item_stride, scratch, p, st, singular, cus, tt);
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_conv_fourstep(int wbits, int logn, const void* f, const void* g, void* h, uint32_t items,
                                uint64_t item_stride, void* scratch, const DevPlan& p, hipStream_t st,
                                uint32_t* singular, uint32_t cus, int tt) {
    if (items == 0) return hipSuccess;
    return wbits == 32 ? conv_fourstep_t<W32>(logn, f, g, h, items, item_stride, scratch, p, st, singular, cus, tt)
                       : conv_fourstep_t<W64>(logn, f, g, h, items, item_stride, scratch, p, st, singular, cus, tt);
}

template <class W, int n, int TT>
static hipError_t ntt_fourstep_g(bool inv, const void* x, void* X, uint32_t batch, void* scratch, const DevPlan& p,
                                 hipStream_t st) {
    using T = typename W::word;
    using SW = typename W::sword;
    using G = FS<n, TT>;
    const uint64_t N = G::N;
    const dim3 rgrid(fs_row_grid(G::la, FS_ROW_LOOP_NAT, G::Bn / G::SR, batch), batch);
    if (!inv) {
        hipLaunchKernelGGL((k_fs_col_fwd<W, n, TT>), dim3(G::A / G::SC, batch), dim3(G::T), 0, st, (const T*)x,
                           (SW*)scratch, N, N, p);
        hipLaunchKernelGGL((k_fs_row_fwd_nat<W, n, TT>), rgrid, dim3(G::T), 0, st, (const SW*)scratch, (T*)X, N, N, p);
    } else {
        hipLaunchKernelGGL((k_fs_row_inv_nat<W, n, TT>), rgrid, dim3(G::T), 0, st, (const T*)x, (SW*)scratch, N, N, p);
        hipLaunchKernelGGL((k_fs_col_inv<W, n, true, TT>), dim3(G::A / G::SC, batch), dim3(G::T), 0, st,
                           (const SW*)scratch, (T*)X, N, N, p);
    }
    return hipGetLastError();
}

template <class W, int n>
static hipError_t ntt_fourstep_n(bool inv, const void* x, void* X, uint32_t batch, void* scratch, const DevPlan& p,
                                 hipStream_t st, uint32_t cus) {
    using G = FS<n>;
    if constexpr (n <= FOURSTEP_256_MAX_LOG2N) {
        if (fs_narrow(n, (uint64_t)batch * (G::A / G::SC), cus))
            return ntt_fourstep_g<W, n, 256>(inv, x, X, batch, scratch, p, st);
    }
    return ntt_fourstep_g<W, n, 512>(inv, x, X, batch, scratch, p, st);
}

template <class W>
static hipError_t ntt_fourstep_t(int logn, bool inv, const void* x, void* X, uint32_t batch, void* scratch,
                                 const DevPlan& p, hipStream_t st, uint32_t cus) {
    switch (logn) {
#define CASE(n) \
    case n: return ntt_fourstep_n<W, n>(inv, x, X, batch, scratch, p, st, cus);
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_ntt_fourstep(int wbits, int logn, bool inv, const void* x, void* X, uint32_t batch, void* scratch,
                               const DevPlan& p, hipStream_t st, uint32_t cus) {
    if (batch == 0) return hipSuccess;
    return wbits == 32 ? ntt_fourstep_t<W32>(logn, inv, x, X, batch, scratch, p, st, cus)
                       : ntt_fourstep_t<W64>(logn, inv, x, X, batch, scratch, p, st, cus);
}

}  // namespace nttmi
