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

template <class W>
static hipError_t conv_fourstep_t(int logn, const void* f, const void* g, void* h, uint32_t items,
                                  uint64_t item_stride, void* scratch, const DevPlan& p, hipStream_t st,
                                  uint32_t* singular) {
    using T = typename W::word;
    using SW = typename W::sword;
    switch (logn) {
#define CASE(n)                                                                                                   \
    case n: {                                                                                                     \
        using G = FS<n>;                                                                                          \
        const uint64_t ys = 2ull * G::N;                                                                          \
        SW* Yf = (SW*)scratch;                                                                                    \
        SW* Yg = Yf + G::N;                                                                                       \
        if (2ull * items <= 65535) {                                                                              \
            hipLaunchKernelGGL((k_fs_col_fwd2<W, n>), dim3(G::A / G::SC, 2 * items), dim3(G::T), 0, st,            \
                               (const T*)f, (const T*)g, Yf, item_stride, ys, items, p);                          \
        } else {                                                                                                  \
            hipLaunchKernelGGL((k_fs_col_fwd<W, n>), dim3(G::A / G::SC, items), dim3(G::T), 0, st, (const T*)f,   \
                               Yf, item_stride, ys, p);                                                           \
            hipLaunchKernelGGL((k_fs_col_fwd<W, n>), dim3(G::A / G::SC, items), dim3(G::T), 0, st, (const T*)g,   \
                               Yg, item_stride, ys, p);                                                           \
        }                                                                                                         \
        if (singular)                                                                                             \
            hipLaunchKernelGGL((k_fs_row_conv<W, n, OP_DIV>),                                                     \
                               dim3(fs_row_grid(G::la, FS_ROW_LOOP_CONV, G::Bn / G::SR, items), items),           \
                               dim3(G::T), 0, st, Yf,                                                             \
                               (const SW*)Yg, ys, p, singular);                                                   \
        else                                                                                                      \
            hipLaunchKernelGGL((k_fs_row_conv<W, n, OP_MUL>),                                                     \
                               dim3(fs_row_grid(G::la, FS_ROW_LOOP_CONV, G::Bn / G::SR, items), items),           \
                               dim3(G::T), 0, st, Yf,                                                             \
                               (const SW*)Yg, ys, p, singular);                                                   \
        hipLaunchKernelGGL((k_fs_col_inv<W, n, false>), dim3(G::A / G::SC, items), dim3(G::T), 0, st,              \
                           (const SW*)Yf, (T*)h, item_stride, ys, p);                                             \
        return hipGetLastError();                                                                                 \
    }
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_conv_fourstep(int wbits, int logn, const void* f, const void* g, void* h, uint32_t items,
                                uint64_t item_stride, void* scratch, const DevPlan& p, hipStream_t st,
                                uint32_t* singular) {
    if (items == 0) return hipSuccess;
    return wbits == 32 ? conv_fourstep_t<W32>(logn, f, g, h, items, item_stride, scratch, p, st, singular)
                       : conv_fourstep_t<W64>(logn, f, g, h, items, item_stride, scratch, p, st, singular);
}

template <class W>
static hipError_t ntt_fourstep_t(int logn, bool inv, const void* x, void* X, uint32_t batch, void* scratch,
                                 const DevPlan& p, hipStream_t st) {
    using T = typename W::word;
    using SW = typename W::sword;
    switch (logn) {
#define CASE(n)                                                                                                   \
    case n: {                                                                                                     \
        using G = FS<n>;                                                                                          \
        const uint64_t N = G::N;                                                                                  \
        if (!inv) {                                                                                               \
            hipLaunchKernelGGL((k_fs_col_fwd<W, n>), dim3(G::A / G::SC, batch), dim3(G::T), 0, st, (const T*)x,   \
                               (SW*)scratch, N, N, p);                                                            \
            hipLaunchKernelGGL((k_fs_row_fwd_nat<W, n>),                                                          \
                               dim3(fs_row_grid(G::la, FS_ROW_LOOP_NAT, G::Bn / G::SR, batch), batch),            \
                               dim3(G::T), 0, st,                                                                 \
                               (const SW*)scratch, (T*)X, N, N, p);                                               \
        } else {                                                                                                  \
            hipLaunchKernelGGL((k_fs_row_inv_nat<W, n>),                                                          \
                               dim3(fs_row_grid(G::la, FS_ROW_LOOP_NAT, G::Bn / G::SR, batch), batch),            \
                               dim3(G::T), 0, st,                                                                 \
                               (const T*)x, (SW*)scratch, N, N, p);                                               \
            hipLaunchKernelGGL((k_fs_col_inv<W, n, true>), dim3(G::A / G::SC, batch), dim3(G::T), 0, st,          \
                               (const SW*)scratch, (T*)X, N, N, p);                                               \
        }                                                                                                         \
        return hipGetLastError();                                                                                 \
    }
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_ntt_fourstep(int wbits, int logn, bool inv, const void* x, void* X, uint32_t batch, void* scratch,
                               const DevPlan& p, hipStream_t st) {
    if (batch == 0) return hipSuccess;
    return wbits == 32 ? ntt_fourstep_t<W32>(logn, inv, x, X, batch, scratch, p, st)
                       : ntt_fourstep_t<W64>(logn, inv, x, X, batch, scratch, p, st);
}

}  // namespace nttmi
