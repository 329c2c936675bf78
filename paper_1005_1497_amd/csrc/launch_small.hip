// Launchers of the LDS kernels (lengths up to 2^12).
#include "kernels.hpp"

namespace nttmi {

template <class W, int L, int S, int OP = OP_MUL>
static hipError_t conv_small_launch(const void* f, const void* g, void* h, const uint64_t* offs, uint32_t count,
                                    const DevPlan& p, hipStream_t st, uint32_t* singular = nullptr) {
    using T = typename W::word;
    hipLaunchKernelGGL((k_conv_small<W, L, S, OP>), dim3((count + S - 1) / S), dim3(small_threads(L, S)), 0, st,
                       (const T*)f, (const T*)g, (T*)h, offs, count, p, singular);
    return hipGetLastError();
}

template <class W>
static hipError_t conv_small_t(int logn, const void* f, const void* g, void* h, const uint64_t* offs, uint32_t count,
                               const DevPlan& p, hipStream_t st, int tile, uint32_t* singular) {
    switch (logn) {
#define CASE(n)                                                                                                   \
    case n:                                                                                                       \
        return singular ? conv_small_launch<W, 1 << n, small_s(1 << n), OP_DIV>(f, g, h, offs, count, p, st,     \
                                                                                 singular)                        \
               : tile == SMALL_TILE_WAVE                                                                          \
                   ? conv_small_launch<W, 1 << n, small_s_wave(1 << n)>(f, g, h, offs, count, p, st)            \
                   : conv_small_launch<W, 1 << n, small_s(1 << n)>(f, g, h, offs, count, p, st);
        NTT_SMALL_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_conv_small(int wbits, int logn, const void* f, const void* g, void* h, const uint64_t* offs,
                             uint32_t count, const DevPlan& p, hipStream_t st, int tile, uint32_t* singular) {
    if (count == 0) return hipSuccess;
    return wbits == 32 ? conv_small_t<W32>(logn, f, g, h, offs, count, p, st, tile, singular)
                       : conv_small_t<W64>(logn, f, g, h, offs, count, p, st, tile, singular);
}

template <class W>
static hipError_t ntt_small_t(int logn, bool inv, const void* x, void* X, uint32_t batch, const DevPlan& p,
                              hipStream_t st, const void* y) {
    using T = typename W::word;
    switch (logn) {
#define CASE(n)                                                                                                   \
    case n: {                                                                                                     \
        const uint32_t S = small_s(1 << n);                                                                       \
        if (inv && y)                                                                                             \
            hipLaunchKernelGGL((k_ntt_small<W, 1 << n, true, true>), dim3((batch + S - 1) / S), dim3(256), 0, st, \
                               (const T*)x, (T*)X, batch, p, (const T*)y);                                        \
        else if (inv)                                                                                             \
            hipLaunchKernelGGL((k_ntt_small<W, 1 << n, true>), dim3((batch + S - 1) / S), dim3(256), 0, st,       \
                               (const T*)x, (T*)X, batch, p, nullptr);                                            \
        else                                                                                                      \
            hipLaunchKernelGGL((k_ntt_small<W, 1 << n, false>), dim3((batch + S - 1) / S), dim3(256), 0, st,      \
                               (const T*)x, (T*)X, batch, p, nullptr);                                            \
        return hipGetLastError();                                                                                 \
    }
        NTT_SMALL_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_ntt_small(int wbits, int logn, bool inv, const void* x, void* X, uint32_t batch, const DevPlan& p,
                            hipStream_t st, const void* y) {
    if (batch == 0) return hipSuccess;
    if (y && !inv) return hipErrorInvalidValue;
    return wbits == 32 ? ntt_small_t<W32>(logn, inv, x, X, batch, p, st, y)
                       : ntt_small_t<W64>(logn, inv, x, X, batch, p, st, y);
}

}  // namespace nttmi
