// Launchers of the persistent fused kernel of one length, and its occupancy.
#include "kernels.hpp"

namespace nttmi {

template <class W, int OP>
static hipError_t conv_fused_t(int logn, const void* f, const void* g, void* h, const uint64_t* offs,
                               uint32_t count, void* scratch, uint32_t* queue, uint32_t grid, const DevPlan& p,
                               hipStream_t st, uint32_t* singular, CrtStore crt = CrtStore{}) {
    using T = typename W::word;
    using SW = typename W::sword;
    switch (logn) {
#define CASE(n)                                                                                                   \
    case n:                                                                                                       \
        hipLaunchKernelGGL((k_conv_fused<W, n, OP>), dim3(grid), dim3(FS<n>::T), 0, st, (const T*)f, (const T*)g, \
                           (T*)h, offs, count, (SW*)scratch, queue, p, singular, crt);                            \
        return hipGetLastError();
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_conv_fused(int wbits, int logn, const void* f, const void* g, void* h, const uint64_t* offs,
                             uint32_t count, void* scratch, uint32_t* queue, uint32_t grid, const DevPlan& p,
                             hipStream_t st, uint32_t* singular, const CrtStore* crt) {
    if (count == 0) return hipSuccess;
    if (crt) {
        if (wbits != 32 || singular) return hipErrorInvalidValue;
        return conv_fused_t<W32, OP_CRT>(logn, f, g, h, offs, count, scratch, queue, grid, p, st, nullptr, *crt);
    }
    if (singular)
        return wbits == 32
                   ? conv_fused_t<W32, OP_DIV>(logn, f, g, h, offs, count, scratch, queue, grid, p, st, singular)
                   : conv_fused_t<W64, OP_DIV>(logn, f, g, h, offs, count, scratch, queue, grid, p, st, singular);
    return wbits == 32 ? conv_fused_t<W32, OP_MUL>(logn, f, g, h, offs, count, scratch, queue, grid, p, st, nullptr)
                       : conv_fused_t<W64, OP_MUL>(logn, f, g, h, offs, count, scratch, queue, grid, p, st, nullptr);
}

template <class W, int OP>
static int fused_bpc_t(int logn) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (logn) {
#define CASE(n) \
    case n: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_conv_fused<W, n, OP>, FS<n>::T, 0); break;
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            break;
    }
    return e == hipSuccess ? nb : 0;
}

// Occupancy of the fused kernel, queried once per (word width, length, the
// pointwise step: 0 product, 1 quotient) so that later calls (also under graph
// capture) make no runtime query.
int fused_blocks_per_cu(int wbits, int logn, int div) {
    // thread-safe one-time initialisation of the table (-1: not yet queried)
    constexpr int PER = MAX_LOG2N + 1;
    static std::atomic<int>* cache = [] {
        auto* c = new std::atomic<int>[4 * PER];
        for (int i = 0; i < 4 * PER; ++i) c[i].store(-1);
        return c;
    }();
    if (logn < 0 || logn > MAX_LOG2N) return 0;
    std::atomic<int>& c = cache[((wbits == 32 ? 0 : 1) + (div ? 2 : 0)) * PER + logn];
    int v = c.load(std::memory_order_relaxed);
    if (v < 0) {
        if (div) v = wbits == 32 ? fused_bpc_t<W32, OP_DIV>(logn) : fused_bpc_t<W64, OP_DIV>(logn);
        else v = wbits == 32 ? fused_bpc_t<W32, OP_MUL>(logn) : fused_bpc_t<W64, OP_MUL>(logn);
        c.store(v, std::memory_order_relaxed);
    }
    return v;
}

int fused_threads(int logn) {
    switch (logn) {
#define CASE(n) \
    case n: return FS<n>::T;
        NTT_LARGE_CASES(CASE)
#undef CASE
        default:
            return 0;
    }
}

}  // namespace nttmi
