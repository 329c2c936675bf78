// Launchers of the single persistent launch for a batch of uneven lengths.
#include "kernels.hpp"

namespace nttmi {

template <class W>
static hipError_t conv_multi_t(const void* f, const void* g, void* h, const void* tasks, uint32_t ntasks,
                               const uint64_t* toffs, void* scratch, uint64_t scratch_words, uint32_t* queue,
                               uint32_t grid, const DevPlan* plans, hipStream_t st) {
    using T = typename W::word;
    hipLaunchKernelGGL(k_conv_multi<W>, dim3(grid), dim3(512), 0, st, (const T*)f, (const T*)g, (T*)h,
                       (const MultiTask*)tasks, ntasks, toffs, (typename W::sword*)scratch, scratch_words, queue,
                       plans);
    return hipGetLastError();
}

hipError_t launch_conv_multi(int wbits, const void* f, const void* g, void* h, const void* tasks, uint32_t ntasks,
                             const uint64_t* toffs, void* scratch, uint64_t scratch_words, uint32_t* queue,
                             uint32_t grid, const DevPlan* plans, hipStream_t st) {
    if (ntasks == 0) return hipSuccess;
    return wbits == 32 ? conv_multi_t<W32>(f, g, h, tasks, ntasks, toffs, scratch, scratch_words, queue, grid, plans, st)
                       : conv_multi_t<W64>(f, g, h, tasks, ntasks, toffs, scratch, scratch_words, queue, grid, plans, st);
}

int multi_max_log2n(int wbits) { return wbits == 32 ? MultiCfg<W32>::NMAX : MultiCfg<W64>::NMAX; }
int multi_tile(int logn) { return multi_s(1 << logn); }
int multi_blocks_per_cu(int wbits) {
    static std::atomic<int> cache[2] = {{-1}, {-1}};
    std::atomic<int>& c = cache[wbits == 32 ? 0 : 1];
    int v = c.load(std::memory_order_relaxed);
    if (v < 0) {
        int nb = 0;
        const hipError_t e = wbits == 32
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_conv_multi<W32>, 512, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_conv_multi<W64>, 512, 0);
        v = e == hipSuccess ? nb : 0;
        c.store(v, std::memory_order_relaxed);
    }
    return v;
}

}  // namespace nttmi
