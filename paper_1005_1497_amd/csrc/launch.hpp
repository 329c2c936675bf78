// Internal interface between the host library and the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "arith.hpp"

namespace nttmi {

// Device-resident tables and constants of one (m, N, root) plan, passed to
// every kernel by value.
struct DevPlan {
    const double2* P;    // P[e] = (w^e, w^e / m), e < N: powers of the N-th root
    const double* TT;    // four-step twiddles TT[u2 * A + t1] = w^(t1 u2) (large N only)
    const double* TTi;   // w^-(t1 u2)
    ModC M;
    double ninv, ninvq;  // N^-1 mod m and N^-1 / m
    int logn, nmask;
};

constexpr int SMALL_MAX_LOG2N = 12;
constexpr int MAX_LOG2N = 22;   // 32-bit words: m < 2^24, and no such prime has nu = 2^23

hipError_t launch_conv_small(int logn, const uint32_t* f, const uint32_t* g, uint32_t* h, const uint64_t* offs,
                             uint32_t count, const DevPlan& p, hipStream_t st);
hipError_t launch_ntt_small(int logn, bool inv, const uint32_t* x, uint32_t* X, uint32_t batch, const DevPlan& p,
                            hipStream_t st);
// scratch: items * 2N words (conv), batch * N words (ntt)
hipError_t launch_conv_fourstep(int logn, const uint32_t* f, const uint32_t* g, uint32_t* h, uint32_t items,
                                uint64_t item_stride, int32_t* scratch, const DevPlan& p, hipStream_t st);
hipError_t launch_ntt_fourstep(int logn, bool inv, const uint32_t* x, uint32_t* X, uint32_t batch,
                               int32_t* scratch, const DevPlan& p, hipStream_t st);
// scratch: grid * 2N words
hipError_t launch_conv_fused(int logn, const uint32_t* f, const uint32_t* g, uint32_t* h, const uint64_t* offs,
                             uint32_t count, int32_t* scratch, uint32_t grid, const DevPlan& p, hipStream_t st);
int fused_blocks_per_cu(int logn);
hipError_t launch_range_check(const uint32_t* x, uint64_t n, uint32_t m, uint32_t* flag, hipStream_t st);

}  // namespace nttmi
