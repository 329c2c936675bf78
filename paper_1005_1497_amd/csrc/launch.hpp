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
    const double* TT;    // four-step twiddles TT[u2 * A + t1] = w^(t1 u2) (large N only; the
                         // inverse transforms use them too: they run as forward transforms)
    const uint32_t* TT32;   // the same as 32-bit words (m < 2^32 only)
    ModC M;
    double ninv, ninvq;  // N^-1 mod m and N^-1 / m
    int logn, nmask;
};

// Final store of the fused convolution as the two-prime combination: a1 holds
// the item's residues mod m1 (same element offsets as h); the convolution runs
// mod m2 = the plan's modulus; c = m1^-1 mod m2; h receives 64-bit words.
struct CrtStore {
    const uint32_t* a1;
    uint64_t* h;
    uint32_t m1;
    uint32_t c;
};

constexpr int SMALL_MAX_LOG2N = 12;
// Four-step split of N = 2^n above 2^SMALL_MAX_LOG2N: N = A B with A = 2^fs_la(n)
// (row length) and B = 2^(n - fs_la(n)) (column length).  Shared by the kernels
// and the host tables of the twiddles w^(t1 u2).  Balanced up to 2^16; for
// 2^17..2^19 the columns stay at 256 (two radix-16 passes, 32-column blocks of
// whole cache lines) and the rows take the rest (measured 12-17% faster than
// the balanced 512 x 512 and 1024 x 512 at 2^18 and 2^19); balanced again
// above, where the row pass tables would no longer fit LDS.
constexpr int fs_la(int n) { return (n >= 17 && n <= 19) ? n - 8 : (n + 1) / 2; }
constexpr int MAX_LOG2N = 22;   // no prime below 2^24 has nu = 2^23; 64-bit words use the same kernels

// wbits = 32 (uint32 words, m < 2^24) or 64 (uint64 words, m < 2^46).
// tile: SMALL_TILE_256 (4096/N convolutions per 256-thread workgroup) or
// SMALL_TILE_WAVE (one wave per workgroup up to N = 1024).
enum { SMALL_TILE_256 = 0, SMALL_TILE_WAVE = 1 };
// singular != null: deconvolution, h = inverse(forward(g) / forward(f)); a zero
// forward(f) coefficient sets *singular (convolution otherwise).
hipError_t launch_conv_small(int wbits, int logn, const void* f, const void* g, void* h, const uint64_t* offs,
                             uint32_t count, const DevPlan& p, hipStream_t st, int tile = SMALL_TILE_256,
                             uint32_t* singular = nullptr);
hipError_t launch_ntt_small(int wbits, int logn, bool inv, const void* x, void* X, uint32_t batch, const DevPlan& p,
                            hipStream_t st, const void* y = nullptr);
// scratch: items * 2N scratch words (conv), batch * N (ntt); scratch words are
// wbits/8 bytes.  cus: the device's compute units (the workgroup size is
// halved when 512-thread column blocks would not give each of them one).  tt:
// 0 for that rule, or 256 / 512 threads per workgroup (256 only up to
// 2^FOURSTEP_256_MAX_LOG2N; above it 512).
constexpr int FOURSTEP_256_MAX_LOG2N = 19;
hipError_t launch_conv_fourstep(int wbits, int logn, const void* f, const void* g, void* h, uint32_t items,
                                uint64_t item_stride, void* scratch, const DevPlan& p, hipStream_t st,
                                uint32_t* singular, uint32_t cus, int tt = 0);
hipError_t launch_ntt_fourstep(int wbits, int logn, bool inv, const void* x, void* X, uint32_t batch, void* scratch,
                               const DevPlan& p, hipStream_t st, uint32_t cus);
// scratch: grid * 2N scratch words; queue: two uint32 work-queue words, zero
// before the launch and zero again after it (launches sharing a queue must be
// ordered, e.g. on one stream).  singular != null selects the deconvolution
// (h = g / f in the spectrum; a zero coefficient of f sets *singular).
// crt != null (32-bit words): the result is stored as the combination with
// crt->a1 into crt->h (h itself is not written).
hipError_t launch_conv_fused(int wbits, int logn, const void* f, const void* g, void* h, const uint64_t* offs,
                             uint32_t count, void* scratch, uint32_t* queue, uint32_t grid, const DevPlan& p,
                             hipStream_t st, uint32_t* singular = nullptr, const CrtStore* crt = nullptr);
int fused_blocks_per_cu(int wbits, int logn, int div = 0);
// One launch for a batch of uneven lengths <= 2^multi_max_log2n(wbits).  tasks:
// device array of {uint64 first item; uint32 log2n; uint32 item count} listed
// longest first; toffs: device item offsets in task order; plans: device array
// of DevPlan indexed by log2n; scratch: grid * scratch_words scratch words
// (2N words for the longest length above 2^12).
hipError_t launch_conv_multi(int wbits, const void* f, const void* g, void* h, const void* tasks, uint32_t ntasks,
                             const uint64_t* toffs, void* scratch, uint64_t scratch_words, uint32_t* queue,
                             uint32_t grid, const DevPlan* plans, hipStream_t st);
int multi_max_log2n(int wbits);
int multi_tile(int logn);            // convolutions per task below 2^(SMALL_MAX_LOG2N + 1)
int multi_blocks_per_cu(int wbits);
int fused_threads(int logn);
// h[i] = the integer in [0, m1 m2) that is a1[i] mod m1 and a2[i] mod m2 (m1, m2
// primes below 2^24, a1 < m1, a2 < m2); c = m1^-1 mod m2.
hipError_t launch_crt_combine(const uint32_t* a1, const uint32_t* a2, uint64_t* h, uint64_t n, uint32_t m1,
                              uint32_t m2, uint32_t c, hipStream_t st);
// out (cols x rows) = transpose of in (rows x cols); words of wbits.
hipError_t launch_transpose(int wbits, const void* in, void* out, uint32_t rows, uint32_t cols, hipStream_t st);
// c = a b mod m for n canonical words.
hipError_t launch_pointwise_mul(int wbits, const void* a, const void* b, void* c, uint64_t n, const ModC& M,
                                hipStream_t st);
hipError_t launch_range_check(int wbits, const void* x, uint64_t n, uint64_t m, uint32_t* flag, hipStream_t st);

// Size of the static device scratch (launch_noalloc.hip): the 2N scratch words
// of one four-step convolution up to 2^19 32-bit or 2^18 64-bit words.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)4 << 20;
// Device address of the static scratch on the current device (looked up once
// per device).
hipError_t noalloc_scratch(void** out);

}  // namespace nttmi
