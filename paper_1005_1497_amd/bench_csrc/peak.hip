// Measurement helpers for bench.py (not part of the convolution library):
// the sustained vector-ALU rate of the instruction kinds the kernels use,
// measured on the device the caller has made current.
//
// Each thread runs eight independent dependency chains of one instruction
// kind (so every SIMD has enough independent work to issue every cycle), with
// operands that are kernel arguments (nothing folds at compile time); the
// chains' results are written only under a condition the host never meets,
// which keeps them live.  The integer chains are written as single
// instructions (the compiler would otherwise fold repeated additions).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int CHAINS = 8;
constexpr int UNROLL = 16;

__global__ __launch_bounds__(256) void k_fma_f64(double a, double b, uint32_t iters, double* out, uint32_t key) {
    double x[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = (double)(threadIdx.x + c);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) x[c] = __builtin_fma(x[c], a, b);
    }
    double s = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s += x[c];
    if (blockIdx.x == key) out[threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_add_f64(double a, uint32_t iters, double* out, uint32_t key) {
    double x[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = (double)(threadIdx.x + c);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) x[c] = x[c] + a;
    }
    double s = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s += x[c];
    if (blockIdx.x == key) out[threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_add_u32(uint32_t a, uint32_t iters, uint32_t* out, uint32_t key) {
    uint32_t x[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = threadIdx.x + c;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[c]) : "v"(a));
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s ^= x[c];
    if (blockIdx.x == key) out[threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mad_u24(uint32_t a, uint32_t b, uint32_t iters, uint32_t* out, uint32_t key) {
    uint32_t x[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = threadIdx.x + c;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) asm volatile("v_mad_u32_u24 %0, %0, %1, %2" : "+v"(x[c]) : "v"(a), "v"(b));
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s ^= x[c];
    if (blockIdx.x == key) out[threadIdx.x] = s;
}

}  // namespace

extern "C" {

// kind: 0 fp64 FMA, 1 fp64 add, 2 int32 add, 3 int32 24-bit multiply-add
// (mul_u24 + add).  Runs `blocks` workgroups of 256 threads for `iters`
// unrolled iterations on the current device and stream 0; writes the elapsed
// milliseconds and the lane operations executed (an FMA or a multiply-add
// counts one).  Returns 0, or a HIP error code.
int ntt_bench_valu(int kind, uint32_t blocks, uint32_t iters, float* ms, double* lane_ops) {
    void* out = nullptr;
    hipError_t e = hipMalloc(&out, 256 * sizeof(double));
    if (e != hipSuccess) return (int)e;
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    const uint32_t never = 0xFFFFFFFFu;
    auto launch = [&]() {
        switch (kind) {
            case 0: hipLaunchKernelGGL(k_fma_f64, dim3(blocks), dim3(256), 0, 0, 1.0000001, 1e-9, iters, (double*)out, never); break;
            case 1: hipLaunchKernelGGL(k_add_f64, dim3(blocks), dim3(256), 0, 0, 1e-9, iters, (double*)out, never); break;
            case 2: hipLaunchKernelGGL(k_add_u32, dim3(blocks), dim3(256), 0, 0, 12345u, iters, (uint32_t*)out, never); break;
            default: hipLaunchKernelGGL(k_mad_u24, dim3(blocks), dim3(256), 0, 0, 7u, 3u, iters, (uint32_t*)out, never); break;
        }
    };
    launch();   // warm-up (clock ramp, code load)
    e = hipEventRecord(t0, 0);
    launch();
    if (e == hipSuccess) e = hipEventRecord(t1, 0);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, t0, t1);
    if (e == hipSuccess) e = hipGetLastError();
    *lane_ops = (double)blocks * 256.0 * iters * UNROLL * CHAINS;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(out);
    return (int)e;
}

}  // extern "C"
