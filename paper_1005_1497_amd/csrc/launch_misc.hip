// Element-wise kernels: residue (CRT) combination, transpose, pointwise product, range check.
#include "kernels.hpp"

namespace nttmi {

// ------------------------------------------------------------------ residue combination
// Chinese remainder combination of two convolutions modulo the primes m1, m2:
// h = a1 + m1 t, t = ((a2 - a1) m1^-1) mod m2, the unique integer in
// [0, m1 m2) congruent to a1 mod m1 and to a2 mod m2 (exact, in fp64 residues:
// every product is below 2^47).  c = m1^-1 mod m2; M2 the constants of m2.
__global__ void k_crt_combine(const uint32_t* __restrict__ a1, const uint32_t* __restrict__ a2,
                              uint64_t* __restrict__ h, uint64_t n, uint32_t m1, double c, ModC M2) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const double x1 = (double)a1[i];
        const double d = reduce((double)a2[i] - x1, M2);              // a2 - a1 mod m2, |d| <= m2/2 + 2
        double t = mulmod_var(d, c, M2);                              // in [-m2/2 - 2, m2/2 + 2]
        t = (t < 0.0) ? t + M2.m : t;
        t = (t >= M2.m) ? t - M2.m : t;
        h[i] = (uint64_t)x1 + (uint64_t)m1 * (uint64_t)t;
    }
}

hipError_t launch_crt_combine(const uint32_t* a1, const uint32_t* a2, uint64_t* h, uint64_t n, uint32_t m1,
                              uint32_t m2, uint32_t c, hipStream_t st) {
    if (n == 0) return hipSuccess;
    ModC M2;
    M2.m = (double)m2;
    M2.minv = 1.0 / (double)m2;
    M2.C = 6755399441055744.0;
    M2.Cm = M2.C * (double)m2;
    M2.c32 = (double)((1ull << 32) % m2);
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_crt_combine, dim3((uint32_t)blocks), dim3(256), 0, st, a1, a2, h, n, m1, (double)c, M2);
    return hipGetLastError();
}

// ------------------------------------------------------------------ 2-D helpers
// out (cols x rows) = transpose of in (rows x cols), row-major, through a
// padded 32 x 32 LDS tile (coalesced reads and writes); any sizes.
template <class T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ in, T* __restrict__ out, uint32_t rows,
                                                   uint32_t cols) {
    __shared__ T tile[32][33];
    const uint32_t c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const uint32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
    for (uint32_t k = ty; k < 32; k += 8) {
        const uint32_t r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) tile[k][tx] = in[(size_t)r * cols + c];
    }
    __syncthreads();
    for (uint32_t k = ty; k < 32; k += 8) {
        const uint32_t c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) out[(size_t)c * rows + r] = tile[tx][k];
    }
}

// c = a b mod m, canonical, for canonical a, b (transform outputs).
template <class W>
__global__ __launch_bounds__(256) void k_pointwise_mul(const typename W::word* __restrict__ a,
                                                       const typename W::word* __restrict__ b,
                                                       typename W::word* __restrict__ c, uint64_t n, ModC M) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const double x = W::load_reduce(a[i], M), y = W::load_reduce(b[i], M);
        c[i] = W::canon(W::mul_var(x, y, M), M);
    }
}

hipError_t launch_transpose(int wbits, const void* in, void* out, uint32_t rows, uint32_t cols, hipStream_t st) {
    if (rows == 0 || cols == 0) return hipSuccess;
    const dim3 grid((cols + 31) / 32, (rows + 31) / 32);
    if (wbits == 32)
        hipLaunchKernelGGL(k_transpose<uint32_t>, grid, dim3(256), 0, st, (const uint32_t*)in, (uint32_t*)out, rows,
                           cols);
    else
        hipLaunchKernelGGL(k_transpose<uint64_t>, grid, dim3(256), 0, st, (const uint64_t*)in, (uint64_t*)out, rows,
                           cols);
    return hipGetLastError();
}

hipError_t launch_pointwise_mul(int wbits, const void* a, const void* b, void* c, uint64_t n, const ModC& M,
                                hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (wbits == 32)
        hipLaunchKernelGGL(k_pointwise_mul<W32>, dim3((uint32_t)blocks), dim3(256), 0, st, (const uint32_t*)a,
                           (const uint32_t*)b, (uint32_t*)c, n, M);
    else
        hipLaunchKernelGGL(k_pointwise_mul<W64>, dim3((uint32_t)blocks), dim3(256), 0, st, (const uint64_t*)a,
                           (const uint64_t*)b, (uint64_t*)c, n, M);
    return hipGetLastError();
}

// Sets *flag when some x[i] >= m.
template <class T>
__global__ void k_range_check(const T* __restrict__ x, uint64_t n, T m, uint32_t* flag) {
    uint32_t bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        bad |= (x[i] >= m) ? 1u : 0u;
    if (bad) atomicOr(flag, 1u);
}

hipError_t launch_range_check(int wbits, const void* x, uint64_t n, uint64_t m, uint32_t* flag, hipStream_t st) {
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(uint32_t), st);
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (wbits == 32)
        hipLaunchKernelGGL(k_range_check<uint32_t>, dim3((uint32_t)blocks), dim3(256), 0, st, (const uint32_t*)x, n,
                           (uint32_t)m, flag);
    else
        hipLaunchKernelGGL(k_range_check<uint64_t>, dim3((uint32_t)blocks), dim3(256), 0, st, (const uint64_t*)x, n,
                           (uint64_t)m, flag);
    return hipGetLastError();
}

}  // namespace nttmi
