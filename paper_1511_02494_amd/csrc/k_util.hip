// Cache eviction and HBM bandwidth probes (measurement support).
#include "dev.h"
#include "internal.h"

namespace spmvsel {

// Read and rewrite every 16-byte word: evicts the Infinity Cache when the
// buffer is twice its size.
__global__ __launch_bounds__(kBlock) void k_flush(u32x4 *__restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        u32x4 v = p[i];
        v.x += 1u;
        p[i] = v;
    }
}

hipError_t launch_flush(void *buf, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(k_flush, dim3(8192), dim3(kBlock), 0, s, (u32x4 *)buf, n);
    return hipGetLastError();
}

// Streaming read: each thread xors its words; one value per block is kept.
__global__ __launch_bounds__(kBlock) void k_read(const u32x4 *__restrict__ p, int64_t n,
                                                 double *__restrict__ sink) {
    unsigned acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const u32x4 a = ld_nt(p + i), b = ld_nt(p + i + stride);
        const u32x4 c = ld_nt(p + i + 2 * stride), d = ld_nt(p + i + 3 * stride);
        acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w;
        acc ^= c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n; i += stride) {
        const u32x4 a = ld_nt(p + i);
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    if (acc == 0x9E3779B9u) sink[blockIdx.x] = (double)acc;  // keeps the loads alive
}

hipError_t launch_read_probe(const void *buf, size_t bytes, double *sink, hipStream_t s) {
    hipLaunchKernelGGL(k_read, dim3(4096), dim3(kBlock), 0, s, (const u32x4 *)buf,
                       (int64_t)(bytes / 16), sink);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_copy(const u32x4 *__restrict__ a,
                                                 u32x4 *__restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        __builtin_nontemporal_store(ld_nt(a + i), b + i);
}

hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(4096), dim3(kBlock), 0, s, (const u32x4 *)src, (u32x4 *)dst,
                       (int64_t)(bytes / 16));
    return hipGetLastError();
}

// Random gathers: the ceiling of an x-gather-bound SpMV.  Workgroup b runs
// on XCD b mod 8 and reads from window (b mod 8) mod ns (windows of w
// elements one after another), as the x-block kernels give each XCD one
// slice of x.  Each thread draws its element indices from a 64-bit linear
// congruential sequence (Knuth's MMIX constants) seeded by its global id,
// ((h >> 32) w) >> 32 being uniform on [0, w), and keeps four gathers in
// flight; the loaded bits are xor-folded so the loads stay live.
template <class T>
__global__ __launch_bounds__(kBlock) void k_gather_probe(const T *__restrict__ buf, uint32_t w,
                                                         int ns, int per_thread,
                                                         unsigned long long *__restrict__ sink) {
    const T *__restrict__ win = buf + (size_t)((blockIdx.x % 8) % ns) * w;
    uint64_t h = ((uint64_t)blockIdx.x * kBlock + threadIdx.x + 1) * 0x9E3779B97F4A7C15ull;
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int k = 0; k < per_thread; k += 4) {
        uint32_t i[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            h = h * 6364136223846793005ull + 1442695040888963407ull;
            i[j] = (uint32_t)(((h >> 32) * (uint64_t)w) >> 32);
        }
        a0 ^= win[i[0]];
        a1 ^= win[i[1]];
        a2 ^= win[i[2]];
        a3 ^= win[i[3]];
    }
    const unsigned long long r = (unsigned long long)(a0 ^ a1 ^ a2 ^ a3);
    if (r == 0x9E3779B97F4A7C15ull) sink[blockIdx.x] = r;
}

hipError_t launch_gather_probe(const void *buf, int64_t w, int elem_bytes, int ns,
                               int64_t gathers, unsigned long long *sink, hipStream_t s) {
    constexpr int per_thread = 8;
    const int64_t threads = (gathers + per_thread - 1) / per_thread;
    const unsigned g = (unsigned)((threads + kBlock - 1) / kBlock);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_gather_probe<uint64_t>, dim3(g), dim3(kBlock), 0, s,
                           (const uint64_t *)buf, (uint32_t)w, ns, per_thread, sink);
    else
        hipLaunchKernelGGL(k_gather_probe<uint32_t>, dim3(g), dim3(kBlock), 0, s,
                           (const uint32_t *)buf, (uint32_t)w, ns, per_thread, sink);
    return hipGetLastError();
}

}  // namespace spmvsel
