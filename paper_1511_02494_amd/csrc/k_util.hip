// Cache eviction and HBM bandwidth probes (measurement support).
#include "dev.h"
#include "internal.h"

namespace spmvsel {

// Cache eviction: every 16-byte word of a buffer twice the Infinity Cache's
// size is read with ordinary (allocating) loads, which replaces what the L2s
// and the Infinity Cache hold.  Read only, so that the caches are left with
// clean lines and the next kernel's misses cost no write-backs: a flush that
// rewrites its buffer leaves up to 256 MiB of dirty lines, whose write-back
// then lands inside the kernel that follows.  A thread stores its xor of the
// words only if it equals an arbitrary constant, which keeps the loads.
__global__ __launch_bounds__(kBlock) void k_flush(const u32x4 *__restrict__ p, int64_t n,
                                                  uint32_t *__restrict__ sink) {
    uint32_t acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const u32x4 v = p[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x5bd1e995u) sink[blockIdx.x & 63] = acc;
}

hipError_t launch_flush(void *buf, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(k_flush, dim3(8192), dim3(kBlock), 0, s, (const u32x4 *)buf, n,
                       (uint32_t *)((char *)buf + bytes));
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

// The indexed form of the gather ceiling: what any CSR kernel must at least
// do per nonzero - stream its column index (4 bytes) and value (8 or 4),
// gather x at that column - with no row structure, no sums across threads
// and no y.  Thread t of the grid takes nonzeros t + j T (j < 8, T threads
// in all), so every stream is coalesced; workgroup b gathers from window
// (b mod 8) mod ns as the x-block kernels' XCDs do; the columns are uniform
// random in [0, w) (k_fill_cols).
template <class T>
__global__ __launch_bounds__(kBlock) void k_indexed_probe(const int32_t *__restrict__ col,
                                                          const T *__restrict__ val,
                                                          const T *__restrict__ buf, uint32_t w,
                                                          int ns, int64_t nnz,
                                                          unsigned long long *__restrict__ sink) {
    constexpr int PER = 8;
    const T *__restrict__ win = buf + (size_t)((blockIdx.x % 8) % ns) * w;
    const int64_t TT = (int64_t)gridDim.x * kBlock;
    const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    int32_t c[PER];
    T v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t k = t + j * TT;
        c[j] = k < nnz ? __builtin_nontemporal_load(col + k) : 0;
        v[j] = k < nnz ? __builtin_nontemporal_load(val + k) : T(0);
    }
    T a = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) a ^= v[j] ^ win[c[j]];
    if ((unsigned long long)a == 0x9E3779B97F4A7C15ull) sink[blockIdx.x] = (unsigned long long)a;
}

__global__ __launch_bounds__(kBlock) void k_fill_cols(int32_t *__restrict__ col, int64_t nnz,
                                                      uint32_t w) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock) {
        uint64_t h = ((uint64_t)k + 1) * 0x9E3779B97F4A7C15ull;
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        col[k] = (int32_t)(((h >> 32) * (uint64_t)w) >> 32);
    }
}

hipError_t launch_fill_cols(int32_t *col, int64_t nnz, int64_t w, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_cols, dim3(4096), dim3(kBlock), 0, s, col, nnz, (uint32_t)w);
    return hipGetLastError();
}

hipError_t launch_indexed_probe(const int32_t *col, const void *val, const void *buf, int64_t w,
                                int elem_bytes, int ns, int64_t nnz, unsigned long long *sink,
                                hipStream_t s) {
    const int64_t threads = (nnz + 7) / 8;
    const unsigned g = (unsigned)((threads + kBlock - 1) / kBlock);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_indexed_probe<uint64_t>, dim3(g), dim3(kBlock), 0, s, col,
                           (const uint64_t *)val, (const uint64_t *)buf, (uint32_t)w, ns, nnz, sink);
    else
        hipLaunchKernelGGL(k_indexed_probe<uint32_t>, dim3(g), dim3(kBlock), 0, s, col,
                           (const uint32_t *)val, (const uint32_t *)buf, (uint32_t)w, ns, nnz, sink);
    return hipGetLastError();
}

}  // namespace spmvsel
