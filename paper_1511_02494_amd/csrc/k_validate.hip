// CSR validation (Section 2 invariants plus the sortedness the features and
// the 16-bit offsets rely on).
//
// flags[0] bit 0: rowptr[0] != 0, rowptr[N] != NNZ, a decrease, or a value
//                 outside [0, NNZ];  bit 1: a column outside [0, M).
// flags[1]: number of pairs (k-1, k) with colind[k] <= colind[k-1];
// flags[2]: how many of those pairs straddle a row start (allowed).
// Columns are strictly increasing inside every row iff flags[1] == flags[2].
// The column passes read rowptr-derived positions only when bit 0 is clear.
#include "dev.h"
#include "internal.h"

namespace spmvsel {

__global__ __launch_bounds__(kBlock) void k_check_rowptr(int64_t n, int64_t nnz,
                                                         const int32_t *__restrict__ rp,
                                                         unsigned long long *flags) {
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i <= n;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t v = rp[i];
        if (v < 0 || v > nnz) bad = true;
        if (i == 0 && v != 0) bad = true;
        if (i == n && v != nnz) bad = true;
        if (i < n && rp[i + 1] < v) bad = true;
    }
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(&flags[0], 1ull);
}

__global__ __launch_bounds__(kBlock) void k_check_cols(int64_t nnz, int64_t m,
                                                       const int32_t *__restrict__ ci,
                                                       unsigned long long *flags) {
    if (flags[0] & 1ull) return;
    bool range = false;
    unsigned long long desc = 0;
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock) {
        const int32_t c = ci[k];
        if (c < 0 || c >= m) range = true;
        if (k > 0 && c <= ci[k - 1]) ++desc;
    }
    if (__ballot(range) != 0 && (threadIdx.x & 63) == 0) atomicOr(&flags[0], 2ull);
    if (desc) atomicAdd(&flags[1], desc);
}

__global__ __launch_bounds__(kBlock) void k_check_rowstarts(int64_t n,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            unsigned long long *flags) {
    if (flags[0] & 1ull) return;
    unsigned long long ok = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t a = rp[i], b = rp[i + 1];
        if (b > a && a >= 1 && ci[a] <= ci[a - 1]) ++ok;
    }
    if (ok) atomicAdd(&flags[2], ok);
}

hipError_t launch_validate(const spmv_plan &P, uint64_t *d_flags, hipStream_t s) {
    unsigned long long *f = reinterpret_cast<unsigned long long *>(d_flags);
    hipError_t e = hipMemsetAsync(f, 0, 3 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    const int64_t cap = (int64_t)P.num_cus * 16;
    auto grid = [&](int64_t items) {
        int64_t g = (items + kBlock - 1) / kBlock;
        return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
    };
    hipLaunchKernelGGL(k_check_rowptr, dim3(grid(P.n + 1)), dim3(kBlock), 0, s, P.n, P.nnz,
                       P.rowptr, f);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (P.nnz > 0) {
        hipLaunchKernelGGL(k_check_cols, dim3(grid(P.nnz)), dim3(kBlock), 0, s, P.nnz, P.m,
                           P.colind, f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (P.n > 0) {
            hipLaunchKernelGGL(k_check_rowstarts, dim3(grid(P.n)), dim3(kBlock), 0, s, P.n,
                               P.rowptr, P.colind, f);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace spmvsel
