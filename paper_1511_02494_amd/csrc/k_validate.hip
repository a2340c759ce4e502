// CSR validation (Section 2 invariants plus the sortedness the features and
// the 16-bit offsets rely on), one launch over rows and nonzeros.
//
// flags[0] bit 0: rowptr[0] != 0, rowptr[N] != NNZ, a decrease, or a value
//                 outside [0, NNZ];  bit 1: a column outside [0, M).
// flags[1]: number of pairs (k-1, k) with colind[k] <= colind[k-1];
// flags[2]: how many of those pairs straddle the start of a non-empty row.
// Columns are strictly increasing inside every row iff flags[1] == flags[2]
// (and rowptr is valid).  Reads of colind at row starts are made only for
// rows whose two row pointers are themselves within [0, NNZ] and ordered,
// so every access stays in bounds whatever the input.
#include "dev.h"
#include "internal.h"

namespace spmvsel {

constexpr int kValRows = 4;    // rows per thread
constexpr int kValNnz = 8;     // nonzeros per thread

__global__ __launch_bounds__(kBlock) void k_validate(int64_t n, int64_t m, int64_t nnz,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     int64_t row_blocks,
                                                     unsigned long long *flags) {
    bool bad_rp = false, bad_col = false;
    unsigned long long desc = 0, excused = 0;
    if ((int64_t)blockIdx.x < row_blocks) {
        const int64_t i0 = (blockIdx.x * (int64_t)kBlock + threadIdx.x) * kValRows;
        int32_t r[kValRows + 1];
#pragma unroll
        for (int j = 0; j <= kValRows; ++j) r[j] = i0 + j <= n ? rp[i0 + j] : 0;
#pragma unroll
        for (int j = 0; j < kValRows; ++j) {
            const int64_t i = i0 + j;
            if (i > n) break;
            if (r[j] < 0 || r[j] > nnz) bad_rp = true;
            if (i == 0 && r[j] != 0) bad_rp = true;
            if (i == n && r[j] != nnz) bad_rp = true;
            if (i < n && r[j + 1] < r[j]) bad_rp = true;
        }
        if (i0 + kValRows == n && r[kValRows] != nnz) bad_rp = true;
        int32_t cur[kValRows], prev[kValRows];
        bool use[kValRows];
#pragma unroll
        for (int j = 0; j < kValRows; ++j) {
            const int64_t i = i0 + j;
            const int32_t a = r[j], b = r[j + 1];
            use[j] = i < n && a >= 1 && a < b && b <= nnz;
            cur[j] = use[j] ? ci[a] : 0;
            prev[j] = use[j] ? ci[a - 1] : 0;
        }
#pragma unroll
        for (int j = 0; j < kValRows; ++j)
            if (use[j] && cur[j] <= prev[j]) ++excused;
    } else {
        const int64_t k0 = ((blockIdx.x - row_blocks) * (int64_t)kBlock + threadIdx.x) * kValNnz;
        if (k0 < nnz) {
            int32_t c[kValNnz];
            if (k0 + kValNnz <= nnz) {
                load8_nt(ci + k0, c);
            } else {
#pragma unroll
                for (int j = 0; j < kValNnz; ++j) c[j] = k0 + j < nnz ? ci[k0 + j] : INT32_MAX;
            }
            int32_t p = k0 > 0 ? ci[k0 - 1] : INT32_MIN;
#pragma unroll
            for (int j = 0; j < kValNnz; ++j) {
                if (k0 + j >= nnz) break;
                if (c[j] < 0 || c[j] >= m) bad_col = true;
                if (k0 + j > 0 && c[j] <= p) ++desc;
                p = c[j];
            }
        }
    }
    // one atomic per wavefront (counts per thread are at most 8)
    const unsigned long long b_rp = __ballot(bad_rp), b_col = __ballot(bad_col);
    int d = (int)desc, x = (int)excused;
    for (int o = 32; o > 0; o >>= 1) {
        d += __shfl_xor(d, o, 64);
        x += __shfl_xor(x, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (b_rp | b_col) atomicOr(&flags[0], (b_rp ? 1ull : 0ull) | (b_col ? 2ull : 0ull));
        if (d) atomicAdd(&flags[1], (unsigned long long)d);
        if (x) atomicAdd(&flags[2], (unsigned long long)x);
    }
}

hipError_t launch_validate(const spmv_plan &P, uint64_t *d_flags, hipStream_t s) {
    unsigned long long *f = reinterpret_cast<unsigned long long *>(d_flags);
    hipError_t e = hipMemsetAsync(f, 0, 3 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    const int64_t row_blocks = (P.n + 1 + kBlock * kValRows - 1) / (kBlock * kValRows);
    const int64_t nnz_blocks = (P.nnz + kBlock * kValNnz - 1) / (kBlock * kValNnz);
    const int64_t g = row_blocks + nnz_blocks;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)g), dim3(kBlock), 0, s, P.n, P.m, P.nnz,
                       P.rowptr, P.colind, row_blocks, f);
    return hipGetLastError();
}

}  // namespace spmvsel
