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

constexpr int kValRows = 4;    // rows per work item
constexpr int kValNnz = 8;     // nonzeros per work item

// Work items: row groups of kValRows rows first, then nonzero groups of
// kValNnz, taken grid-stride.  Block b writes (error bits, descents,
// excused descents) to part[3b .. 3b+2]; k_validate_final adds them.
__global__ __launch_bounds__(kBlock) void k_validate(int64_t n, int64_t m, int64_t nnz,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     unsigned long long *__restrict__ part) {
    bool bad_rp = false, bad_col = false;
    unsigned long long desc = 0, excused = 0;
    const int64_t row_items = (n + 1 + kValRows - 1) / kValRows;
    const int64_t items = row_items + (nnz + kValNnz - 1) / kValNnz;
    for (int64_t w = blockIdx.x * (int64_t)kBlock + threadIdx.x; w < items;
         w += (int64_t)gridDim.x * kBlock) {
        if (w < row_items) {
            const int64_t i0 = w * kValRows;
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
            const int64_t k0 = (w - row_items) * kValNnz;
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
    __shared__ unsigned long long sh[3][kBlock / 64];
    const unsigned long long b_rp = __ballot(bad_rp), b_col = __ballot(bad_col);
    unsigned long long d = desc, x = excused;
    for (int o = 32; o > 0; o >>= 1) {
        d += __shfl_xor(d, o, 64);
        x += __shfl_xor(x, o, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][wv] = (b_rp ? 1ull : 0ull) | (b_col ? 2ull : 0ull);
        sh[1][wv] = d;
        sh[2][wv] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long f = 0, dd = 0, xx = 0;
        for (int q = 0; q < kBlock / 64; ++q) {
            f |= sh[0][q];
            dd += sh[1][q];
            xx += sh[2][q];
        }
        part[3 * blockIdx.x] = f;
        part[3 * blockIdx.x + 1] = dd;
        part[3 * blockIdx.x + 2] = xx;
    }
}

__global__ __launch_bounds__(kBlock) void k_validate_final(int nparts,
                                                           const unsigned long long *__restrict__ part,
                                                           unsigned long long *__restrict__ flags) {
    __shared__ unsigned long long sh[3][kBlock];
    unsigned long long f = 0, d = 0, x = 0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
        f |= part[3 * b];
        d += part[3 * b + 1];
        x += part[3 * b + 2];
    }
    sh[0][threadIdx.x] = f;
    sh[1][threadIdx.x] = d;
    sh[2][threadIdx.x] = x;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sh[0][threadIdx.x] |= sh[0][threadIdx.x + st];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        flags[0] = sh[0][0];
        flags[1] = sh[1][0];
        flags[2] = sh[2][0];
    }
}

hipError_t launch_validate(const spmv_plan &P, uint64_t *d_flags, uint64_t *d_part,
                           hipStream_t s) {
    unsigned long long *f = reinterpret_cast<unsigned long long *>(d_flags);
    unsigned long long *part = reinterpret_cast<unsigned long long *>(d_part);
    const int64_t items = (P.n + 1 + kValRows - 1) / kValRows + (P.nnz + kValNnz - 1) / kValNnz;
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g > kValGrid) g = kValGrid;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)g), dim3(kBlock), 0, s, P.n, P.m, P.nnz,
                       P.rowptr, P.colind, part);
    hipLaunchKernelGGL(k_validate_final, dim3(1), dim3(kBlock), 0, s, (int)g, part, f);
    return hipGetLastError();
}

}  // namespace spmvsel
