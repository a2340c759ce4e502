// Structural features of Table 1 as exact integer sums (one pass).
//
// Per row i (L_i nonzeros, sorted columns c_0 < ... < c_{L-1}):
//   bw_i = c_{L-1} - c_0 (0 for L_i <= 1),
//   q_i  = floor(2^31 L_i / (bw_i + 1)) (dispersion L/(bw+1) in Q31, 0 if empty).
// Misses (a gap of more than 128 bytes of x between consecutive nonzeros of a
// row) are counted as: all adjacent pairs (k-1, k) over the whole colind
// array whose gap exceeds the line, minus those pairs where k starts a
// non-empty row.  Every sum is an exact integer, so the block partials can
// be combined in any order.
//
// Record words: 0 nnz_min, 1 nnz_max, 2 bw_max, 3 S_L2, 4 S_bw, 5/6 S_bw2
// (lo/hi), 7 S_q, 8/9 S_q2 (lo/hi), 10 long gaps (all pairs), 11 long gaps at
// row starts.
#include "dev.h"
#include "feat_acc.h"
#include "internal.h"

namespace spmvsel {
using namespace feat;


__global__ __launch_bounds__(kBlock) void k_features(int64_t n, int64_t nnz, int xb,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     uint64_t *__restrict__ partials) {
    Acc a;
    a.init();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += stride)
        a.row(ci, rp[i], rp[i + 1], xb);
    for (int64_t k = 1 + blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nnz; k += stride)
        if ((int64_t)(ci[k] - ci[k - 1]) * xb > kLineBytes) ++a.gaps;
    block_reduce(a, partials + 16 * blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_features_final(int nparts,
                                                           const uint64_t *__restrict__ partials,
                                                           uint64_t *__restrict__ rec) {
    Acc a;
    a.init();
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
        Acc o;
        o.load(partials + 16 * b);
        a.merge(o);
    }
    block_reduce(a, rec);
}

// one row (and one nonzero) per thread up to kFeatBlocks workgroups: a small
// matrix is then one round of dependent loads, not several
hipError_t launch_features(const spmv_plan &P, uint64_t *d_partials, uint64_t *d_rec, int xb,
                           hipStream_t s) {
    int64_t items = P.n > P.nnz ? P.n : P.nnz;
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > kFeatBlocks) g = kFeatBlocks;
    hipLaunchKernelGGL(k_features, dim3((unsigned)g), dim3(kBlock), 0, s, P.n, P.nnz, xb,
                       P.rowptr, P.colind, d_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_features_final, dim3(1), dim3(kBlock), 0, s, (int)g, d_partials, d_rec);
    return hipGetLastError();
}

// ---------------------------------------------------------------- one-pass selection
// The feature sums of k_features and the delta16 block spans in one pass
// over the rows.  Blocks of H0 = R * 256 rows are walked by workgroups in
// turn; thread t takes rows t, t + 256, ..., t + (R - 1) 256 of a block, so
// its k-th row lies in 256-row sub-block k.  Each sub-block's window [min
// first column, max last column] gives its span at H1 = 256, their union the
// block's span at H0 (the windows k_panel_windows computes); the largest go
// to words 12 (H0) and 13 (H1) of the partial records.  The rows' feature
// sums and the nonzero gap count are the same integers as k_features's, in
// another grouping.
template <int R>
__global__ __launch_bounds__(kBlock) void k_select_pass(int64_t n, int64_t nnz, int xb,
                                                        const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        uint64_t *__restrict__ partials) {
    __shared__ int32_t wlo[R][kBlock / 64], whi[R][kBlock / 64];
    Acc a;
    a.init();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t blocks0 = (n + R * kBlock - 1) / (R * kBlock);
    for (int64_t p = blockIdx.x; p < blocks0; p += gridDim.x) {
        int32_t lo[R], hi[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            lo[k] = INT32_MAX;
            hi[k] = -1;
            const int64_t i = p * (R * kBlock) + k * kBlock + threadIdx.x;
            if (i < n) {
                const int32_t s = rp[i], e = rp[i + 1];
                a.row(ci, s, e, xb);
                if (s < e) {
                    lo[k] = ci[s];
                    hi[k] = ci[e - 1];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            for (int o = 32; o > 0; o >>= 1) {
                const int32_t lo2 = __shfl_xor(lo[k], o, 64), hi2 = __shfl_xor(hi[k], o, 64);
                lo[k] = lo2 < lo[k] ? lo2 : lo[k];
                hi[k] = hi2 > hi[k] ? hi2 : hi[k];
            }
            if (lane == 0) {
                wlo[k][wv] = lo[k];
                whi[k][wv] = hi[k];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t l0 = INT32_MAX, h0 = -1;
            for (int k = 0; k < R; ++k) {
                int32_t l1 = INT32_MAX, h1 = -1;
                for (int w = 0; w < kBlock / 64; ++w) {
                    l1 = wlo[k][w] < l1 ? wlo[k][w] : l1;
                    h1 = whi[k][w] > h1 ? whi[k][w] : h1;
                }
                const uint64_t d = h1 < 0 ? 0 : (uint64_t)(h1 - l1);
                a.span1 = d > a.span1 ? d : a.span1;
                l0 = l1 < l0 ? l1 : l0;
                h0 = h1 > h0 ? h1 : h0;
            }
            const uint64_t d = h0 < 0 ? 0 : (uint64_t)(h0 - l0);
            a.span0 = d > a.span0 ? d : a.span0;
        }
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = 1 + blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nnz; k += stride)
        if ((int64_t)(ci[k] - ci[k - 1]) * xb > kLineBytes) ++a.gaps;
    block_reduce(a, partials + 16 * blockIdx.x);
}

int launch_select_pass(const spmv_plan &P, int R, uint64_t *d_partials, int xb, hipStream_t s,
                       hipError_t *err) {
    const int64_t blocks0 = (P.n + (int64_t)R * kBlock - 1) / ((int64_t)R * kBlock);
    const int64_t by_nnz = (P.nnz + kBlock - 1) / kBlock;
    int64_t g = blocks0 > by_nnz ? blocks0 : by_nnz;
    g = g < 1 ? 1 : g > kFeatBlocks ? kFeatBlocks : g;
    const dim3 grid((unsigned)g), blk(kBlock);
    switch (R) {
    case 1: hipLaunchKernelGGL(k_select_pass<1>, grid, blk, 0, s, P.n, P.nnz, xb, P.rowptr, P.colind, d_partials); break;
    case 2: hipLaunchKernelGGL(k_select_pass<2>, grid, blk, 0, s, P.n, P.nnz, xb, P.rowptr, P.colind, d_partials); break;
    case 4: hipLaunchKernelGGL(k_select_pass<4>, grid, blk, 0, s, P.n, P.nnz, xb, P.rowptr, P.colind, d_partials); break;
    case 8: hipLaunchKernelGGL(k_select_pass<8>, grid, blk, 0, s, P.n, P.nnz, xb, P.rowptr, P.colind, d_partials); break;
    default: *err = hipErrorInvalidValue; return 0;
    }
    *err = hipGetLastError();
    return (int)g;
}

}  // namespace spmvsel
