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
#include "internal.h"

namespace spmvsel {

namespace {
typedef unsigned __int128 u128;

struct Acc {
    uint64_t lmin, lmax, bwmax, sl2, sbw, sq, gaps, corr;
    u128 sbw2, sq2;
    __device__ void init() {
        lmin = ~0ull; lmax = 0; bwmax = 0; sl2 = 0; sbw = 0; sq = 0; gaps = 0; corr = 0;
        sbw2 = 0; sq2 = 0;
    }
    __device__ void merge(const Acc &o) {
        lmin = o.lmin < lmin ? o.lmin : lmin;
        lmax = o.lmax > lmax ? o.lmax : lmax;
        bwmax = o.bwmax > bwmax ? o.bwmax : bwmax;
        sl2 += o.sl2; sbw += o.sbw; sq += o.sq; gaps += o.gaps; corr += o.corr;
        sbw2 += o.sbw2; sq2 += o.sq2;
    }
    __device__ void store(uint64_t *w) const {
        w[0] = lmin; w[1] = lmax; w[2] = bwmax; w[3] = sl2; w[4] = sbw;
        w[5] = (uint64_t)sbw2; w[6] = (uint64_t)(sbw2 >> 64); w[7] = sq;
        w[8] = (uint64_t)sq2; w[9] = (uint64_t)(sq2 >> 64); w[10] = gaps; w[11] = corr;
        w[12] = w[13] = w[14] = w[15] = 0;
    }
    __device__ void load(const uint64_t *w) {
        lmin = w[0]; lmax = w[1]; bwmax = w[2]; sl2 = w[3]; sbw = w[4];
        sbw2 = ((u128)w[6] << 64) | w[5]; sq = w[7]; sq2 = ((u128)w[9] << 64) | w[8];
        gaps = w[10]; corr = w[11];
    }
};

__device__ void block_reduce(Acc &a, uint64_t *out) {
    __shared__ uint64_t sw[kBlock][16];
    a.store(sw[threadIdx.x]);
    __syncthreads();
    for (int stride = kBlock / 2; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride) {
            Acc o;
            o.load(sw[threadIdx.x + stride]);
            a.merge(o);
            a.store(sw[threadIdx.x]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a.store(out);
}
}  // namespace

__global__ __launch_bounds__(kBlock) void k_features(int64_t n, int64_t nnz, int xb,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     uint64_t *__restrict__ partials) {
    Acc a;
    a.init();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += stride) {
        const int32_t s = rp[i], e = rp[i + 1];
        const uint64_t L = (uint64_t)(e - s);
        a.lmin = L < a.lmin ? L : a.lmin;
        a.lmax = L > a.lmax ? L : a.lmax;
        a.sl2 += L * L;
        if (L > 0) {
            const int32_t c0 = ci[s], cl = ci[e - 1];
            const uint64_t bw = (uint64_t)(cl - c0);
            const uint64_t q = (L << 31) / (bw + 1);
            a.bwmax = bw > a.bwmax ? bw : a.bwmax;
            a.sbw += bw;
            a.sbw2 += (u128)bw * bw;
            a.sq += q;
            a.sq2 += (u128)q * q;
            if (s >= 1 && (int64_t)(c0 - ci[s - 1]) * xb > kLineBytes) ++a.corr;
        }
    }
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

hipError_t launch_features(const spmv_plan &P, uint64_t *d_partials, uint64_t *d_rec, int xb,
                           hipStream_t s) {
    int64_t items = P.n > P.nnz ? P.n : P.nnz;
    int64_t g = (items + kBlock * 8 - 1) / (kBlock * 8);
    if (g < 1) g = 1;
    if (g > kFeatBlocks) g = kFeatBlocks;
    hipLaunchKernelGGL(k_features, dim3((unsigned)g), dim3(kBlock), 0, s, P.n, P.nnz, xb,
                       P.rowptr, P.colind, d_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_features_final, dim3(1), dim3(kBlock), 0, s, (int)g, d_partials, d_rec);
    return hipGetLastError();
}

}  // namespace spmvsel
