// Exact integer accumulators of the structural features (record layout:
// 0 nnz_min, 1 nnz_max, 2 bw_max, 3 S_L2, 4 S_bw, 5/6 S_bw2 lo/hi, 7 S_q,
// 8/9 S_q2 lo/hi, 10 long gaps over all pairs, 11 long gaps at row starts,
// 12/13 delta16 block spans), shared by the feature kernels and the
// one-pass selection kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace spmvsel {
namespace feat {
typedef unsigned __int128 u128;

// Words 12 and 13 carry the largest column span of a row block at the two
// delta16 block heights when the one-pass selection kernel fills them (0
// from k_features).
struct Acc {
    uint64_t lmin, lmax, bwmax, sl2, sbw, sq, gaps, corr, span0, span1;
    u128 sbw2, sq2;
    __device__ void init() {
        lmin = ~0ull; lmax = 0; bwmax = 0; sl2 = 0; sbw = 0; sq = 0; gaps = 0; corr = 0;
        span0 = 0; span1 = 0;
        sbw2 = 0; sq2 = 0;
    }
    __device__ void merge(const Acc &o) {
        lmin = o.lmin < lmin ? o.lmin : lmin;
        lmax = o.lmax > lmax ? o.lmax : lmax;
        bwmax = o.bwmax > bwmax ? o.bwmax : bwmax;
        span0 = o.span0 > span0 ? o.span0 : span0;
        span1 = o.span1 > span1 ? o.span1 : span1;
        sl2 += o.sl2; sbw += o.sbw; sq += o.sq; gaps += o.gaps; corr += o.corr;
        sbw2 += o.sbw2; sq2 += o.sq2;
    }
    __device__ void store(uint64_t *w) const {
        w[0] = lmin; w[1] = lmax; w[2] = bwmax; w[3] = sl2; w[4] = sbw;
        w[5] = (uint64_t)sbw2; w[6] = (uint64_t)(sbw2 >> 64); w[7] = sq;
        w[8] = (uint64_t)sq2; w[9] = (uint64_t)(sq2 >> 64); w[10] = gaps; w[11] = corr;
        w[12] = span0; w[13] = span1; w[14] = w[15] = 0;
    }
    __device__ void load(const uint64_t *w) {
        lmin = w[0]; lmax = w[1]; bwmax = w[2]; sl2 = w[3]; sbw = w[4];
        sbw2 = ((u128)w[6] << 64) | w[5]; sq = w[7]; sq2 = ((u128)w[9] << 64) | w[8];
        gaps = w[10]; corr = w[11]; span0 = w[12]; span1 = w[13];
    }
    // row i = [s, e) of a CSR matrix with sorted columns
    __device__ __forceinline__ void row(const int32_t *__restrict__ ci, int32_t s, int32_t e,
                                        int xb) {
        const uint64_t L = (uint64_t)(e - s);
        lmin = L < lmin ? L : lmin;
        lmax = L > lmax ? L : lmax;
        sl2 += L * L;
        if (L > 0) {
            const int32_t c0 = ci[s], cl = ci[e - 1];
            const uint64_t bw = (uint64_t)(cl - c0);
            const uint64_t q = (L << 31) / (bw + 1);
            bwmax = bw > bwmax ? bw : bwmax;
            sbw += bw;
            sbw2 += (u128)bw * bw;
            sq += q;
            sq2 += (u128)q * q;
            if (s >= 1 && (int64_t)(c0 - ci[s - 1]) * xb > kLineBytes) ++corr;
        }
    }
};

// Tree reduction of the NT threads' accumulators into out (16 words).
template <int NT> __device__ inline void block_reduce_n(Acc &a, uint64_t *out) {
    __shared__ uint64_t sw[NT][16];
    a.store(sw[threadIdx.x]);
    __syncthreads();
    for (int stride = NT / 2; stride > 0; stride >>= 1) {
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

__device__ inline void block_reduce(Acc &a, uint64_t *out) { block_reduce_n<kBlock>(a, out); }

// The 64-thread reduction of nparts partial records into out.
__device__ inline void reduce_partials_64(int nparts, const uint64_t *__restrict__ partials,
                                          uint64_t *out) {
    Acc a;
    a.init();
    for (int b = threadIdx.x; b < nparts; b += 64) {
        Acc o;
        o.load(partials + 16 * b);
        a.merge(o);
    }
    block_reduce_n<64>(a, out);
}

}  // namespace feat
}  // namespace spmvsel
