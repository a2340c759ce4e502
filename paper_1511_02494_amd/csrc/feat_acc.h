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

// The 64-thread reduction of nparts partial records into out.  Each thread
// loads four records before merging them, so that four round trips to the
// records (written by workgroups on every XCD) are in flight at once instead
// of one; the merge is exact integer arithmetic, so its order does not
// change the result.
__device__ inline void reduce_partials_64(int nparts, const uint64_t *__restrict__ partials,
                                          uint64_t *out) {
    constexpr int U = 4;
    Acc a;
    a.init();
    int b = threadIdx.x;
    for (; b + 64 * (U - 1) < nparts; b += 64 * U) {
        Acc o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) o[u].load(partials + 16 * (b + 64 * u));
#pragma unroll
        for (int u = 0; u < U; ++u) a.merge(o[u]);
    }
    for (; b < nparts; b += 64) {
        Acc o;
        o.load(partials + 16 * b);
        a.merge(o);
    }
    block_reduce_n<64>(a, out);
}


// ---------------------------------------------------------------- device finalisation
// The twelve features from the exact integer record (words as above, the
// miss count as word 10 minus word 11), by the same sequence of IEEE double
// operations as the host finalisation: u128 numerators rounded to double
// once (with a sticky bit), correctly rounded division and square root.  So
// a selection can take the features on the device without a host round trip
// and get the same bits.
__device__ __forceinline__ double u128_to_double_dev(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    if (hi == 0) return (double)lo;
    const int sh = 64 - __builtin_clzll(hi);
    const uint64_t top = (uint64_t)(v >> sh);
    const uint64_t sticky = (v & (((u128)1 << sh) - 1)) != 0 ? 1 : 0;
    return ldexp((double)(top | sticky), sh);
}

__device__ inline void finalize_features_dev(const uint64_t *w, int64_t n, int64_t m, int64_t nnz,
                                             int vb, int xb, double *f) {
    for (int i = 0; i < 12; ++i) f[i] = 0.0;
    if (n == 0) return;
    const double f0 = (double)n, f1 = (double)nnz, nn = f0 * f0;
    const u128 sl2 = w[3], sbw = w[4], sbw2 = ((u128)w[6] << 64) | w[5];
    const u128 sq = w[7], sq2 = ((u128)w[9] << 64) | w[8];
    const int64_t smiss = (int64_t)(w[10] - w[11]);
    f[0] = f0;
    f[1] = f1;
    f[2] = f1 / f0;
    f[3] = sqrt(u128_to_double_dev((u128)n * sl2 - (u128)nnz * (u128)nnz) / nn);
    f[4] = (double)w[1];
    f[5] = (double)w[0];
    f[6] = (double)(uint64_t)sbw / f0;
    f[7] = sqrt(u128_to_double_dev((u128)n * sbw2 - sbw * sbw) / nn);
    f[8] = ((double)(uint64_t)sq / 2147483648.0) / f0;
    f[9] = sqrt(u128_to_double_dev((u128)n * sq2 - sq * sq) / 4611686018427387904.0 / nn);
    f[10] = nnz > 0 ? (double)smiss / f1 : 0.0;
    const int64_t ws = 4 * (n + 1) + (4 + vb) * nnz + (int64_t)xb * m + (int64_t)xb * n;
    f[11] = ws <= kLlcBytes ? 1.0 : 0.0;
}

// plog2(v) = (e - 1) + (2m - 1) for (m, e) = frexp(v): a piecewise-linear
// log2 that every implementation computes exactly (the selectors' map of the
// first eight features, g_k = plog2(1 + f_k)).
__device__ __forceinline__ double plog2(double v) {
    int e;
    const double m = frexp(v, &e);
    return (double)(e - 1) + (2.0 * m - 1.0);
}

// The one-pass selection's first step on 64 threads: the reduced record into
// w (shared), the features into f (shared), the feasibility bits (feas_base,
// plus delta16 when a block span fits 16 bits: word 12 at the short_row
// height, word 13 at 256 rows when two_heights) into *feas; ends with a
// workgroup barrier.
__device__ inline void select_prologue(int nparts, const uint64_t *__restrict__ partials, int64_t n,
                                       int64_t m, int64_t nnz, int vb, int xb, int two_heights,
                                       uint32_t feas_base, uint64_t *w, double *f, uint32_t *feas) {
    reduce_partials_64(nparts, partials, w);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (n == 0) w[0] = 0;
        finalize_features_dev(w, n, m, nnz, vb, xb, f);
        const bool d16 = w[12] <= 65535ull || (two_heights && w[13] <= 65535ull);
        *feas = feas_base | (d16 ? (1u << V_DELTA16) : 0u);
    }
    __syncthreads();
}

// The selector-independent part of a one-pass selection record (bytes):
// 0..127 the selector's own result, 128 the feasibility bits, 192..287 the
// twelve features (doubles), 288..415 the reduced record (16 words).
constexpr int kRecFeas = 128, kRecFeatures = 192, kRecWords = 288, kRecBytes = 416;

__device__ inline void select_store_common(char *out, const double *f, uint32_t feas,
                                           const uint64_t *w) {
    *reinterpret_cast<uint32_t *>(out + kRecFeas) = feas;
    double *fo = reinterpret_cast<double *>(out + kRecFeatures);
    for (int i = 0; i < 12; ++i) fo[i] = f[i];
    uint64_t *wo = reinterpret_cast<uint64_t *>(out + kRecWords);
    for (int i = 0; i < 16; ++i) wo[i] = w[i];
}

}  // namespace feat
}  // namespace spmvsel
