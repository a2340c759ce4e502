// Seeded synthetic CSR matrices on the device.
//
// Counter-based draws: SplitMix64's output function (Steele, Lea and Flood,
// OOPSLA 2014) on a Weyl sequence:
//   key(seed, s) = fmix(seed*G + s*S + 1),  h(seed, s, i) = fmix(key + (i+1)*G)
// u01(h) = (h >> 11) 2^-53, upm1 = 2 u01 - 1, below(h, n) = ((h >> 32) n) >> 32.
// Columns are drawn one per stratum: a row with L entries over [lo, hi)
// (R = hi - lo) takes one uniform column in each [lo + jR/L, lo + (j+1)R/L).
// Nonzero k (its CSR position) selects its column and value draws.
#include "dev.h"
#include "internal.h"

namespace spmvsel {

namespace {
constexpr uint64_t G = 0x9E3779B97F4A7C15ull, SS = 0xD1B54A32D192ED03ull;
constexpr int ST_X = 1, ST_VAL = 2, ST_LEN = 3, ST_COL = 4, ST_MISC = 5;
typedef unsigned __int128 u128;

__host__ __device__ __forceinline__ uint64_t fmix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t gkey(uint64_t seed, uint64_t s) {
    return fmix(seed * G + s * SS + 1);
}
__device__ __forceinline__ uint64_t hsh(uint64_t key, uint64_t i) { return fmix(key + (i + 1) * G); }
__device__ __forceinline__ double upm1(uint64_t h) {
    return 2.0 * ((double)(h >> 11) * 0x1.0p-53) - 1.0;
}
__device__ __forceinline__ int64_t below(uint64_t h, uint64_t n) {
    return (int64_t)(((h >> 32) * n) >> 32);
}

struct Prm {
    int64_t p[6];
};

// stencil geometry: dims and the (sorted) neighbour offsets of each family
struct Stencil {
    int nd, no;
    int off[27][3];
    double diag, offv;
};

__device__ void stencil_of(int fam, Stencil &S) {
    S.no = 0;
    if (fam == 0 || fam == 1) {
        S.nd = 2;
        for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b) {
                if (fam == 0 && (a != 0) + (b != 0) > 1) continue;
                S.off[S.no][0] = a; S.off[S.no][1] = b; S.off[S.no][2] = 0; ++S.no;
            }
        S.diag = fam == 0 ? 4.0 : 8.0;
    } else {
        S.nd = 3;
        for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b)
                for (int c = -1; c <= 1; ++c) {
                    if (fam == 2 && (a != 0) + (b != 0) + (c != 0) > 1) continue;
                    S.off[S.no][0] = a; S.off[S.no][1] = b; S.off[S.no][2] = c; ++S.no;
                }
        S.diag = fam == 2 ? 6.0 : 26.0;
    }
    S.offv = -1.0;
}

// Largest l in [0, cap] with l^3 (k+1)^2 <= p16^3 2^52, at least 1.
__device__ int64_t pareto_len(uint64_t h, int64_t p16, int64_t cap) {
    const u128 kk = (u128)((h >> 32) + 1);
    const u128 rhs = ((u128)(p16 * p16 * p16)) << 52;
    int64_t lo = 0, hi = cap;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        const u128 l3 = (u128)mid * (u128)mid * (u128)mid;
        if (l3 * kk * kk <= rhs) lo = mid; else hi = mid - 1;
    }
    return lo < 1 ? 1 : lo;
}

__device__ int64_t banded_len(uint64_t h, int64_t d16) {
    const int64_t v = (int64_t)(h >> 32);
    const int64_t L = (d16 * ((1ll << 31) + v) + (1ll << 35)) >> 36;
    return L < 1 ? 1 : L;
}

// row length and column range [lo, hi) of row i for the random families
__device__ void row_shape(int fam, const Prm &P, uint64_t seed, int64_t i, int64_t &L,
                          int64_t &lo, int64_t &hi) {
    const uint64_t kl = gkey(seed, ST_LEN);
    switch (fam) {
    case 4:
        lo = 0; hi = P.p[1];
        L = P.p[2] < hi ? P.p[2] : hi;
        break;
    case 5: {
        const int64_t n = P.p[0], w = P.p[2];
        lo = i - w > 0 ? i - w : 0;
        hi = i + w + 1 < n ? i + w + 1 : n;
        L = banded_len(hsh(kl, i), P.p[1]);
        if (L > hi - lo) L = hi - lo;
        break;
    }
    case 6:
        lo = 0; hi = P.p[0];
        L = banded_len(hsh(kl, i), P.p[1]);
        if (L > hi) L = hi;
        break;
    case 7: {
        const int64_t n = P.p[0], cap = P.p[2];
        lo = 0; hi = n;
        L = pareto_len(hsh(kl, i), P.p[1], cap);
        if (L > n) L = n;
        if (P.p[3] && i == below(hsh(gkey(seed, ST_MISC), 0), (uint64_t)n)) L = cap < n ? cap : n;
        break;
    }
    default: {  // 8: short rows
        const int64_t n = P.p[0];
        lo = i; hi = i + 2;
        L = 1 + (((hsh(kl, i) >> 63) == 0 && i + 1 < n) ? 1 : 0);
        break;
    }
    }
}
}  // namespace

__global__ __launch_bounds__(kBlock) void k_gen_lengths(int fam, Prm P, uint64_t seed, int64_t n,
                                                        int32_t *__restrict__ lens) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int64_t L, lo, hi;
        if (fam <= 3) {
            Stencil S;
            stencil_of(fam, S);
            const int64_t side = P.p[0];
            int64_t c[3];
            int64_t r = i;
            for (int a = S.nd - 1; a >= 0; --a) { c[a] = r % side; r /= side; }
            L = 0;
            for (int o = 0; o < S.no; ++o) {
                bool ok = true;
                for (int a = 0; a < S.nd; ++a) {
                    const int64_t v = c[a] + S.off[o][a];
                    ok = ok && v >= 0 && v < side;
                }
                L += ok;
            }
        } else {
            row_shape(fam, P, seed, i, L, lo, hi);
        }
        lens[i] = (int32_t)L;
    }
}

__global__ __launch_bounds__(kBlock) void k_gen_fill(int fam, Prm P, uint64_t seed, int64_t n,
                                                     const int32_t *__restrict__ rp,
                                                     int32_t *__restrict__ ci,
                                                     double *__restrict__ val) {
    const uint64_t kc = gkey(seed, ST_COL), kv = gkey(seed, ST_VAL);
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int64_t k = rp[i];
        if (fam <= 3) {
            Stencil S;
            stencil_of(fam, S);
            const int64_t side = P.p[0];
            const bool rnd = P.p[1] != 0;
            int64_t c[3];
            int64_t r = i;
            for (int a = S.nd - 1; a >= 0; --a) { c[a] = r % side; r /= side; }
            for (int o = 0; o < S.no; ++o) {
                bool ok = true;
                int64_t col = 0;
                for (int a = 0; a < S.nd; ++a) {
                    const int64_t v = c[a] + S.off[o][a];
                    ok = ok && v >= 0 && v < side;
                    col = col * side + v;
                }
                if (!ok) continue;
                ci[k] = (int32_t)col;
                val[k] = rnd ? upm1(hsh(kv, (uint64_t)k)) : (col == i ? S.diag : S.offv);
                ++k;
            }
        } else {
            int64_t L, lo, hi;
            row_shape(fam, P, seed, i, L, lo, hi);
            const int64_t R = hi - lo;
            for (int64_t j = 0; j < L; ++j, ++k) {
                int64_t col;
                if (fam == 8) {
                    col = i + j;
                } else {
                    const int64_t st = (j * R) / L;
                    const int64_t w = ((j + 1) * R) / L - st;
                    col = lo + st + below(hsh(kc, (uint64_t)k), (uint64_t)w);
                }
                ci[k] = (int32_t)col;
                val[k] = upm1(hsh(kv, (uint64_t)k));
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_gen_vector(int64_t n, uint64_t seed,
                                                       double *__restrict__ x) {
    const uint64_t kx = gkey(seed, ST_X);
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        x[i] = upm1(hsh(kx, (uint64_t)i));
}

static unsigned grid_of(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

hipError_t launch_gen_lengths(int family, const int64_t *prm, uint64_t seed, int64_t n,
                              int32_t *lens, hipStream_t s) {
    Prm P;
    for (int i = 0; i < 6; ++i) P.p[i] = prm[i];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_lengths, dim3(grid_of(n)), dim3(kBlock), 0, s, family, P, seed, n, lens);
    return hipGetLastError();
}

hipError_t launch_gen_fill(int family, const int64_t *prm, uint64_t seed, int64_t n,
                           const int32_t *rowptr, int32_t *colind, double *val, hipStream_t s) {
    Prm P;
    for (int i = 0; i < 6; ++i) P.p[i] = prm[i];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_fill, dim3(grid_of(n)), dim3(kBlock), 0, s, family, P, seed, n,
                       rowptr, colind, val);
    return hipGetLastError();
}

hipError_t launch_gen_vector(int64_t n, uint64_t seed, double *x, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_vector, dim3(grid_of(n)), dim3(kBlock), 0, s, n, seed, x);
    return hipGetLastError();
}

// ---- exclusive scans of row lengths into row pointers, for `segs`
// independent arrays at once (input s at lens + s*n, output s at
// rowptr + s*(n+1)); int64 block sums, the caller checks that totals fit
// below 2^31.  Per segment: tile sums, a scan of the tile sums by one block,
// then each tile's scan.
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

// Exclusive scan of v over the block (all threads take part); returns this
// thread's exclusive prefix and sets *total to the block's sum.
__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t *sh, int64_t *total) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const int64_t t = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const int64_t incl = sh[threadIdx.x];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(const int32_t *__restrict__ in, int64_t n,
                                                      int64_t nb, int64_t *__restrict__ sums) {
    __shared__ int64_t red[kBlock];
    const int64_t seg = blockIdx.x / nb, b = blockIdx.x % nb;
    in += seg * n;
    const int64_t base = b * kScanTile;
    int64_t s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j * kBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[seg * (nb + 1) + b] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_scan_top(int64_t *sums, int64_t nb, int64_t *totals) {
    __shared__ int64_t sh[kBlock];
    int64_t *sg = sums + blockIdx.x * (nb + 1);
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kBlock) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nb ? sg[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, sh, &tot);
        if (i < nb) sg[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        sg[nb] = carry;
        if (totals) totals[blockIdx.x] = carry;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const int32_t *__restrict__ in, int64_t n,
                                                       int64_t nb,
                                                       const int64_t *__restrict__ sums,
                                                       int32_t *__restrict__ out) {
    __shared__ int64_t sh[kBlock];
    const int64_t seg = blockIdx.x / nb, b = blockIdx.x % nb;
    in += seg * n;
    out += seg * (n + 1);
    const int64_t base = b * kScanTile;
    int64_t carry = sums[seg * (nb + 1) + b];
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j * kBlock + threadIdx.x;
        const int64_t v = i < n ? in[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, sh, &tot);
        if (i < n) out[i + 1] = (int32_t)(carry + ex + v);
        carry += tot;
    }
    if (b == 0 && threadIdx.x == 0) out[0] = 0;
}

hipError_t launch_exclusive_scan_i32(const int32_t *lens, int32_t *rowptr, int64_t n, int segs,
                                     int64_t *totals, void *tmp, size_t tmp_bytes, hipStream_t s,
                                     size_t *tmp_needed) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    const size_t need = (size_t)(nb + 1) * 8 * (size_t)segs;
    if (tmp_needed) *tmp_needed = need;
    if (!tmp) return hipSuccess;
    if (tmp_bytes < need || segs < 1) return hipErrorInvalidValue;
    if (nb == 0) {  // n == 0: every output is the single entry 0
        hipError_t e = hipMemsetAsync(rowptr, 0, 4 * (size_t)segs, s);
        if (e == hipSuccess) e = hipMemsetAsync(tmp, 0, need, s);  // segment totals
        if (e == hipSuccess && totals) e = hipMemsetAsync(totals, 0, 8 * (size_t)segs, s);
        return e;
    }
    int64_t *sums = static_cast<int64_t *>(tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)(nb * segs)), dim3(kBlock), 0, s, lens, n, nb,
                       sums);
    hipLaunchKernelGGL(k_scan_top, dim3((unsigned)segs), dim3(kBlock), 0, s, sums, nb, totals);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)(nb * segs)), dim3(kBlock), 0, s, lens, n, nb,
                       sums, rowptr);
    return hipGetLastError();
}

}  // namespace spmvsel
