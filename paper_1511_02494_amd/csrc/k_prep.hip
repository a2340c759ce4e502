// Format preparation for the variants (built once per plan, lazily).
#include "dev.h"
#include "internal.h"

namespace spmvsel {

// ---- delta16: off_k = c_k - base[row(k) / H], base = the block's smallest
// column (from the panel windows with H rows per panel).  A sub-wavefront
// of W lanes per row.
template <int W>
__global__ __launch_bounds__(kBlock) void k_delta16_encode(int64_t n, int H,
                                                           const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const int32_t *__restrict__ base,
                                                           uint16_t *__restrict__ off) {
    const int lane = threadIdx.x & (W - 1);
    const int64_t nsub = (int64_t)gridDim.x * (kBlock / W);
    for (int64_t i = blockIdx.x * (int64_t)(kBlock / W) + threadIdx.x / W; i < n; i += nsub) {
        const int32_t a = rp[i], b = rp[i + 1];
        const int32_t b0 = base[i / H];
        for (int32_t k = a + lane; k < b; k += W) off[k] = (uint16_t)(ci[k] - b0);
    }
}

hipError_t launch_delta16_encode(const spmv_plan &P, const int32_t *base, uint16_t *off, hipStream_t s) {
    if (P.n == 0) return hipSuccess;
    const int W = P.vec_width;
    int64_t g = (P.n + (kBlock / W) - 1) / (kBlock / W);
    if (g > (int64_t)P.num_cus * 32) g = (int64_t)P.num_cus * 32;
    switch (W) {
#define ENC(WW) case WW: hipLaunchKernelGGL((k_delta16_encode<WW>), dim3((unsigned)g), dim3(kBlock), 0, s, P.n, P.d16_rows, P.rowptr, P.colind, base, off); break;
        ENC(2) ENC(4) ENC(8) ENC(16) ENC(32) ENC(64)
#undef ENC
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- delta16, sliced layout.  Slice s = rows [64 s, 64 s + 64), one per
// lane of a wavefront.  Offset slices: width = the longest row rounded up to
// an even count, reference column = the smallest column of the slice; the
// k-th nonzero of the row in lane l is stored at slot
//   128 units[s] + 128 (k / 2) + 2 l + (k % 2)
// (units = exclusive prefix sums of the half widths), so lane l reads its
// nonzeros in pairs and a wavefront's pair load is 64 consecutive pairs.
// Diagonal slices (see internal.h) use the same slots with k = the index of
// the nonzero's diagonal c - r among the slice's sorted diagonals.
__global__ __launch_bounds__(kBlock) void k_sliced_shape(int64_t n, int64_t nsl,
                                                         const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const int32_t *__restrict__ perm,
                                                         int32_t *__restrict__ width,
                                                         int32_t *__restrict__ halfw,
                                                         int32_t *__restrict__ base,
                                                         int32_t *__restrict__ kind,
                                                         int32_t *__restrict__ diag,
                                                         int32_t *__restrict__ snnz,
                                                         int32_t *__restrict__ span) {
    constexpr int kWaves = kBlock / kSellRows;
    __shared__ int32_t s_ci[kWaves][kSellRows * kSellMaxDiag];  // a slice's nonzeros
    const int wv = threadIdx.x / kSellRows;
    const int64_t sl = blockIdx.x * (int64_t)kWaves + wv;
    const bool live = sl < nsl;  // (no early exit: every thread reaches the barrier)
    const int lane = threadIdx.x & (kSellRows - 1);
    const int64_t pos = sl * kSellRows + lane;
    // the row at this position (sorted layout: perm; else the position)
    const int64_t r = perm && live && pos < n ? perm[pos] : pos;
    int32_t a = 0, e = 0;
    if (live && pos < n) {
        a = rp[r];
        e = rp[r + 1];
    }
    int len = e - a, first = len > 0 ? ci[a] : INT32_MAX, cnt = len;
    int last = len > 0 ? ci[e - 1] : -1;  // columns increase along a row
#pragma unroll
    for (int d = kSellRows / 2; d > 0; d >>= 1) {
        const int ol = __shfl_xor(len, d, kSellRows);
        const int of = __shfl_xor(first, d, kSellRows);
        const int oz = __shfl_xor(last, d, kSellRows);
        cnt += __shfl_xor(cnt, d, kSellRows);
        len = ol > len ? ol : len;
        first = of < first ? of : first;
        last = oz > last ? oz : last;
    }
    const int w_off = len + (len & 1);
    // A slice with a row longer than 32 has more than 32 diagonals.  Else its
    // nonzeros (at most 64 x 32) are staged in LDS with coalesced loads.  The
    // sorted layout has offset slices only.
    const bool maybe = live && len <= kSellMaxDiag && !perm;
    const int32_t A = live ? rp[sl * kSellRows] : 0;
    const int32_t E = live ? rp[(sl + 1) * kSellRows < n ? (sl + 1) * kSellRows : n] : 0;
    if (maybe)
        for (int32_t i = lane; i < E - A; i += kSellRows) s_ci[wv][i] = ci[A + i];
    __syncthreads();
    // the slice's distinct diagonals in increasing order: each round takes
    // the smallest head c - r over the lanes (c - r fits int32; INT32_MAX
    // marks an exhausted lane, so a row reaching that diagonal, possible only
    // for column 2^31 - 1 of row 0, makes the slice an offset slice), and the
    // lanes holding it move on
    int32_t p = a, mine = 0, D = 0;
    bool fits = maybe;
    if (maybe)
        fits = wave_min(e > a && s_ci[wv][e - 1 - A] - (int32_t)r == INT32_MAX ? 0 : 1) == 1;
    while (fits) {
        const int32_t head = p < e ? s_ci[wv][p - A] - (int32_t)r : INT32_MAX;
        const int32_t m = wave_min(head);
        if (m == INT32_MAX) break;
        if (D >= kSellMaxDiag) {
            fits = false;
            break;
        }
        if (lane == D) mine = m;
        ++D;
        if (head == m) ++p;
    }
    if (!live) return;
    const int d_even = D + (D & 1);
    const bool is_diag = fits && d_even <= w_off;
    if (lane < kSellMaxDiag) diag[sl * kSellMaxDiag + lane] = is_diag && lane < D ? mine : 0;
    if (lane == 0) {
        const int w = is_diag ? d_even : w_off;
        width[sl] = w;
        halfw[sl] = w / 2;
        base[sl] = first == INT32_MAX ? 0 : first;
        kind[sl] = is_diag ? 1 + D : 0;
        snnz[sl] = cnt;
        span[sl] = cnt > 0 ? last - first : 0;  // largest offset c - base
    }
}

hipError_t launch_sliced_shape(const spmv_plan &P, const int32_t *perm, int32_t *width,
                               int32_t *halfw, int32_t *base, int32_t *kind, int32_t *diag,
                               int32_t *snnz, int32_t *span, hipStream_t s) {
    const int64_t nsl = (P.n + kSellRows - 1) / kSellRows;
    if (nsl == 0) return hipSuccess;
    const int64_t per = kBlock / kSellRows;
    hipLaunchKernelGGL(k_sliced_shape, dim3((unsigned)((nsl + per - 1) / per)), dim3(kBlock), 0, s,
                       P.n, nsl, P.rowptr, P.colind, perm, width, halfw, base, kind, diag, snnz,
                       span);
    return hipGetLastError();
}

// Row order of the length-sorted sliced layout: inside each window of
// kBlock rows, the rows by decreasing length, ties in row order (a row's
// position is the number of rows of its window that come before it).
// perm[p] = the row at position p, pinv[r] = the position of row r.
__global__ __launch_bounds__(kBlock) void k_sell_perm(int64_t n, const int32_t *__restrict__ rp,
                                                      int32_t *__restrict__ perm,
                                                      int32_t *__restrict__ pinv) {
    __shared__ int32_t s_len[kBlock];
    const int64_t r0 = (int64_t)blockIdx.x * kBlock;
    const int t = threadIdx.x;
    const int64_t r = r0 + t;
    const int32_t mine = r < n ? rp[r + 1] - rp[r] : -1;  // past the end: after every row
    s_len[t] = mine;
    __syncthreads();
    if (r >= n) return;
    int rank = 0;
    for (int u = 0; u < kBlock; ++u) {
        const int32_t l = s_len[u];
        rank += (l > mine || (l == mine && u < t)) ? 1 : 0;
    }
    perm[r0 + rank] = (int32_t)r;
    pinv[r] = (int32_t)(r0 + rank);
}

hipError_t launch_sell_perm(const spmv_plan &P, int32_t *perm, int32_t *pinv, hipStream_t s) {
    if (P.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sell_perm, dim3((unsigned)((P.n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, P.n, P.rowptr, perm, pinv);
    return hipGetLastError();
}

// One workgroup per kBlock rows (kBlock / 64 slices): thread t takes the
// block's nonzeros t, t + kBlock, ... (coalesced reads) and finds its row by
// a binary search of the block's row pointers in LDS.  In an offset slice
// it writes its offset and value; in a diagonal slice it finds its diagonal
// among the slice's (in LDS) by a binary search, writes its value to that
// position and sets the diagonal's bit in the row's mask (LDS atomics; the
// masks are stored once at the end, zero for rows of offset slices).
template <class V>
__global__ __launch_bounds__(kBlock) void k_sliced_scatter(int64_t n, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const V *__restrict__ val,
                                                           const int32_t *__restrict__ units,
                                                           const int32_t *__restrict__ base,
                                                           const int32_t *__restrict__ kind,
                                                           const int32_t *__restrict__ diag,
                                                           uint16_t *__restrict__ off,
                                                           uint8_t *__restrict__ codes,
                                                           V *__restrict__ vals,
                                                           uint32_t *__restrict__ mask,
                                                           const int32_t *__restrict__ pinv) {
    constexpr int kWaves = kBlock / kSellRows;
    __shared__ int32_t s_rp[kBlock + 1];
    __shared__ int32_t s_dg[kWaves][kSellMaxDiag];
    __shared__ int32_t s_kind[kWaves];
    __shared__ uint32_t s_mask[kBlock];
    const int64_t r0 = (int64_t)blockIdx.x * kBlock;
    const int nrows = (int)((n - r0) < kBlock ? (n - r0) : kBlock);
    const int64_t sl0 = r0 / kSellRows;
    const int nsl = (nrows + kSellRows - 1) / kSellRows;
    for (int r = threadIdx.x; r <= nrows; r += kBlock) s_rp[r] = rp[r0 + r];
    if ((int)threadIdx.x < kWaves)
        s_kind[threadIdx.x] = (int)threadIdx.x < nsl ? kind[sl0 + threadIdx.x] : 0;
    for (int i = threadIdx.x; i < kWaves * kSellMaxDiag; i += kBlock)
        s_dg[i / kSellMaxDiag][i % kSellMaxDiag] =
            i / kSellMaxDiag < nsl ? diag[sl0 * kSellMaxDiag + i] : 0;
    s_mask[threadIdx.x] = 0;
    __syncthreads();
    const int32_t e = s_rp[nrows];
    for (int32_t j = s_rp[0] + (int32_t)threadIdx.x; j < e; j += kBlock) {
        int lo = 0, hi = nrows - 1;  // last row i with s_rp[i] <= j
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_rp[mid] <= j) lo = mid; else hi = mid - 1;
        }
        // the row's position within the block (the sorted layout permutes the
        // rows of each block), then its slice within the block and lane
        const int q = pinv ? (int)(pinv[r0 + lo] - r0) : lo;
        const int ls = q / kSellRows;
        const int lane = q % kSellRows;
        const int64_t sl = sl0 + ls;
        const int kd = s_kind[ls];
        int k = j - s_rp[lo];
        if (kd > 0) {  // position of the diagonal c - r among the slice's D
            const int32_t rel = ci[j] - (int32_t)(r0 + lo);
            int a = 0, b = kd - 2;  // it is present: search [0, D - 1]
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (s_dg[ls][mid] < rel) a = mid + 1; else b = mid;
            }
            k = a;
            atomicOr(&s_mask[lo], 1u << k);
        } else {
            const int32_t c = ci[j];
            if (off)
                off[2 * kSellRows * ((int64_t)units[sl] + k / 2) + 2 * lane + (k & 1)] =
                    (uint16_t)(c - base[sl]);
            if (codes) {  // 8-bit delta code (k_sliced_escape_cols stores escaped columns)
                const int32_t d = c - (k > 0 ? ci[j - 1] : base[sl]);
                codes[2 * kSellRows * ((int64_t)units[sl] + sl) + 4 * kSellRows * (int64_t)(k / 4) +
                      4 * lane + (k & 3)] = (uint8_t)(d >= 255 ? 255 : d);
            }
        }
        vals[2 * kSellRows * ((int64_t)units[sl] + k / 2) + 2 * lane + (k & 1)] = val[j];
    }
    __syncthreads();
    if ((int)threadIdx.x < nrows) mask[r0 + threadIdx.x] = s_mask[threadIdx.x];
}

hipError_t launch_sliced_scatter(const spmv_plan &P, const int32_t *units, const int32_t *base,
                                 const int32_t *kind, const int32_t *diag, uint16_t *off,
                                 uint8_t *codes, void *vals, uint32_t *mask, hipStream_t s) {
    if (P.n == 0) return hipSuccess;  // (with no nonzeros it still writes the zero masks)
    const dim3 g((unsigned)((P.n + kBlock - 1) / kBlock));
    const int32_t *pinv = P.d16_sort ? P.d16s_pinv.as<int32_t>() : nullptr;
    switch (P.dtype) {
    case SPMV_F64:
        hipLaunchKernelGGL(k_sliced_scatter<double>, g, dim3(kBlock), 0, s, P.n, P.rowptr, P.colind,
                           (const double *)P.val, units, base, kind, diag, off, codes, (double *)vals,
                           mask, pinv);
        break;
    case SPMV_F32:
        hipLaunchKernelGGL(k_sliced_scatter<float>, g, dim3(kBlock), 0, s, P.n, P.rowptr, P.colind,
                           (const float *)P.val, units, base, kind, diag, off, codes, (float *)vals,
                           mask, pinv);
        break;
    default:
        hipLaunchKernelGGL(k_sliced_scatter<uint16_t>, g, dim3(kBlock), 0, s, P.n, P.rowptr,
                           P.colind, (const uint16_t *)P.val, units, base, kind, diag, off,
                           codes, (uint16_t *)vals, mask, pinv);
    }
    return hipGetLastError();
}

// 8-bit delta coding of the offset slices (Section 3.3).  The code of a
// nonzero is its column minus the previous one of its row (the slice's
// reference column before the first), or the escape code 255 when that gap
// is 255 or more, in which case the column itself is stored: the e-th escape
// of lane l of slice s is esc[64 (eunits[s] + e) + l].  Codes go in groups
// of four positions per lane (a 4-byte load per lane per step): code k of
// lane l is byte 128 (units[s] + s) + 256 (k / 4) + 4 l + k % 4, one spare
// unit per slice covering a width that is not a multiple of 4.  The scatter
// kernel writes the codes, nonzero by nonzero.  Here a wavefront per slice,
// a lane per row, walks the rows in column order: k_sliced_escapes counts
// the escapes (the per-slice maximum E and the sum), k_sliced_escape_cols
// stores the escaped columns of the slices that have any.  Neither kernel
// has a barrier, so whole wavefronts leave early.
constexpr int kEscape = 255;

__global__ __launch_bounds__(kBlock) void k_sliced_escapes(int64_t n, int64_t nsl,
                                                           const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const int32_t *__restrict__ base,
                                                           const int32_t *__restrict__ kind,
                                                           const int32_t *__restrict__ perm,
                                                           int32_t *__restrict__ E,
                                                           int32_t *__restrict__ nesc) {
    const int64_t sl = blockIdx.x * (int64_t)(kBlock / kSellRows) + threadIdx.x / kSellRows;
    if (sl >= nsl) return;
    const int lane = threadIdx.x & (kSellRows - 1);
    const int64_t pos = sl * kSellRows + lane;
    const int64_t r = perm && pos < n ? perm[pos] : pos;  // the row at this position
    int cnt = 0;
    if (kind[sl] == 0 && pos < n) {
        int32_t prev = base[sl];  // the slice's smallest column: no gap is negative
        int32_t j = rp[r];
        const int32_t b = rp[r + 1];
        for (; j + 4 <= b; j += 4) {  // four loads in flight per lane
            const int32_t c0 = ci[j], c1 = ci[j + 1], c2 = ci[j + 2], c3 = ci[j + 3];
            cnt += (c0 - prev >= kEscape) + (c1 - c0 >= kEscape) + (c2 - c1 >= kEscape) +
                   (c3 - c2 >= kEscape);
            prev = c3;
        }
        for (; j < b; ++j) {
            const int32_t c = ci[j];
            cnt += (c - prev >= kEscape) ? 1 : 0;
            prev = c;
        }
    }
    int mx = cnt, sum = cnt;
#pragma unroll
    for (int d = kSellRows / 2; d > 0; d >>= 1) {
        const int om = __shfl_xor(mx, d, kSellRows);
        sum += __shfl_xor(sum, d, kSellRows);
        mx = om > mx ? om : mx;
    }
    if (lane == 0) {
        E[sl] = mx;
        nesc[sl] = sum;
    }
}

// eunits has S + 1 entries (the last is the total), so E_s = eunits[s + 1] -
// eunits[s]; slices without escapes are skipped
__global__ __launch_bounds__(kBlock) void k_sliced_escape_cols(int64_t n, int64_t nsl,
                                                               const int32_t *__restrict__ rp,
                                                               const int32_t *__restrict__ ci,
                                                               const int32_t *__restrict__ base,
                                                               const int32_t *__restrict__ kind,
                                                               const int32_t *__restrict__ eunits,
                                                               const int32_t *__restrict__ perm,
                                                               int32_t *__restrict__ esc) {
    const int64_t sl = blockIdx.x * (int64_t)(kBlock / kSellRows) + threadIdx.x / kSellRows;
    if (sl >= nsl || kind[sl] != 0 || eunits[sl + 1] == eunits[sl]) return;
    const int lane = threadIdx.x & (kSellRows - 1);
    const int64_t pos = sl * kSellRows + lane;
    if (pos >= n) return;
    const int64_t r = perm ? perm[pos] : pos;  // the row at this position
    int64_t q = (int64_t)kSellRows * eunits[sl] + lane;  // this lane's next escape entry
    int32_t prev = base[sl];
    for (int32_t j = rp[r]; j < rp[r + 1]; ++j) {
        const int32_t c = ci[j];
        if (c - prev >= kEscape) {
            esc[q] = c;
            q += kSellRows;
        }
        prev = c;
    }
}

hipError_t launch_sliced_escapes(const spmv_plan &P, const int32_t *base, const int32_t *kind,
                                 int32_t *E, int32_t *nesc, hipStream_t s) {
    const int64_t nsl = (P.n + kSellRows - 1) / kSellRows;
    if (nsl == 0) return hipSuccess;
    const int64_t per = kBlock / kSellRows;
    hipLaunchKernelGGL(k_sliced_escapes, dim3((unsigned)((nsl + per - 1) / per)), dim3(kBlock), 0,
                       s, P.n, nsl, P.rowptr, P.colind, base, kind,
                       P.d16_sort ? P.d16s_perm.as<int32_t>() : nullptr, E, nesc);
    return hipGetLastError();
}

hipError_t launch_sliced_escape_cols(const spmv_plan &P, const int32_t *base, const int32_t *kind,
                                    const int32_t *eunits, int32_t *esc, hipStream_t s) {
    const int64_t nsl = (P.n + kSellRows - 1) / kSellRows;
    if (nsl == 0) return hipSuccess;
    const int64_t per = kBlock / kSellRows;
    hipLaunchKernelGGL(k_sliced_escape_cols, dim3((unsigned)((nsl + per - 1) / per)), dim3(kBlock), 0,
                       s, P.n, nsl, P.rowptr, P.colind, base, kind, eunits,
                       P.d16_sort ? P.d16s_perm.as<int32_t>() : nullptr, esc);
    return hipGetLastError();
}

// one bit per row from the long-row flags (a thread per 32-row word)
__global__ __launch_bounds__(kBlock) void k_long_mask(int64_t n, const int32_t *__restrict__ flags,
                                                      uint32_t *__restrict__ mask) {
    const int64_t w = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (w * 32 >= n) return;
    uint32_t m = 0;
    for (int b = 0; b < 32; ++b) {
        const int64_t i = w * 32 + b;
        if (i < n && flags[i] != 0) m |= 1u << b;
    }
    mask[w] = m;
}

hipError_t launch_long_mask(int64_t n, const int32_t *flags, uint32_t *mask, hipStream_t s) {
    const int64_t words = (n + 31) / 32;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_long_mask, dim3((unsigned)((words + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, n, flags, mask);
    return hipGetLastError();
}

// largest window span (cmax - cmin) over panels, for the 16-bit feasibility test
__global__ __launch_bounds__(kBlock) void k_max_span(const int32_t *__restrict__ cmin,
                                                     const int32_t *__restrict__ cmax,
                                                     int64_t panels, unsigned long long *mx) {
    unsigned long long t = 0;
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < panels;
         p += (int64_t)gridDim.x * kBlock) {
        const int64_t d = (int64_t)cmax[p] - cmin[p];
        if (d > (int64_t)t) t = (unsigned long long)d;
    }
    if (t) atomicMax(mx, t);
}

hipError_t launch_max_span(const int32_t *cmin, const int32_t *cmax, int64_t panels,
                           unsigned long long *d_max, hipStream_t s) {
    hipError_t e = hipMemsetAsync(d_max, 0, sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    int64_t g = (panels + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_max_span, dim3((unsigned)g), dim3(kBlock), 0, s, cmin, cmax, panels, d_max);
    return hipGetLastError();
}

// ---- 16-bit column codes over ranges of a column array: range k covers
// positions [bnd[min(k H, nb)], bnd[min((k + 1) H, nb)]) (merge-path tiles:
// bnd = the tiles' nonzero coordinates, H = 1; x-block row blocks of one
// slice: bnd = the slice's row pointers, H = the block height).  Each range
// takes its smallest column as reference; its span is its largest column
// minus that (0 for an empty range, whose reference is 0).
__global__ __launch_bounds__(kBlock) void k_range_ref(int64_t nb, int64_t H,
                                                      const int32_t *__restrict__ bnd,
                                                      const int32_t *__restrict__ ci,
                                                      int32_t *__restrict__ base,
                                                      int32_t *__restrict__ span) {
    __shared__ int32_t s_lo[kBlock / 64], s_hi[kBlock / 64];
    const int64_t k = blockIdx.x;
    const int64_t i0 = k * H < nb ? k * H : nb, i1 = (k + 1) * H < nb ? (k + 1) * H : nb;
    const int32_t a = bnd[i0], e = bnd[i1];
    int32_t lo = INT32_MAX, hi = -1;
    for (int32_t j = a + (int32_t)threadIdx.x; j < e; j += kBlock) {
        const int32_t c = ci[j];
        lo = c < lo ? c : lo;
        hi = c > hi ? c : hi;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t lo2 = __shfl_xor(lo, o, 64), hi2 = __shfl_xor(hi, o, 64);
        lo = lo2 < lo ? lo2 : lo;
        hi = hi2 > hi ? hi2 : hi;
    }
    if ((threadIdx.x & 63) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            lo = s_lo[w] < lo ? s_lo[w] : lo;
            hi = s_hi[w] > hi ? s_hi[w] : hi;
        }
        base[k] = hi < 0 ? 0 : lo;
        span[k] = hi < 0 ? 0 : hi - lo;
    }
}

// off[j] = ci[j] - base[k] for every position j of range k (ranges as above;
// only called once every span is known to fit 16 bits).
__global__ __launch_bounds__(kBlock) void k_range_encode(int64_t nb, int64_t H,
                                                         const int32_t *__restrict__ bnd,
                                                         const int32_t *__restrict__ ci,
                                                         const int32_t *__restrict__ base,
                                                         uint16_t *__restrict__ off) {
    const int64_t k = blockIdx.x;
    const int64_t i0 = k * H < nb ? k * H : nb, i1 = (k + 1) * H < nb ? (k + 1) * H : nb;
    const int32_t a = bnd[i0], e = bnd[i1], b0 = base[k];
    for (int32_t j = a + (int32_t)threadIdx.x; j < e; j += kBlock) off[j] = (uint16_t)(ci[j] - b0);
}

hipError_t launch_range_ref(int64_t nranges, int64_t nb, int64_t H, const int32_t *bnd,
                            const int32_t *ci, int32_t *base, int32_t *span, hipStream_t s) {
    if (nranges <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_range_ref, dim3((unsigned)nranges), dim3(kBlock), 0, s, nb, H, bnd, ci, base,
                       span);
    return hipGetLastError();
}

hipError_t launch_range_encode(int64_t nranges, int64_t nb, int64_t H, const int32_t *bnd,
                               const int32_t *ci, const int32_t *base, uint16_t *off, hipStream_t s) {
    if (nranges <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_range_encode, dim3((unsigned)nranges), dim3(kBlock), 0, s, nb, H, bnd, ci,
                       base, off);
    return hipGetLastError();
}

// ---- merge path: start coordinate of every tile (t = 0..tiles).  On
// diagonal d the row coordinate is the smallest i in [max(0, d-NNZ),
// min(d, N)] with rowptr[i+1] > d - i - 1; the nonzero coordinate is d - i.
__global__ __launch_bounds__(kBlock) void k_merge_splits(int64_t n, int64_t nnz, int64_t tiles,
                                                         const int32_t *__restrict__ rp,
                                                         int32_t *__restrict__ srow,
                                                         int32_t *__restrict__ snnz) {
    const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (t > tiles) return;
    const int64_t total = n + nnz;
    const int64_t d = t * kMergeTile < total ? t * kMergeTile : total;
    int64_t lo = d - nnz > 0 ? d - nnz : 0, hi = d < n ? d : n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rp[mid + 1] <= d - mid - 1) lo = mid + 1; else hi = mid;
    }
    srow[t] = (int32_t)lo;
    snnz[t] = (int32_t)(d - lo);
}

hipError_t launch_merge_splits(const int32_t *rowptr, int64_t n, int64_t nnz, int32_t *srow,
                               int32_t *snnz, int64_t tiles, hipStream_t s) {
    const int64_t g = (tiles + 1 + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_merge_splits, dim3((unsigned)g), dim3(kBlock), 0, s, n, nnz, tiles,
                       rowptr, srow, snnz);
    return hipGetLastError();
}

// ---- x blocking: column slices of width cw (slice of column c = c / cw,
// the last slice also takes the remainder).  Slice preparation walks the
// merge path of the CSR (row ends and nonzeros) in tiles of kMergeTile items
// whose start coordinates come from k_merge_splits: a long row is shared by
// many workgroups and a run of empty rows costs one item per row.  Each
// thread consumes kMergeIpt consecutive items and so knows the row of every
// nonzero it takes.  Within a row the columns are sorted, so the nonzeros of
// one slice form one run.
__device__ inline int slice_of(int32_t c, int64_t cw, int ns) {
    const int64_t s = (int64_t)c / cw;
    return s < ns - 1 ? (int)s : ns - 1;
}

// First position in [lo, hi] whose column is in slice s or later (ci[hi] is);
// slice s > 0 starts at column s*cw whatever the slice count.
__device__ inline int32_t run_start(const int32_t *__restrict__ ci, int32_t lo, int32_t hi, int s,
                                    int64_t cw) {
    if (s == 0) return lo;
    const int64_t bound = (int64_t)s * cw;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)ci[mid] < bound) lo = mid + 1; else hi = mid;
    }
    return lo;
}

struct SliceTile {
    int32_t i0, j0, nr, nz, rs0;  // first row, first nonzero, sizes, start of row i0
    int xi, yj, dend, it;          // this thread's walk
};

// Loads the tile's row ends into s_end[0..nr] and its columns (and the one
// after) into s_ci[0..nz]; positions this thread on the merge path.
__device__ inline SliceTile slice_tile_begin(int64_t tile, int64_t n, int64_t nnz,
                                             const int32_t *__restrict__ rp,
                                             const int32_t *__restrict__ ci,
                                             const int32_t *__restrict__ srow,
                                             const int32_t *__restrict__ snnz, int32_t *s_end,
                                             int32_t *s_ci) {
    SliceTile T;
    T.i0 = srow[tile];
    T.j0 = snnz[tile];
    T.nr = srow[tile + 1] - T.i0;
    T.nz = snnz[tile + 1] - T.j0;
    T.rs0 = rp[T.i0];
    for (int r = threadIdx.x; r <= T.nr; r += kBlock) {
        const int64_t row = (int64_t)T.i0 + r;
        s_end[r] = row < n ? rp[row + 1] : INT32_MAX;
    }
    for (int q = threadIdx.x; q <= T.nz; q += kBlock)
        s_ci[q] = (int64_t)T.j0 + q < nnz ? ci[T.j0 + q] : INT32_MAX;
    __syncthreads();
    const int total = T.nr + T.nz;
    const int d = (int)threadIdx.x * kMergeIpt < total ? (int)threadIdx.x * kMergeIpt : total;
    int lo = d - T.nz > 0 ? d - T.nz : 0, hi = d < T.nr ? d : T.nr;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_end[mid] <= T.j0 + d - mid - 1) lo = mid + 1; else hi = mid;
    }
    T.xi = lo;
    T.yj = d - lo;
    T.it = d;
    T.dend = (d + kMergeIpt) < total ? (d + kMergeIpt) : total;
    return T;
}

// lens[s * n + i] = nonzeros of row i in slice s; lens must be zero on entry
// (only non-empty runs are written, each by the thread holding its last
// nonzero).
__global__ __launch_bounds__(kBlock) void k_slice_count(int64_t n, int64_t nnz, int64_t cw, int ns,
                                                        const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const int32_t *__restrict__ srow,
                                                        const int32_t *__restrict__ snnz,
                                                        int32_t *__restrict__ lens) {
    __shared__ int32_t s_end[kMergeTile + 1];
    __shared__ int32_t s_ci[kMergeTile + 1];
    SliceTile T = slice_tile_begin(blockIdx.x, n, nnz, rp, ci, srow, snnz, s_end, s_ci);
    for (; T.it < T.dend; ++T.it) {
        if (T.yj < T.nz && T.j0 + T.yj < s_end[T.xi]) {
            const int32_t k = T.j0 + T.yj;
            const int s = slice_of(s_ci[T.yj], cw, ns);
            const bool last = k + 1 == s_end[T.xi] || slice_of(s_ci[T.yj + 1], cw, ns) != s;
            if (last) {
                const int32_t rs = T.xi == 0 ? T.rs0 : s_end[T.xi - 1];
                lens[(int64_t)s * n + T.i0 + T.xi] = k + 1 - run_start(ci, rs, k, s, cw);
            }
            ++T.yj;
        } else {
            ++T.xi;
        }
    }
}

// ---- long rows of the x-block split
__global__ __launch_bounds__(kBlock) void k_long_flags(int64_t n, int ns,
                                                       const int32_t *__restrict__ lens,
                                                       int32_t *__restrict__ flags) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int32_t mx = 0;
        for (int s = 0; s < ns; ++s) mx = lens[(int64_t)s * n + i] > mx ? lens[(int64_t)s * n + i] : mx;
        flags[i] = mx > kSliceStreamMaxLen;
    }
}

__global__ __launch_bounds__(kBlock) void k_long_compact(int64_t n, const int32_t *__restrict__ flags,
                                                         const int32_t *__restrict__ pos,
                                                         const int32_t *__restrict__ rp,
                                                         int32_t *__restrict__ rows,
                                                         int32_t *__restrict__ beg,
                                                         int32_t *__restrict__ end) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        if (flags[i]) {
            const int32_t t = pos[i];
            rows[t] = (int32_t)i;
            beg[t] = rp[i];
            end[t] = rp[i + 1];
        }
}

__global__ __launch_bounds__(kBlock) void k_long_zero(int64_t L, int ns, int64_t n,
                                                      const int32_t *__restrict__ rows,
                                                      int32_t *__restrict__ lens) {
    for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < L;
         t += (int64_t)gridDim.x * kBlock)
        for (int s = 0; s < ns; ++s) lens[(int64_t)s * n + rows[t]] = 0;
}

// Slice boundaries inside each long row: bounds[t (S + 1) + s] is the first
// nonzero of long row t whose column is at least s cw (the row's columns
// increase), from beg[t] (s = 0) to end[t] (s = S).
__global__ __launch_bounds__(kBlock) void k_long_bounds(int64_t L, int ns, int64_t cw,
                                                       const int32_t *__restrict__ ci,
                                                       const int32_t *__restrict__ beg,
                                                       const int32_t *__restrict__ end,
                                                       int32_t *__restrict__ bounds) {
    const int64_t total = L * (ns + 1);
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t t = i / (ns + 1);
        const int sl = (int)(i % (ns + 1));
        int32_t lo = beg[t], hi = end[t];
        if (sl > 0 && sl < ns) {
            const int64_t c = (int64_t)sl * cw;
            while (lo < hi) {
                const int32_t mid = lo + (hi - lo) / 2;
                if (ci[mid] < c) lo = mid + 1; else hi = mid;
            }
        }
        bounds[i] = sl == ns ? hi : lo;
    }
}

hipError_t launch_long_bounds(int64_t L, int ns, int64_t cw, const int32_t *ci, const int32_t *beg,
                              const int32_t *end, int32_t *bounds, hipStream_t s) {
    if (L == 0) return hipSuccess;
    int64_t g = (L * (ns + 1) + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_long_bounds, dim3((unsigned)g), dim3(kBlock), 0, s, L, ns, cw, ci, beg, end,
                       bounds);
    return hipGetLastError();
}

hipError_t launch_long_flags(int64_t n, int ns, const int32_t *lens, int32_t *flags, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_long_flags, dim3((unsigned)g), dim3(kBlock), 0, s, n, ns, lens, flags);
    return hipGetLastError();
}

hipError_t launch_long_compact(int64_t n, const int32_t *flags, const int32_t *pos,
                               const int32_t *rp, int32_t *rows, int32_t *beg, int32_t *end,
                               hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_long_compact, dim3((unsigned)g), dim3(kBlock), 0, s, n, flags, pos, rp,
                       rows, beg, end);
    return hipGetLastError();
}

hipError_t launch_long_zero(int64_t L, int ns, int64_t n, const int32_t *rows, int32_t *lens,
                            hipStream_t s) {
    if (L == 0) return hipSuccess;
    int64_t g = (L + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_long_zero, dim3((unsigned)g), dim3(kBlock), 0, s, L, ns, n, rows, lens);
    return hipGetLastError();
}

// Maximum of a non-negative int32 array: per-block maxima into part[], then
// one block folds them (no same-address atomics).
constexpr int kMaxGrid = 2048;

__global__ __launch_bounds__(kBlock) void k_max_i32(const int32_t *__restrict__ a, int64_t n,
                                                    int32_t *__restrict__ part) {
    __shared__ int32_t sh[kBlock / 64];
    int32_t t = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        t = a[i] > t ? a[i] : t;
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t u = __shfl_xor(t, o, 64);
        t = u > t ? u : t;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBlock / 64; ++q) t = sh[q] > t ? sh[q] : t;
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_max_final(const int32_t *__restrict__ part, int np,
                                                      unsigned long long *__restrict__ mx) {
    __shared__ int32_t sh[kBlock / 64];
    int32_t t = 0;
    for (int i = threadIdx.x; i < np; i += kBlock) t = part[i] > t ? part[i] : t;
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t u = __shfl_xor(t, o, 64);
        t = u > t ? u : t;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBlock / 64; ++q) t = sh[q] > t ? sh[q] : t;
        *mx = (unsigned long long)t;
    }
}

hipError_t launch_max_i32(const int32_t *a, int64_t n, int32_t *d_part,
                          unsigned long long *d_max, hipStream_t s) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > kMaxGrid) g = kMaxGrid;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_max_i32, dim3((unsigned)g), dim3(kBlock), 0, s, a, n, d_part);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kBlock), 0, s, d_part, (int)g, d_max);
    return hipGetLastError();
}

// Copy every row's slice runs into the slice-major arrays: nonzero k of row
// i in slice s moves to off[s] + srp_s[i] + (k - start of its run).  A thread
// finds the start of its first run by a search inside the row; later runs it
// meets start at the nonzero where the row or the slice changes.
template <class V>
__global__ __launch_bounds__(kBlock) void k_slice_scatter(int64_t n, int64_t nnz, int64_t cw,
                                                          int ns, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci,
                                                          const V *__restrict__ val,
                                                          const int32_t *__restrict__ srow,
                                                          const int32_t *__restrict__ snnz,
                                                          const int32_t *__restrict__ srp,
                                                          SliceOffsets so,
                                                          int32_t *__restrict__ xci,
                                                          V *__restrict__ xval) {
    __shared__ int32_t s_end[kMergeTile + 1];
    __shared__ int32_t s_ci[kMergeTile + 1];
    __shared__ int64_t s_dst[kMergeTile];  // each of the tile's nonzeros: its position, or -1
    SliceTile T = slice_tile_begin(blockIdx.x, n, nnz, rp, ci, srow, snnz, s_end, s_ci);
    int cur_row = -1, cur_s = -1;
    int64_t shift = 0;
    int32_t run_end = 0;  // first position past the run's slot (writes stay inside it)
    // the merge-path walk only finds positions; the copies below go
    // nonzero by nonzero across the workgroup, so that the value loads are
    // coalesced and the stores too within each run
    for (; T.it < T.dend; ++T.it) {
        if (T.yj < T.nz && T.j0 + T.yj < s_end[T.xi]) {
            const int32_t k = T.j0 + T.yj;
            const int32_t c = s_ci[T.yj];
            const int s = slice_of(c, cw, ns);
            if (T.xi != cur_row || s != cur_s) {
                const int32_t rs = T.xi == 0 ? T.rs0 : s_end[T.xi - 1];
                const int32_t st = (T.xi == cur_row || k == rs) ? k : run_start(ci, rs, k, s, cw);
                const int32_t *r = srp + (int64_t)s * (n + 1) + T.i0 + T.xi;
                shift = so.off[s] + r[0] - st;
                run_end = st + (r[1] - r[0]);
                cur_row = T.xi;
                cur_s = s;
            }
            s_dst[T.yj] = k < run_end ? k + shift : -1;
            ++T.yj;
        } else {
            ++T.xi;
        }
    }
    __syncthreads();
    for (int q = (int)threadIdx.x; q < T.nz; q += kBlock) {
        const int64_t d = s_dst[q];
        if (d >= 0) {
            xci[d] = s_ci[q];
            xval[d] = val[T.j0 + q];
        }
    }
}

hipError_t launch_slice_count(const spmv_plan &P, int64_t cw, const int32_t *srow,
                              const int32_t *snnz, int64_t tiles, int32_t *lens, hipStream_t s) {
    if (P.n == 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(lens, 0, (size_t)P.xs_slices * P.n * 4, s);
    if (e != hipSuccess || tiles == 0) return e;
    hipLaunchKernelGGL(k_slice_count, dim3((unsigned)tiles), dim3(kBlock), 0, s, P.n, P.nnz, cw,
                       P.xs_slices, P.rowptr, P.colind, srow, snnz, lens);
    return hipGetLastError();
}

hipError_t launch_slice_scatter(const spmv_plan &P, const int32_t *srow, const int32_t *snnz,
                                int64_t tiles, const int32_t *srp, const SliceOffsets &so,
                                int32_t *xci, void *xval, hipStream_t s) {
    if (P.n == 0 || tiles == 0) return hipSuccess;
    const int64_t cw = P.xs_width;
    const dim3 g((unsigned)tiles);
    switch (P.dtype) {
    case SPMV_F64:
        hipLaunchKernelGGL(k_slice_scatter<double>, g, dim3(kBlock), 0, s, P.n, P.nnz, cw,
                           P.xs_slices, P.rowptr, P.colind, (const double *)P.val, srow, snnz, srp, so, xci,
                           (double *)xval);
        break;
    case SPMV_F32:
        hipLaunchKernelGGL(k_slice_scatter<float>, g, dim3(kBlock), 0, s, P.n, P.nnz, cw,
                           P.xs_slices, P.rowptr, P.colind, (const float *)P.val, srow, snnz, srp, so, xci,
                           (float *)xval);
        break;
    default:
        hipLaunchKernelGGL(k_slice_scatter<uint16_t>, g, dim3(kBlock), 0, s, P.n, P.nnz, cw,
                           P.xs_slices, P.rowptr, P.colind, (const uint16_t *)P.val, srow, snnz, srp, so, xci,
                           (uint16_t *)xval);
    }
    return hipGetLastError();
}

// ---- row panels: the column window [min first col, max last col] of each
// panel of H rows ((0, -1) when the panel has no nonzeros), which gives the
// delta16 reference columns and its 16-bit span test.  One wavefront per
// panel.
__global__ __launch_bounds__(kBlock) void k_panel_windows(int64_t n, int H, int64_t panels,
                                                          const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci,
                                                          int32_t *__restrict__ cmin,
                                                          int32_t *__restrict__ cmax) {
    const int64_t p = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (p >= panels) return;
    const int64_t r0 = p * H;
    const int64_t r1 = (r0 + H) < n ? (r0 + H) : n;
    int32_t lo = INT32_MAX, hi = -1;
    for (int64_t r = r0 + lane; r < r1; r += 64) {
        const int32_t a = rp[r], b = rp[r + 1];
        if (a < b) {
            lo = ci[a] < lo ? ci[a] : lo;
            hi = ci[b - 1] > hi ? ci[b - 1] : hi;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t lo2 = __shfl_xor(lo, o, 64), hi2 = __shfl_xor(hi, o, 64);
        lo = lo2 < lo ? lo2 : lo;
        hi = hi2 > hi ? hi2 : hi;
    }
    if (lane == 0) {
        cmin[p] = hi < 0 ? 0 : lo;
        cmax[p] = hi;
    }
}

hipError_t launch_panel_windows(const spmv_plan &P, int H, int32_t *cmin, int32_t *cmax,
                                int64_t panels, hipStream_t s) {
    const int64_t g = (panels * 64 + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_panel_windows, dim3((unsigned)g), dim3(kBlock), 0, s, P.n, H, panels,
                       P.rowptr, P.colind, cmin, cmax);
    return hipGetLastError();
}

// ---- static partition with equal nonzeros: b_0 = 0, b_P = N, and b_p the
// first row whose start offset reaches ceil(p NNZ / P).
__global__ __launch_bounds__(kBlock) void k_partition(int64_t n, int parts,
                                                      const int32_t *__restrict__ rp,
                                                      int32_t *__restrict__ b) {
    const int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (p > parts) return;
    if (p == 0) { b[0] = 0; return; }
    if (p == parts) { b[parts] = (int32_t)n; return; }
    const int64_t nnz = rp[n];
    const int64_t target = (p * nnz + parts - 1) / parts;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rp[mid] < target) lo = mid + 1; else hi = mid;
    }
    b[p] = (int32_t)lo;
}

hipError_t launch_partition(const int32_t *rowptr, int64_t n, int parts, int32_t *bounds,
                            hipStream_t s) {
    const int64_t g = (parts + 1 + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_partition, dim3((unsigned)g), dim3(kBlock), 0, s, n, parts, rowptr, bounds);
    return hipGetLastError();
}

// noxmiss column array: every nonzero of row i gets column i mod M (x read
// as a regular stream, one element per row).  A sub-wavefront of W lanes
// per row.
template <int W>
__global__ __launch_bounds__(kBlock) void k_row_columns(int64_t n, int64_t m,
                                                        const int32_t *__restrict__ rp,
                                                        int32_t *__restrict__ out) {
    const int lane = threadIdx.x & (W - 1);
    const int64_t nsub = (int64_t)gridDim.x * (kBlock / W);
    for (int64_t i = blockIdx.x * (int64_t)(kBlock / W) + threadIdx.x / W; i < n; i += nsub) {
        const int32_t a = rp[i], b = rp[i + 1];
        const int32_t c = (int32_t)(m > 0 ? i % m : 0);
        for (int32_t k = a + lane; k < b; k += W) out[k] = c;
    }
}

hipError_t launch_row_columns(const spmv_plan &P, int32_t *out, hipStream_t s) {
    if (P.n == 0 || P.nnz == 0) return hipSuccess;
    const int W = P.vec_width;
    int64_t g = (P.n + (kBlock / W) - 1) / (kBlock / W);
    if (g > (int64_t)P.num_cus * 32) g = (int64_t)P.num_cus * 32;
    switch (W) {
#define RC(WW) case WW: hipLaunchKernelGGL((k_row_columns<WW>), dim3((unsigned)g), dim3(kBlock), 0, s, P.n, P.m, P.rowptr, out); break;
        RC(2) RC(4) RC(8) RC(16) RC(32) RC(64)
#undef RC
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_widen(const int32_t *__restrict__ in,
                                                  int64_t *__restrict__ out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        out[i] = in[i];
}

hipError_t launch_widen(const int32_t *in, int64_t *out, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)g), dim3(kBlock), 0, s, in, out, n);
    return hipGetLastError();
}

// ---- value rounding from FP64, one round-to-nearest-even.
// FP32: the conversion instruction.  BF16: round to odd into FP32 (truncate
// toward zero, then set the last bit if anything was dropped), then round to
// nearest even into 8 significant bits; rounding to odd first with at least
// two extra bits makes the two-step rounding equal to a single rounding
// (Boldo and Melquiond, IEEE TC 2008).
__device__ __forceinline__ uint16_t f64_to_bf16(double d) {
    if (d != d) return 0x7FC0;
    float f = __double2float_rz(d);
    uint32_t u = __float_as_uint(f);
    if ((double)f != d) u |= 1u;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(kBlock) void k_quantize(const double *__restrict__ in, void *out,
                                                     int64_t n, int to) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double d = in[i];
        if (to == SPMV_F32) static_cast<float *>(out)[i] = __double2float_rn(d);
        else static_cast<uint16_t *>(out)[i] = f64_to_bf16(d);
    }
}

hipError_t launch_quantize(const double *in, void *out, int64_t n, int to, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)g), dim3(kBlock), 0, s, in, out, n, to);
    return hipGetLastError();
}

}  // namespace spmvsel
