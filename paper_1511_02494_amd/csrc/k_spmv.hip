// The six SpMV variants of the optimisation pool (gfx950, wave64).
//
// All compute y_i = sum_j A_ij x_j for CSR A (Algorithm 1).  FP64 plans
// accumulate in FP64; FP32/BF16 plans accumulate in FP32 with Kahan
// compensation on rows of more than 256 nonzeros.  Reductions use fixed
// pairings and fixed orders, so every variant is deterministic.
#include "dev.h"
#include "internal.h"

namespace spmvsel {

// ============================================================ csr_scalar
// One lane per row, summing the row in increasing column order from +0:
// exactly the order of Algorithm 1.  The unoptimised baseline.
template <class V>
__global__ __launch_bounds__(kBlock) void k_csr_scalar(int64_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const V *__restrict__ val,
                                                       const typename VT<V>::A *__restrict__ x,
                                                       typename VT<V>::A *__restrict__ y, int kmin) {
    using A = typename VT<V>::A;
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t a = rp[i], b = rp[i + 1];
    const bool comp = is_f32<A>() && (b - a) >= kmin;
    Sum<A> s;
    for (int32_t k = a; k < b; ++k) s.add(VT<V>::cvt(val[k]) * x[ci[k]], comp);
    __builtin_nontemporal_store(s.s, y + i);
}

// ============================================================ csr_vector
// A sub-wavefront of W lanes per row (Bell and Garland's vector kernel with
// the width adapted to the mean row length); lanes stride the row, then a
// DPP/swizzle butterfly sums the lane partials.
template <class V, int W>
__global__ __launch_bounds__(kBlock) void k_csr_vector(int64_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const V *__restrict__ val,
                                                       const typename VT<V>::A *__restrict__ x,
                                                       typename VT<V>::A *__restrict__ y, int kmin) {
    using A = typename VT<V>::A;
    const int lane = threadIdx.x & (W - 1);
    const int64_t nsub = (int64_t)gridDim.x * (kBlock / W);
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    for (int64_t i = blk * (kBlock / W) + threadIdx.x / W; i < n; i += nsub) {
        const int32_t a = rp[i], b = rp[i + 1];
        const bool comp = is_f32<A>() && (b - a) >= kmin;
        Sum<A> s;
        int32_t k = a + lane;
        // two independent loads in flight per lane
        for (; k + W < b; k += 2 * W) {
            const A v0 = VT<V>::cvt(ld_nt(val + k));
            const A v1 = VT<V>::cvt(ld_nt(val + k + W));
            const int32_t c0 = ld_nt(ci + k), c1 = ld_nt(ci + k + W);
            const A p0 = v0 * x[c0];
            const A p1 = v1 * x[c1];
            s.add(p0, comp);
            s.add(p1, comp);
        }
        if (k < b) s.add(VT<V>::cvt(ld_nt(val + k)) * x[ld_nt(ci + k)], comp);
        const A t = group_sum<W>(s.s);
        if (lane == 0) __builtin_nontemporal_store(t, y + i);
    }
}

// ============================================================ row streaming
// short_row and delta16 (CSR-stream style).  A workgroup owns 256*R
// consecutive rows.  Their nonzeros are streamed in LDS chunks of 2048 in a
// striped layout: lane t of the workgroup takes the pairs starting at
// chunk + 2t + 512j (j = 0..3) with 2-element vector loads, so that each
// load and each x gather of a wavefront covers consecutive nonzeros.  The
// products go to LDS; then thread t sums its R rows from LDS in column
// order (the order of Algorithm 1, so FP64 results equal the sequential sum
// bit for bit).
// With D16 the column of nonzero k is base[block] + off[k]: 16-bit offsets
// from the smallest column of the workgroup's block of rows.
template <class T> struct Pair;
template <> struct Pair<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Pair<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Pair<uint16_t> { typedef unsigned short type __attribute__((ext_vector_type(2))); };
template <> struct Pair<uint8_t> { typedef unsigned char type __attribute__((ext_vector_type(2))); };
template <> struct Pair<int32_t> { typedef int type __attribute__((ext_vector_type(2))); };

template <class V, bool D16, int R, bool STAGE>
__device__ __forceinline__ void rowstream_block(
    int64_t blk, int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const uint16_t *__restrict__ off, const int32_t *__restrict__ rbase,
    const V *__restrict__ val, const typename VT<V>::A *__restrict__ x,
    typename VT<V>::A *__restrict__ y, int kmin) {
    using A = typename VT<V>::A;
    using VP = typename Pair<V>::type;
    using IP = typename Pair<int32_t>::type;
    using OP = typename Pair<uint16_t>::type;
    constexpr int RB = kBlock * R;
    constexpr int NP = kRunLen / 2;  // pairs per thread per chunk
    __shared__ int32_t s_rp[RB + 1];
    __shared__ A s_prod[kChunk];
    // STAGE: with several rows per thread, results are staged here and
    // written coalesced at the end (direct stores stride lanes by R rows);
    // pays off where y is a large share of the traffic (x-block partials)
    constexpr bool SY = STAGE && R > 1;
    __shared__ A s_y[SY ? RB : 1];

    const int64_t r0 = blk * RB;
    const int nrows = (int)((n - r0) < RB ? (n - r0) : RB);
    for (int r = threadIdx.x; r <= nrows; r += kBlock) s_rp[r] = rp[r0 + r];
    __syncthreads();
    const int32_t s = s_rp[0], e = s_rp[nrows];
    const int32_t bbase = D16 ? rbase[blk] : 0;

    int myr = threadIdx.x * R;
    const int myr_end = (myr + R) < nrows ? (myr + R) : nrows;
    int32_t k = myr < nrows ? s_rp[myr] : e;
    bool comp = is_f32<A>() && myr < nrows && (s_rp[myr + 1] - s_rp[myr]) >= kmin;
    Sum<A> acc;

    const int32_t a0 = s & ~1;
    for (int32_t cs = a0; cs < e; cs += kChunk) {
        // ---- phase 1: products of this thread's pairs
        A p[kRunLen];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int32_t kk = cs + 2 * threadIdx.x + 2 * kBlock * j;
            V v0 = V(0), v1 = V(0);
            int32_t c0 = 0, c1 = 0;
            if (kk + 1 < e) {
                const VP vv = __builtin_nontemporal_load(reinterpret_cast<const VP *>(val + kk));
                v0 = vv.x;
                v1 = vv.y;
                if (D16) {
                    const OP oo = __builtin_nontemporal_load(reinterpret_cast<const OP *>(off + kk));
                    c0 = oo.x;
                    c1 = oo.y;
                } else {
                    const IP cc = __builtin_nontemporal_load(reinterpret_cast<const IP *>(ci + kk));
                    c0 = cc.x;
                    c1 = cc.y;
                }
            } else if (kk < e) {
                v0 = val[kk];
                c0 = D16 ? (int32_t)off[kk] : ci[kk];
            }
            const bool ok0 = kk >= s && kk < e, ok1 = kk + 1 >= s && kk + 1 < e;
            if (D16) {
                c0 += bbase;
                c1 += bbase;
            }
            p[2 * j] = ok0 ? VT<V>::cvt(v0) * x[c0] : A(0);
            p[2 * j + 1] = ok1 ? VT<V>::cvt(v1) * x[c1] : A(0);
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            s_prod[2 * threadIdx.x + 2 * kBlock * j] = p[2 * j];
            s_prod[2 * threadIdx.x + 2 * kBlock * j + 1] = p[2 * j + 1];
        }
        __syncthreads();
        // ---- phase 2: each thread sums its rows' products in this chunk
        const int32_t ce = (cs + kChunk) < e ? (cs + kChunk) : e;
        while (myr < myr_end) {
            const int32_t rend = s_rp[myr + 1];
            const int32_t lim = rend < ce ? rend : ce;
            for (; k < lim; ++k) acc.add(s_prod[k - cs], comp);
            if (k != rend) break;
            // plain stores: with R rows per thread the lanes' stores are R rows
            // apart, and streaming stores of such scattered words ran the
            // 8M short-rows matrix at half speed (the L2 no longer merges them)
            if (SY) s_y[myr] = acc.s; else y[r0 + myr] = acc.s;
            acc.reset();
            ++myr;
            comp = is_f32<A>() && myr < myr_end && (s_rp[myr + 1] - s_rp[myr]) >= kmin;
        }
        __syncthreads();
    }
    for (; myr < myr_end; ++myr) {  // rows with no nonzeros left (all empty)
        if (SY) s_y[myr] = acc.s; else y[r0 + myr] = acc.s;
        acc.reset();
    }
    if (SY) {
        __syncthreads();
        for (int r = threadIdx.x; r < nrows; r += kBlock) y[r0 + r] = s_y[r];
    }
}

template <class V, bool D16, int R>
__global__ __launch_bounds__(kBlock) void k_rowstream(
    int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const uint16_t *__restrict__ off, const int32_t *__restrict__ rbase,
    const V *__restrict__ val, const typename VT<V>::A *__restrict__ x,
    typename VT<V>::A *__restrict__ y, int kmin) {
    rowstream_block<V, D16, R, false>(xcd_remap(blockIdx.x, gridDim.x), n, rp, ci, off, rbase, val, x, y,
                                      kmin);
}

// Lane l receives lane l + 1's value (DPP wave shift; the last lane keeps
// its own, to be replaced by the caller).
__device__ __forceinline__ float wave_shl1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x130,
                                                      0xF, 0xF, false));
}
__device__ __forceinline__ double wave_shl1(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xF, 0xF, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xF, 0xF, false));
}

// ============================================================ delta16, sliced
// The sliced layout (slices of 64 rows, one row per lane, nonzeros stored
// column-major in pairs; see k_sliced_scatter).  The column codes of offset
// slices are O = uint16_t offsets from the slice's reference column, or
// O = uint8_t deltas from the row's previous column with the escape code 255
// (the column then read from the lane's next escape entry); one width per
// matrix, as the paper's deltas.  Lane l
// of the wavefront of slice s sums its row in column order from +0, so FP64
// results equal the sequential sum bit for bit.  Each step loads two pairs per
// lane (a wavefront load is 64 consecutive pairs, coalesced), then gathers
// their four x entries: on stencils the lanes' columns are consecutive too.
// Every lane loads every pair up to the slice width (padding slots hold zero
// offsets, so their gathers stay in range); products past the row's end are
// dropped, which keeps the loads free of per-lane branches.  A step whose
// second pair lies past the width skips it (a wavefront-uniform branch) with
// 16-bit offsets and in diagonal slices, 2-4% on short rows, whose slices
// are one pair wide; with 8-bit codes it reloads the last pair instead (the
// branch cost 3-5% on bands there).  y is written with
// streaming (non-temporal) stores: 4% faster on the 27-point stencil and 10%
// on short rows from a flushed cache, and no slower warm.
template <class V, class O>
__global__ __launch_bounds__(kBlock) void k_sliced_d16(
    int64_t n, int64_t m, int64_t nsl, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ width, const int32_t *__restrict__ units,
    const int32_t *__restrict__ base, const int32_t *__restrict__ kind,
    const int32_t *__restrict__ diag, const uint32_t *__restrict__ mask,
    const int32_t *__restrict__ span, const int32_t *__restrict__ perm,
    const O *__restrict__ off, const int32_t *__restrict__ eunits,
    const int32_t *__restrict__ esc, const V *__restrict__ val,
    const typename VT<V>::A *__restrict__ x, typename VT<V>::A *__restrict__ y, int kmin) {
    using A = typename VT<V>::A;
    using VP = typename Pair<V>::type;
    using OP = typename Pair<O>::type;
    const int64_t sl = xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kSellRows) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / kSellRows);
    if (sl >= nsl) return;  // whole wavefronts leave together
    const int lane = threadIdx.x & (kSellRows - 1);
    // The slice's descriptors and first four diagonals, all loaded before
    // any is used, so that they cost one scalar round trip; the loads that
    // depend on the lane's row take clamped indices instead of a branch, so
    // that none waits before the step loop issues its own.
    const int w = width[sl];
    const int32_t u = units[sl];
    const int kd = kind[sl];
    const int32_t b = base[sl];
    const int sp = span[sl];
    const int32_t eu = sizeof(O) == 1 ? eunits[sl] : 0;
    const int4 *dg4 = reinterpret_cast<const int4 *>(diag + sl * kSellMaxDiag);
    int4 dn = dg4[0];
    // the row this lane owns: the position's, or the one the length-sorted
    // layout put there (that layout has offset slices only)
    const int64_t pos = sl * kSellRows + lane;
    const int64_t pc = pos < n ? pos : n - 1;  // (n >= 1: slice sl has a row)
    const int64_t r = perm ? (pos < n ? (int64_t)perm[pc] : pos) : pos;
    const int64_t rc = r < n ? r : n - 1;
    const int64_t o = 2 * kSellRows * (int64_t)u + 2 * lane;
    if (kd > 0) {
        // diagonal slice: the column of position k is r + dg[k] (the same
        // diagonals for every lane, so those are scalar loads, four per step
        // and one step ahead); only values are streamed, and the row's mask
        // says which positions it has.  Rows here hold at most 32 nonzeros,
        // so FP32 needs no Kahan sum.
        // (a lane past the last row reads row N-1's mask: its sum is not
        // stored; no select here, which would wait for the load at once)
        const uint32_t mk = mask[rc];
        const int64_t r0 = sl * kSellRows;
        A acc = A(0);
        // consecutive diagonals d, d + 1 (stencils): lane l's x[r + d + 1] is
        // lane l + 1's x[r + d], shifted down the wavefront (DPP), and only
        // the last lane loads (a uniform address, through the scalar cache):
        // a third of the x loads of a 27-point stencil go through the
        // vector memory path.  Slices narrower than 8 positions load every
        // x (there the shift's dependence on the previous load costs more
        // than the load it saves: 17% on short rows)
        const bool reuse = w >= 8;
        A xp = A(0);
        int32_t dp = INT32_MIN;
        for (int k0 = 0; k0 < w; k0 += 4) {
            const int32_t dd[4] = {dn.x, dn.y, dn.z, dn.w};  // diagonals k0 .. k0 + 3
            if (k0 + 4 < w) dn = dg4[k0 / 4 + 1];            // the next step's (uniform)
            const VP v0 = __builtin_nontemporal_load(
                reinterpret_cast<const VP *>(val + o + (int64_t)(k0 / 2) * (2 * kSellRows)));
            const bool two = k0 + 2 < w;  // wavefront-uniform: the step has a second pair
            VP v1 = {};
            if (two)
                v1 = __builtin_nontemporal_load(
                    reinterpret_cast<const VP *>(val + o + (int64_t)(k0 / 2 + 1) * (2 * kSellRows)));
            A xv[4] = {A(0), A(0), A(0), A(0)};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i >= 2 && !two) break;
                const int32_t dk = dd[i];
                A xk;
                if (reuse && dp != INT32_MIN && dk == dp + 1) {
                    int64_t c = r0 + (kSellRows - 1) + dk;
                    c = c < 0 ? 0 : (c >= m ? m - 1 : c);
                    const A e = x[c];
                    const A sh = wave_shl1(xp);
                    xk = lane == kSellRows - 1 ? e : sh;
                } else {  // a position the row lacks may point outside x
                    int64_t c = r + dk;
                    c = c < 0 ? 0 : (c >= m ? m - 1 : c);
                    xk = x[c];
                }
                xv[i] = xk;
                xp = xk;
                dp = dk;
            }
            const A p[4] = {VT<V>::cvt(v0.x) * xv[0], VT<V>::cvt(v0.y) * xv[1],
                            VT<V>::cvt(v1.x) * xv[2], VT<V>::cvt(v1.y) * xv[3]};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k0 + i;
                // a +0 addend leaves a sum that started at +0 unchanged
                acc = acc + ((k < w && ((mk >> k) & 1u)) ? p[i] : A(0));
            }
        }
        if (r < n) __builtin_nontemporal_store(acc, y + r);
        return;
    }
    // the row's nonzeros are [ra, re) (a lane past the last row takes row
    // N-1's and does not store its sum); position k is in the row when
    // ra + k < re, a test the step makes after its own loads, so that these
    // two are not waited for before the step loop starts (in 32-bit unsigned
    // arithmetic: ra + k stays below 2^32 where a signed sum could pass
    // 2^31 - 1 in a wide slice near the end of the nonzeros)
    const int32_t ra = rp[rc], re = rp[rc + 1];
    const uint32_t ua = (uint32_t)ra, ue = (uint32_t)re;
    const bool comp = is_f32<A>() && re - ra >= kmin;
    Sum<A> acc;
    int32_t cprev = b;  // 8-bit codes: the previous column
    const int32_t *ep = nullptr;  // 8-bit codes: this lane's next escape entry
    int64_t oq = 0;  // 8-bit codes: this lane's first group of four
    if constexpr (sizeof(O) == 1) {
        ep = esc + (int64_t)kSellRows * eu + lane;
        oq = 2 * kSellRows * ((int64_t)units[sl] + sl) + 4 * lane;
    }
    // x staging (sell_stages_x): the slice reads x from a copy of its
    // column window in LDS, loaded coalesced.  Band matrices keep the vector
    // memory path's address unit 90% busy with their x gathers otherwise;
    // from LDS they run 8-20% faster (half widths 16 to 200).  16 KiB per
    // workgroup leaves the occupancy at 8 waves per SIMD.
    constexpr int kXs = kSellXWindow;
    __shared__ A xs[kBlock / kSellRows][kXs];
    const int wv = threadIdx.x / kSellRows;
    const bool staged = sell_stages_x(sp, w);
    auto run = [&](auto st) {
        constexpr bool ST = decltype(st)::value;
        A *xw = &xs[wv][0];
        if constexpr (ST) {
            for (int i = lane; i <= sp; i += kSellRows) xw[i] = x[b + i];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // x of column c: from the window in LDS, or from memory
#define GX(c) (ST ? xw[(c) - b] : x[(c)])
        for (int k0 = 0; k0 < w; k0 += 4) {
            const int k1 = (k0 + 2) < w ? k0 + 2 : w - 2;  // past the width: reload the last pair
            const int64_t q0 = o + (int64_t)(k0 / 2) * (2 * kSellRows);
            const int64_t q1 = o + (int64_t)(k1 / 2) * (2 * kSellRows);
            VP v0, v1;
            A x0, x1, x2, x3;
            if constexpr (sizeof(O) == 1) {
                // this lane's four codes of the step in one 4-byte load
                // (positions past the width hold code 0, as padding positions
                // do, and keep the column).  Two 2-byte loads per step, codes
                // stored in pairs like the values, ran a 2M-row band in 305 us
                // cold against 256 us for this (FP64; 16-bit offsets: 277 us)
                const uint32_t cq = __builtin_nontemporal_load(
                    reinterpret_cast<const uint32_t *>(off + oq + (int64_t)k0 * kSellRows));
                v0 = __builtin_nontemporal_load(reinterpret_cast<const VP *>(val + q0));
                v1 = __builtin_nontemporal_load(reinterpret_cast<const VP *>(val + q1));
                const int32_t d[4] = {(int32_t)(cq & 0xff), (int32_t)((cq >> 8) & 0xff),
                                      (int32_t)((cq >> 16) & 0xff), (int32_t)(cq >> 24)};
                const bool esc4 = d[0] == 255 || d[1] == 255 || d[2] == 255 || d[3] == 255;
                int32_t col[4];
                if (__any(esc4)) {  // wavefront-uniform: most steps load no escape
    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (d[i] == 255) {
                            cprev = *ep;
                            ep += kSellRows;
                        } else {
                            cprev += d[i];
                        }
                        col[i] = cprev;
                    }
                    // settle the escape loads on this rare path: left pending,
                    // the paths join with a wait for every load in flight, and
                    // the common path's gathers would also wait for this step's
                    // value loads
                    __builtin_amdgcn_s_waitcnt(0);
                } else {
                    col[0] = cprev + d[0];
                    col[1] = col[0] + d[1];
                    col[2] = col[1] + d[2];
                    col[3] = col[2] + d[3];
                    cprev = col[3];
                }
                x0 = GX(col[0]);
                x1 = GX(col[1]);
                x2 = GX(col[2]);
                x3 = GX(col[3]);
            } else {
                v0 = __builtin_nontemporal_load(reinterpret_cast<const VP *>(val + q0));
                const OP c0 = __builtin_nontemporal_load(reinterpret_cast<const OP *>(off + q0));
                x0 = GX(b + (int32_t)c0.x);
                x1 = GX(b + (int32_t)c0.y);
                if (k0 + 2 < w) {  // wavefront-uniform: the step has a second pair
                    v1 = __builtin_nontemporal_load(reinterpret_cast<const VP *>(val + q1));
                    const OP c1 = __builtin_nontemporal_load(reinterpret_cast<const OP *>(off + q1));
                    x2 = GX(b + (int32_t)c1.x);
                    x3 = GX(b + (int32_t)c1.y);
                } else {
                    v1 = VP{};
                    x2 = x3 = A(0);
                }
            }
            const A p[4] = {VT<V>::cvt(v0.x) * x0, VT<V>::cvt(v0.y) * x1, VT<V>::cvt(v1.x) * x2,
                            VT<V>::cvt(v1.y) * x3};
    #pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (comp) {
                    if (ua + (uint32_t)(k0 + i) < ue) acc.add_comp(p[i]);
                } else {
                    // a +0 addend leaves a sum that started at +0 unchanged
                    acc.add(ua + (uint32_t)(k0 + i) < ue ? p[i] : A(0));
                }
            }
        }
#undef GX
    };
    if (staged)
        run(std::true_type{});
    else
        run(std::false_type{});
    if (r < n) __builtin_nontemporal_store(acc.s, y + r);
}

// ============================================================ merge path
// Merrill and Garland's merge-based CSR SpMV.  Tile t covers the merge
// diagonals [t*T, (t+1)*T) of row ends rowptr[1..N] and nonzero indices;
// its start coordinates come precomputed.  Products and row ends are staged
// in LDS; each thread finds its own start by a merge-path search in LDS and
// consumes 8 items: a nonzero adds its product, a row end emits the row.
// Rows finished inside one thread are summed in column order.  The first
// row end of a thread adds the partial sums carried by the preceding
// threads of the tile (in thread order); the partial row left at the tile's
// end is stored as the tile's carry and added by k_merge_fixup in tile order.
template <class V>
struct MergeSmem {
    using A = typename VT<V>::A;
    int32_t end[kMergeTile + 1];
    A prod[kMergeTile];
    int32_t crow[kBlock];
    A cval[kBlock];
};

// D16: the columns are tbase[tile] + off[j], 16-bit codes from the tile's
// smallest column (delta16 inside merge-path tiles).
template <class V, bool D16 = false>
__device__ __forceinline__ void merge_tile(MergeSmem<V> &sm, int64_t tile, int64_t n,
                                           const int32_t *__restrict__ rp,
                                           const int32_t *__restrict__ ci,
                                           const V *__restrict__ val,
                                           const typename VT<V>::A *__restrict__ x,
                                           typename VT<V>::A *__restrict__ y,
                                           const int32_t *__restrict__ srow,
                                           const int32_t *__restrict__ snnz,
                                           int32_t *__restrict__ carry_row,
                                           typename VT<V>::A *__restrict__ carry_val, bool comp,
                                           const uint16_t *__restrict__ off = nullptr,
                                           const int32_t *__restrict__ tbase = nullptr) {
    using A = typename VT<V>::A;
    const int32_t i0 = srow[tile], j0 = snnz[tile];
    const int32_t i1 = srow[tile + 1], j1 = snnz[tile + 1];
    const int nr = i1 - i0, nz = j1 - j0;

    for (int r = threadIdx.x; r <= nr; r += kBlock) {
        const int64_t row = (int64_t)i0 + r;
        sm.end[r] = row < n ? rp[row + 1] : INT32_MAX;
    }
    {
        // all of this thread's index and value loads first, then the gathers,
        // so every load of the tile is in flight at once
        constexpr int PPT = kMergeTile / kBlock;
        int32_t c[PPT];
        V v[PPT];
        const int32_t tb = D16 ? tbase[tile] : 0;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int q = threadIdx.x + j * kBlock;
            if (D16) c[j] = q < nz ? tb + (int32_t)ld_nt(off + j0 + q) : 0;
            else c[j] = q < nz ? ld_nt(ci + j0 + q) : 0;
            v[j] = q < nz ? ld_nt(val + j0 + q) : V(0);
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int q = threadIdx.x + j * kBlock;
            if (q < nz) sm.prod[q] = VT<V>::cvt(v[j]) * x[c[j]];
        }
    }
    __syncthreads();

    // this thread's start on the merge path inside the tile
    const int total = nr + nz;
    const int d = (int)threadIdx.x * kMergeIpt < total ? (int)threadIdx.x * kMergeIpt : total;
    int lo = d - nz > 0 ? d - nz : 0, hi = d < nr ? d : nr;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sm.end[mid] <= j0 + d - mid - 1) lo = mid + 1; else hi = mid;
    }
    int xi = lo, yj = d - lo;

    Sum<A> run;
    int head_row = -1;
    A head_val = A(0);
    const int dend = (d + kMergeIpt) < total ? (d + kMergeIpt) : total;
    for (int it = d; it < dend; ++it) {
        if (yj < nz && j0 + yj < sm.end[xi]) {
            run.add(sm.prod[yj], comp);
            ++yj;
        } else {
            if (head_row < 0) {
                head_row = xi;
                head_val = run.s;
            } else {
                y[i0 + xi] = run.s;
            }
            run.reset();
            ++xi;
        }
    }
    sm.crow[threadIdx.x] = xi;  // row (local) still open at this thread's end
    sm.cval[threadIdx.x] = run.s;
    __syncthreads();

    if (head_row >= 0) {
        int t0 = threadIdx.x;
        while (t0 > 0 && sm.crow[t0 - 1] == head_row) --t0;
        Sum<A> c;
        for (int t = t0; t < (int)threadIdx.x; ++t) c.add(sm.cval[t], comp);
        c.add(head_val, comp);
        y[i0 + head_row] = c.s;
    }
    if (threadIdx.x == kBlock - 1) {
        // partial sums of row i1 accumulated in this tile (continues later)
        int t0 = kBlock - 1;
        while (t0 > 0 && sm.crow[t0 - 1] == nr) --t0;
        Sum<A> c;
        if (sm.crow[kBlock - 1] == nr)
            for (int t = t0; t < kBlock; ++t) c.add(sm.cval[t], comp);
        carry_row[tile] = i1;
        carry_val[tile] = c.s;
    }
}

template <class V, bool D16>
__global__ __launch_bounds__(kBlock) void k_merge_path(
    int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const V *__restrict__ val, const typename VT<V>::A *__restrict__ x,
    typename VT<V>::A *__restrict__ y, const int32_t *__restrict__ srow,
    const int32_t *__restrict__ snnz, int32_t *__restrict__ carry_row,
    typename VT<V>::A *__restrict__ carry_val, int kmin, const uint16_t *__restrict__ off,
    const int32_t *__restrict__ tbase) {
    __shared__ MergeSmem<V> sm;
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    merge_tile<V, D16>(sm, tile, n, rp, ci, val, x, y, srow, snnz, carry_row, carry_val,
                       is_f32<typename VT<V>::A>() && kmin < INT32_MAX, off, tbase);
}

// Adds the carries of consecutive tiles that end inside the same row, in
// tile order, to that row (the tile finishing the row already wrote its
// own part).  One thread per tile; only the first tile of a run works.
template <class A>
__device__ __forceinline__ void merge_fixup_one(int64_t t, int64_t n, int64_t tiles,
                                                const int32_t *__restrict__ carry_row,
                                                const A *__restrict__ carry_val,
                                                A *__restrict__ y, bool comp) {
    if (t >= tiles) return;
    const int32_t row = carry_row[t];
    if (row >= n) return;
    if (t > 0 && carry_row[t - 1] == row) return;
    Sum<A> c;
    for (int64_t u = t; u < tiles && carry_row[u] == row; ++u) c.add(carry_val[u], comp);
    y[row] = y[row] + c.s;
}

template <class A>
__global__ __launch_bounds__(kBlock) void k_merge_fixup(int64_t n, int64_t tiles,
                                                        const int32_t *__restrict__ carry_row,
                                                        const A *__restrict__ carry_val,
                                                        A *__restrict__ y, int kmin) {
    merge_fixup_one<A>(blockIdx.x * (int64_t)kBlock + threadIdx.x, n, tiles, carry_row, carry_val, y,
                       is_f32<A>() && kmin < INT32_MAX);
}

// ============================================================ x blocking
// The column range is cut into S equal slices (S = 1, 2, 4 or 8, sized so a
// slice of x is at most 4 MB).  Slice s is a CSR matrix of its own (all rows,
// the nonzeros whose columns fall in the slice).  Workgroup b runs on XCD
// x = b mod 8 and works on slice x mod S, so each XCD gathers from one slice
// of x only, which stays in its 4 MB L2 instead of being fetched line by
// line from the Infinity Cache; the 8/S XCDs of a slice take its row blocks
// (or tiles) in turn.  Each slice writes a partial y; k_slice_sum adds the
// partials in slice order.  Where no row leaves the slices, k_phased_slices
// (below) walks the slices in time instead and needs no partial y.
// Work unit (row block or tile) and slice of workgroup b.
__device__ inline int64_t slice_unit(int ns, int *slice) {
    const int x = blockIdx.x % 8;
    *slice = x % ns;
    return (int64_t)(blockIdx.x / 8) * (8 / ns) + x / ns;
}

template <class A>
struct SliceTable {
    int ns;  // slice count S
    const int32_t *rp[kSlices];
    const int32_t *srow[kSlices];
    const int32_t *snnz[kSlices];
    int32_t *crow[kSlices];
    A *cval[kSlices];
    A *y[kSlices];
    int64_t off[kSlices];
    int64_t tiles[kSlices];
    // 16-bit column codes of the slice-major arrays (same positions as the
    // int32 columns) and, per slice, the reference column of each row block
    const uint16_t *code;
    const int32_t *cb[kSlices];
};

template <class V>
__global__ __launch_bounds__(kBlock) void k_merge_slices(int64_t n, const int32_t *__restrict__ ci,
                                                         const V *__restrict__ val,
                                                         const typename VT<V>::A *__restrict__ x,
                                                         SliceTable<typename VT<V>::A> T, int kmin) {
    __shared__ MergeSmem<V> sm;
    int s;
    const int64_t tile = slice_unit(T.ns, &s);
    if (tile >= T.tiles[s]) return;
    merge_tile<V>(sm, tile, n, T.rp[s], ci + T.off[s], val + T.off[s], x, T.y[s], T.srow[s],
                  T.snnz[s], T.crow[s], T.cval[s], is_f32<typename VT<V>::A>() && kmin < INT32_MAX);
}

// Long rows of the split, summed from the original CSR: one block per chunk
// of at most kLongChunk nonzeros of one row inside one column slice (all
// loads first, then the gathers; per-thread sums folded by a fixed tree;
// these blocks ride at the end of the slice kernel's grid, filling CUs as
// slice blocks finish, each on an XCD that gathers from its chunk's slice);
// then k_slice_finish gives each long row a wavefront that adds its chunk
// sums in column order.
// `sh` is kBlock elements of the calling kernel's LDS (its own arrays, so
// the chunk blocks add nothing to the kernel's LDS size and occupancy).
template <class V>
__device__ __forceinline__ void long_chunk_block(int64_t c, const int32_t *__restrict__ ck0,
                                                 const int32_t *__restrict__ ck1,
                                                 const int32_t *__restrict__ ci,
                                                 const V *__restrict__ val,
                                                 const typename VT<V>::A *__restrict__ x,
                                                 typename VT<V>::A *__restrict__ lsum,
                                                 typename VT<V>::A *sh) {
    using A = typename VT<V>::A;
    constexpr int PPT = kLongChunk / kBlock;
    const int32_t k0 = ck0[c], k1 = ck1[c];
    int32_t cc[PPT];
    V v[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int32_t k = k0 + (int32_t)threadIdx.x + j * kBlock;
        cc[j] = k < k1 ? ld_nt(ci + k) : 0;
        v[j] = k < k1 ? ld_nt(val + k) : V(0);
    }
    A t = A(0);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int32_t k = k0 + (int32_t)threadIdx.x + j * kBlock;
        if (k < k1) t = t + VT<V>::cvt(v[j]) * x[cc[j]];
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) lsum[c] = sh[0];
}

// Short slice rows: row-block streaming on each slice; workgroups from
// `sgrid` on sum the long-row chunks instead.
struct LongChunks {
    const int32_t *ck0, *ck1, *ci;
    const void *val;
    void *lsum;
    const int32_t *cmap;  // the chunk of each chunk workgroup (-1: none)
};

template <class V, int R, bool D16>
__global__ __launch_bounds__(kBlock) void k_rowstream_slices(int64_t n, int64_t nblocks,
                                                             const int32_t *__restrict__ ci,
                                                             const V *__restrict__ val,
                                                             const typename VT<V>::A *__restrict__ x,
                                                             SliceTable<typename VT<V>::A> T,
                                                             int64_t sgrid, LongChunks LC, int kmin) {
    using A = typename VT<V>::A;
    if ((int64_t)blockIdx.x >= sgrid) {
        __shared__ A sh[kBlock];
        const int32_t c = LC.cmap[(int64_t)blockIdx.x - sgrid];
        if (c < 0) return;  // the same for the whole workgroup
        long_chunk_block<V>(c, LC.ck0, LC.ck1, LC.ci, static_cast<const V *>(LC.val), x,
                            static_cast<A *>(LC.lsum), sh);
        return;
    }
    int s;
    const int64_t b = slice_unit(T.ns, &s);
    if (b >= nblocks) return;
    rowstream_block<V, D16, R, true>(b, n, T.rp[s], ci + T.off[s], D16 ? T.code + T.off[s] : nullptr,
                                     D16 ? T.cb[s] : nullptr, val + T.off[s], x, T.y[s], kmin);
}

// Phased row streaming on the slices, without partial y vectors.  Workgroup
// w owns the consecutive 256-row blocks [w nblk / G, (w + 1) nblk / G) (at
// most J of them) and walks the slices in order; in each slice it streams the
// nonzeros of all its rows as one run, thread t summing rows t, t + 256, ...
// of its range, each row's sum kept in a register across the slices.  The
// slices are column ranges in increasing order, so every row is summed in
// column order: Algorithm 1's order, bit for bit in FP64.  The grid holds at
// most as many of these workgroups as the CUs run at once, so they walk the
// slices together and the part of x being gathered at any time is about one
// slice, which the L2s hold.  Used when no row leaves the slices: the long
// rows' chunk sums, run as extra workgroups of this grid, as a kernel of
// their own or after the slices, all cost more than the per-slice kernel
// with partial y vectors below saves.
// The block of a phased run (nb blocks, the first positions s_rp[j kBlock])
// holding position kk: the last whose first position is at most kk, so
// empty blocks are passed over.
__device__ __forceinline__ int run_block_of(const int32_t *s_rp, int nb, int32_t kk) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_rp[mid * kBlock] <= kk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <class V, int J, bool D16>
__global__ __launch_bounds__(kBlock) void k_phased_slices(
    int64_t n, int64_t nblk, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const V *__restrict__ val, const typename VT<V>::A *__restrict__ x,
    SliceTable<typename VT<V>::A> T, typename VT<V>::A *__restrict__ y, int kmin) {
    using A = typename VT<V>::A;
    using VP = typename Pair<V>::type;
    using IP = typename Pair<int32_t>::type;
    using OP = typename Pair<uint16_t>::type;
    constexpr int NP = kRunLen / 2;  // pairs per thread per chunk
    __shared__ int32_t s_rp[J * kBlock + 1];
    __shared__ int32_t s_cb[J];
    __shared__ A s_prod[kChunk];
    const int64_t G = gridDim.x, w = blockIdx.x;
    const int t = threadIdx.x;
    // the block range (at least one block: G <= nblk; at most J: G >= nblk / J)
    const int64_t b0 = w * nblk / G, b1 = (w + 1) * nblk / G;
    const int64_t r0 = b0 * kBlock;
    const int64_t rlim = b1 * kBlock < n ? b1 * kBlock : n;
    const int nrows = (int)(rlim - r0);
    const int nb = (nrows + kBlock - 1) / kBlock;  // blocks in the run (1 .. J)
    Sum<A> acc[J];
    bool comp[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int lr = j * kBlock + t;
        comp[j] = is_f32<A>() && lr < nrows && (rp[r0 + lr + 1] - rp[r0 + lr]) >= kmin;
    }
    for (int sl = 0; sl < T.ns; ++sl) {
        const int32_t *__restrict__ srp = T.rp[sl];
        const int32_t *__restrict__ sci = ci + T.off[sl];
        const uint16_t *__restrict__ soff = D16 ? T.code + T.off[sl] : nullptr;
        const V *__restrict__ sv = val + T.off[sl];
        __syncthreads();  // the previous slice is done with s_rp and s_prod
        for (int r = t; r <= nrows; r += kBlock) s_rp[r] = srp[r0 + r];
        if (D16 && t < J) s_cb[t] = b0 + t < b1 ? T.cb[sl][b0 + t] : 0;
        __syncthreads();
        const int32_t a = s_rp[0], e = s_rp[nrows];
        int32_t k[J], kend[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int lr = j * kBlock + t;
            k[j] = lr < nrows ? s_rp[lr] : e;
            kend[j] = lr < nrows ? s_rp[lr + 1] : e;
        }
        for (int32_t cs = a & ~1; cs < e; cs += kChunk) {
            A p[kRunLen];
            // each pair's gathers follow its own loads: with more gathers in
            // flight per thread (all loads first) the kernel ran slower, its
            // L1 miss slots being the limit
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int32_t kk = cs + 2 * t + 2 * kBlock * q;
                V v0 = V(0), v1 = V(0);
                int32_t c0 = 0, c1 = 0;
                if (kk + 1 < e) {
                    const VP vv = __builtin_nontemporal_load(reinterpret_cast<const VP *>(sv + kk));
                    v0 = vv.x;
                    v1 = vv.y;
                    if (D16) {
                        const OP oo = __builtin_nontemporal_load(reinterpret_cast<const OP *>(soff + kk));
                        const int j0 = run_block_of(s_rp, nb, kk);
                        int j1 = j0;
                        while (j1 + 1 < nb && kk + 1 >= s_rp[(j1 + 1) * kBlock]) ++j1;
                        c0 = s_cb[j0] + (int32_t)oo.x;
                        c1 = s_cb[j1] + (int32_t)oo.y;
                    } else {
                        const IP cc = __builtin_nontemporal_load(reinterpret_cast<const IP *>(sci + kk));
                        c0 = cc.x;
                        c1 = cc.y;
                    }
                } else if (kk < e) {
                    v0 = sv[kk];
                    c0 = D16 ? s_cb[run_block_of(s_rp, nb, kk)] + (int32_t)soff[kk] : sci[kk];
                }
                const bool ok0 = kk >= a && kk < e, ok1 = kk + 1 >= a && kk + 1 < e;
                p[2 * q] = ok0 ? VT<V>::cvt(v0) * x[c0] : A(0);
                p[2 * q + 1] = ok1 ? VT<V>::cvt(v1) * x[c1] : A(0);
            }
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                s_prod[2 * t + 2 * kBlock * q] = p[2 * q];
                s_prod[2 * t + 2 * kBlock * q + 1] = p[2 * q + 1];
            }
            __syncthreads();
            const int32_t ce = (cs + kChunk) < e ? (cs + kChunk) : e;
#pragma unroll
            for (int j = 0; j < J; ++j)
                for (; k[j] < kend[j] && k[j] < ce; ++k[j]) acc[j].add(s_prod[k[j] - cs], comp[j]);
            __syncthreads();
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int lr = j * kBlock + t;
        if (lr < nrows) __builtin_nontemporal_store(acc[j].s, y + r0 + lr);
    }
}

template <class A>
__global__ __launch_bounds__(kBlock) void k_merge_fixup_slices(int64_t n, int64_t maxt,
                                                               SliceTable<A> T, int kmin) {
    const int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const int s = (int)(g / (maxt > 0 ? maxt : 1));
    if (s >= T.ns) return;
    merge_fixup_one<A>(g % maxt, n, T.tiles[s], T.crow[s], T.cval[s], T.y[s],
                       is_f32<A>() && kmin < INT32_MAX);
}

// The sum of row i's partials in slice order; the NS loads are issued
// together (streamed once: non-temporal), then added in order.
template <class A, int NS>
__device__ __forceinline__ A slice_total(const SliceTable<A> &T, int64_t i) {
    A v[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = __builtin_nontemporal_load(T.y[k] + i);
    A s = v[0];
#pragma unroll
    for (int k = 1; k < NS; ++k) s = s + v[k];
    return s;
}

// Slice sums and long rows in one launch: blocks below gsum add the partial
// y vectors in slice order for every row whose bit in `longmask` is clear;
// the blocks after them give each long row a wavefront that adds its chunk
// sums (per lane in order, Kahan for FP32, then a fixed butterfly) and
// stores the row.  The two sets of rows are disjoint.
template <class A, int NS>
__global__ __launch_bounds__(kBlock) void k_slice_finish(int64_t n, SliceTable<A> T,
                                                         A *__restrict__ y, int64_t gsum,
                                                         const uint32_t *__restrict__ longmask,
                                                         int64_t L, const int32_t *__restrict__ rows,
                                                         const int32_t *__restrict__ first,
                                                         const A *__restrict__ lsum, int kmin) {
    if ((int64_t)blockIdx.x < gsum) {
        // the partials are loaded with the row's mask word, not after it (a
        // long row's partials are zeros, loaded and dropped); the empty asm
        // uses the sum before the test, so that the loads are not sunk into it
        for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += gsum * kBlock) {
            const uint32_t w = longmask[i >> 5];
            const A v = slice_total<A, NS>(T, i);
            __asm__ volatile("" : : "v"(v));
            if (!((w >> (i & 31)) & 1u)) __builtin_nontemporal_store(v, y + i);
        }
        return;
    }
    const int64_t t = (((int64_t)blockIdx.x - gsum) * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (t >= L) return;  // whole wavefronts leave together
    Sum<A> acc;
    for (int32_t c = first[t] + lane; c < first[t + 1]; c += 64)
        acc.add(lsum[c], is_f32<A>() && kmin < INT32_MAX);
    const A v = group_sum<64>(acc.s);
    if (lane == 0) y[rows[t]] = v;
}

template <class A, int NS>
__global__ __launch_bounds__(kBlock) void k_slice_sum(int64_t n, SliceTable<A> T,
                                                      A *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        __builtin_nontemporal_store(slice_total<A, NS>(T, i), y + i);
}

// ============================================================ launchers
namespace {

template <class F>
hipError_t by_dtype(int dtype, F &&f) {
    switch (dtype) {
    case SPMV_F64: return f((const double *)nullptr);
    case SPMV_F32: return f((const float *)nullptr);
    default: return f((const uint16_t *)nullptr);
    }
}

inline unsigned grid_for(int64_t items, int per_block, int64_t cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_csr_scalar(const spmv_plan &P, const void *x, void *y, hipStream_t s) {
    if (P.n == 0) return hipSuccess;
    return by_dtype(P.dtype, [&](auto tag) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(tag)>>;
        using A = typename VT<V>::A;
        const unsigned g = grid_for(P.n, kBlock, INT32_MAX);
        hipLaunchKernelGGL(k_csr_scalar<V>, dim3(g), dim3(kBlock), 0, s, P.n, P.rowptr, P.colind,
                           (const V *)P.val, (const A *)x, (A *)y, P.kahan_min);
        return hipGetLastError();
    });
}

hipError_t launch_csr_vector(const spmv_plan &P, const void *x, void *y, hipStream_t s) {
    if (P.n == 0) return hipSuccess;
    return by_dtype(P.dtype, [&](auto tag) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(tag)>>;
        using A = typename VT<V>::A;
        const int W = P.vec_width;
        const unsigned g = grid_for(P.n, kBlock / W, (int64_t)P.num_cus * 32);
#define SPMV_VEC(WW)                                                                       \
    case WW:                                                                               \
        hipLaunchKernelGGL((k_csr_vector<V, WW>), dim3(g), dim3(kBlock), 0, s, P.n, P.rowptr, \
                           P.colind, (const V *)P.val, (const A *)x, (A *)y, P.kahan_min); \
        break;
        switch (W) {
            SPMV_VEC(2) SPMV_VEC(4) SPMV_VEC(8) SPMV_VEC(16) SPMV_VEC(32) SPMV_VEC(64)
        default: return hipErrorInvalidValue;
        }
#undef SPMV_VEC
        return hipGetLastError();
    });
}

hipError_t launch_rowstream(const spmv_plan &P, bool d16, const void *x, void *y, hipStream_t s) {
    if (P.n == 0) return hipSuccess;
    return by_dtype(P.dtype, [&](auto tag) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(tag)>>;
        using A = typename VT<V>::A;
        const int R = d16 ? P.d16_rows / kBlock : P.rs_rows;
        const unsigned g = grid_for(P.n, kBlock * R, INT32_MAX);
        const uint16_t *off = P.d16_off.as<uint16_t>();
        const int32_t *base = P.d16_base.as<int32_t>();
#define SPMV_RS(RR)                                                                               \
    case RR:                                                                                      \
        if (d16)                                                                                  \
            hipLaunchKernelGGL((k_rowstream<V, true, RR>), dim3(g), dim3(kBlock), 0, s, P.n,     \
                               P.rowptr, P.colind, off, base, (const V *)P.val, (const A *)x,    \
                               (A *)y, P.kahan_min);                                              \
        else                                                                                      \
            hipLaunchKernelGGL((k_rowstream<V, false, RR>), dim3(g), dim3(kBlock), 0, s, P.n,    \
                               P.rowptr, P.colind, (const uint16_t *)nullptr,                     \
                               (const int32_t *)nullptr, (const V *)P.val, (const A *)x, (A *)y,  \
                               P.kahan_min);                                                      \
        break;
        switch (R) {
            SPMV_RS(1) SPMV_RS(2) SPMV_RS(4) SPMV_RS(8)
        default: return hipErrorInvalidValue;
        }
#undef SPMV_RS
        return hipGetLastError();
    });
}

// Geometry of the phased x-block kernel: the fewest row blocks per workgroup
// J (1, 2, 4 or 8) for which ceil(blocks / J) workgroups fit on the CUs at
// once (by the occupancy the runtime reports for that instance); G is then
// as many workgroups as fit, at most one per block, each taking a range of
// at most J consecutive blocks.  Else J = 8 and G = ceil(blocks / 8), more
// workgroups than fit.
hipError_t phased_geometry(const spmv_plan &P, int *J, int64_t *G) {
    const int64_t nblk = (P.n + kBlock - 1) / kBlock;
    return by_dtype(P.dtype, [&](auto tag) -> hipError_t {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(tag)>>;
        const void *fns[4] = {reinterpret_cast<const void *>(&k_phased_slices<V, 1, false>),
                              reinterpret_cast<const void *>(&k_phased_slices<V, 2, false>),
                              reinterpret_cast<const void *>(&k_phased_slices<V, 4, false>),
                              reinterpret_cast<const void *>(&k_phased_slices<V, 8, false>)};
        for (int i = 0; i < 4; ++i) {
            const int j = 1 << i;
            int per_cu = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fns[i], kBlock, 0);
            if (e != hipSuccess) return e;
            const int64_t need = (nblk + j - 1) / j, cap = (int64_t)P.num_cus * per_cu;
            if (need <= cap || j == 8) {  // all slots that fit, for the smallest J
                *J = j;
                *G = need <= cap ? (cap < nblk ? cap : nblk) : need;
                if (*G < 1) *G = 1;
                return hipSuccess;
            }
        }
        return hipErrorInvalidValue;
    });
}

hipError_t launch_sliced_d16(const spmv_plan &P, const void *x, void *y, hipStream_t s) {
    if (P.n == 0) return hipSuccess;
    if (P.d16_offw != 8 && P.d16_offw != 16) return hipErrorInvalidValue;
    return by_dtype(P.dtype, [&](auto tag) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(tag)>>;
        using A = typename VT<V>::A;
        const int64_t per = kBlock / kSellRows;
        const unsigned g = (unsigned)((P.d16_nsl + per - 1) / per);
        const int32_t *perm = P.d16_sort ? P.d16s_perm.as<int32_t>() : nullptr;
        if (P.d16_offw == 8)
            hipLaunchKernelGGL((k_sliced_d16<V, uint8_t>), dim3(g), dim3(kBlock), 0, s, P.n, P.m,
                               P.d16_nsl, P.rowptr, P.d16s_width.as<int32_t>(),
                               P.d16s_units.as<int32_t>(), P.d16s_base.as<int32_t>(),
                               P.d16s_kind.as<int32_t>(), P.d16s_diag.as<int32_t>(),
                               P.d16s_mask.as<uint32_t>(), P.d16s_span.as<int32_t>(), perm, P.d16s_off.as<uint8_t>(),
                               P.d16s_eunits.as<int32_t>(), P.d16s_esc.as<int32_t>(),
                               P.d16s_val.as<V>(), (const A *)x, (A *)y, P.kahan_min);
        else
            hipLaunchKernelGGL((k_sliced_d16<V, uint16_t>), dim3(g), dim3(kBlock), 0, s, P.n, P.m,
                               P.d16_nsl, P.rowptr, P.d16s_width.as<int32_t>(),
                               P.d16s_units.as<int32_t>(), P.d16s_base.as<int32_t>(),
                               P.d16s_kind.as<int32_t>(), P.d16s_diag.as<int32_t>(),
                               P.d16s_mask.as<uint32_t>(), P.d16s_span.as<int32_t>(), perm, P.d16s_off.as<uint16_t>(),
                               nullptr, nullptr, P.d16s_val.as<V>(), (const A *)x, (A *)y,
                               P.kahan_min);
        return hipGetLastError();
    });
}

hipError_t launch_merge_path_raw(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                                 const void *val, int dtype, const void *x, void *y,
                                 const int32_t *srow, const int32_t *snnz, int32_t *crow,
                                 void *cval, int kmin, hipStream_t s, const uint16_t *off,
                                 const int32_t *tbase) {
    if (n == 0) return hipSuccess;
    return by_dtype(dtype, [&](auto tag) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(tag)>>;
        using A = typename VT<V>::A;
        const int64_t tiles = (n + nnz + kMergeTile - 1) / kMergeTile;
        if (tiles <= 0) return hipSuccess;
        if (off)
            hipLaunchKernelGGL((k_merge_path<V, true>), dim3((unsigned)tiles), dim3(kBlock), 0, s, n, rp,
                               ci, (const V *)val, (const A *)x, (A *)y, srow, snnz, crow, (A *)cval,
                               kmin, off, tbase);
        else
            hipLaunchKernelGGL((k_merge_path<V, false>), dim3((unsigned)tiles), dim3(kBlock), 0, s, n, rp,
                               ci, (const V *)val, (const A *)x, (A *)y, srow, snnz, crow, (A *)cval,
                               kmin, (const uint16_t *)nullptr, (const int32_t *)nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const unsigned g = grid_for(tiles, kBlock, INT32_MAX);
        hipLaunchKernelGGL(k_merge_fixup<A>, dim3(g), dim3(kBlock), 0, s, n, tiles, crow,
                           (const A *)cval, (A *)y, kmin);
        return hipGetLastError();
    });
}

hipError_t launch_merge_path(const spmv_plan &P, const void *x, void *y, hipStream_t s) {
    const bool coded = P.code_of(V_MERGE_PATH) == 1;
    return launch_merge_path_raw(P.n, P.nnz, P.rowptr, P.colind, P.val, P.dtype, x, y,
                                 P.mp_split_row.as<int32_t>(), P.mp_split_nnz.as<int32_t>(),
                                 P.mp_carry_row.as<int32_t>(), P.mp_carry_val.p, P.kahan_min, s,
                                 coded ? P.mpc_off.as<uint16_t>() : nullptr,
                                 coded ? P.mpc_base.as<int32_t>() : nullptr);
}

hipError_t launch_xblock(const spmv_plan &P, const void *x, void *y, hipStream_t s) {
    if (P.n == 0) return hipSuccess;
    return by_dtype(P.dtype, [&](auto tag) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(tag)>>;
        using A = typename VT<V>::A;
        SliceTable<A> T;
        T.ns = P.xs_slices;
        const bool coded = P.code_of(V_XBLOCK_LDS) == 1;
        if (coded && !P.xsc_built) return hipErrorInvalidValue;
        T.code = coded ? P.xsc_off.as<uint16_t>() : nullptr;
        const int G = 8 / T.ns;  // XCDs per slice
        int64_t maxt = 0;
        for (int k = 0; k < T.ns; ++k) {
            T.rp[k] = P.xs_rowptr.as<int32_t>() + (size_t)k * (P.n + 1);
            T.srow[k] = P.xs_srow.as<int32_t>() + P.xs_tile_off[k] + k;
            T.snnz[k] = P.xs_snnz.as<int32_t>() + P.xs_tile_off[k] + k;
            T.crow[k] = P.xs_crow.as<int32_t>() + P.xs_tile_off[k];
            T.cval[k] = P.xs_cval.as<A>() + P.xs_tile_off[k];
            T.y[k] = P.xs_y.p ? P.xs_y.as<A>() + (size_t)k * P.n : nullptr;  // none when phased
            T.off[k] = P.xs_nnz_off[k];
            T.tiles[k] = P.xs_tiles[k];
            T.cb[k] = coded ? P.xsc_base.as<int32_t>() + P.xsc_boff[k] : nullptr;
            if (T.tiles[k] > maxt) maxt = T.tiles[k];
        }
        if (P.xs_nlong > 0 && P.xs_rows == 0) return hipErrorInvalidValue;  // split implies streaming
        const LongChunks LC{P.xs_lck0.as<int32_t>(), P.xs_lck1.as<int32_t>(), P.colind, P.val,
                            P.xs_lsum.p, P.xs_lcmap.as<int32_t>()};
        if (P.xs_rows > 0 && P.xs_pj > 0) {  // phased row streaming: no partial y
            const int64_t nblk = (P.n + kBlock - 1) / kBlock;
            const unsigned g = (unsigned)P.xs_pg;
            const int32_t *xci = P.xs_colind.as<int32_t>();
            const V *xv = (const V *)P.xs_val.p;
#define SPMV_PH(JJ)                                                                                    \
    case JJ:                                                                                           \
        if (coded)                                                                                     \
            hipLaunchKernelGGL((k_phased_slices<V, JJ, true>), dim3(g), dim3(kBlock), 0, s, P.n, nblk, \
                               P.rowptr, xci, xv, (const A *)x, T, (A *)y, P.kahan_min);            \
        else                                                                                           \
            hipLaunchKernelGGL((k_phased_slices<V, JJ, false>), dim3(g), dim3(kBlock), 0, s, P.n,     \
                               nblk, P.rowptr, xci, xv, (const A *)x, T, (A *)y, P.kahan_min);      \
        break;
            if (P.xs_nlong > 0) return hipErrorInvalidValue;  // phased only without long rows
            switch (P.xs_pj) {
                SPMV_PH(1) SPMV_PH(2) SPMV_PH(4) SPMV_PH(8)
            default: return hipErrorInvalidValue;
            }
#undef SPMV_PH
            return hipGetLastError();
        }
        if (P.xs_rows > 0) {  // short slice rows: row-block streaming per slice
            const int R = P.xs_rows / kBlock;
            const int64_t nb = (P.n + P.xs_rows - 1) / P.xs_rows;
            const int64_t sg = (nb + G - 1) / G * 8;
            const unsigned g = (unsigned)(sg + P.xs_nslots);
            const int32_t *xci = P.xs_colind.as<int32_t>();
            const V *xv = (const V *)P.xs_val.p;
#define SPMV_RSS(RR)                                                                                   \
    case RR:                                                                                           \
        if (coded)                                                                                     \
            hipLaunchKernelGGL((k_rowstream_slices<V, RR, true>), dim3(g), dim3(kBlock), 0, s, P.n, nb, \
                               xci, xv, (const A *)x, T, sg, LC, P.kahan_min);                      \
        else                                                                                           \
            hipLaunchKernelGGL((k_rowstream_slices<V, RR, false>), dim3(g), dim3(kBlock), 0, s, P.n,   \
                               nb, xci, xv, (const A *)x, T, sg, LC, P.kahan_min);                  \
        break;
            switch (R) {
                SPMV_RSS(1) SPMV_RSS(2) SPMV_RSS(4) SPMV_RSS(8)
            default: return hipErrorInvalidValue;
            }
#undef SPMV_RSS
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        } else if (maxt > 0) {
            if (coded) return hipErrorInvalidValue;  // codes only for row-streamed slices
            hipLaunchKernelGGL(k_merge_slices<V>, dim3((unsigned)((maxt + G - 1) / G * 8)), dim3(kBlock), 0,
                               s, P.n, P.xs_colind.as<int32_t>(), (const V *)P.xs_val.p,
                               (const A *)x, T, P.kahan_min);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            const unsigned g = grid_for(maxt * T.ns, kBlock, INT32_MAX);
            hipLaunchKernelGGL(k_merge_fixup_slices<A>, dim3(g), dim3(kBlock), 0, s, P.n, maxt, T,
                               P.kahan_min);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (P.xs_nlong > 0) {  // rows taken out of the slices (chunks summed above)
            const int64_t gsum = grid_for(P.n, kBlock, (int64_t)P.num_cus * 16);
            const int64_t glong = (P.xs_nlong * 64 + kBlock - 1) / kBlock;
#define SPMV_FIN(NS)                                                                              \
    case NS:                                                                                      \
        hipLaunchKernelGGL((k_slice_finish<A, NS>), dim3((unsigned)(gsum + glong)), dim3(kBlock), 0, \
                           s, P.n, T, (A *)y, gsum, P.xs_lmask.as<uint32_t>(), P.xs_nlong,        \
                           P.xs_lrows.as<int32_t>(), P.xs_lfirst.as<int32_t>(),                    \
                           P.xs_lsum.as<A>(), P.kahan_min);                                        \
        break;
            switch (T.ns) {
                SPMV_FIN(1) SPMV_FIN(2) SPMV_FIN(4) SPMV_FIN(8)
            default: return hipErrorInvalidValue;
            }
#undef SPMV_FIN
            return hipGetLastError();
        }
        const unsigned g = grid_for(P.n, kBlock, (int64_t)P.num_cus * 16);
#define SPMV_SUM(NS)                                                                              \
    case NS:                                                                                      \
        hipLaunchKernelGGL((k_slice_sum<A, NS>), dim3(g), dim3(kBlock), 0, s, P.n, T, (A *)y);      \
        break;
        switch (T.ns) {
            SPMV_SUM(1) SPMV_SUM(2) SPMV_SUM(4) SPMV_SUM(8)
        default: return hipErrorInvalidValue;
        }
#undef SPMV_SUM
        return hipGetLastError();
    });
}

}  // namespace spmvsel
