// Host side of libspmvsel: the C ABI declared in include/spmvsel.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace spmvsel {

// ============================================================ errors
static thread_local std::string g_err;

void clear_error() { g_err.clear(); }

spmv_status_t fail(spmv_status_t st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

spmv_status_t fail_hip(hipError_t e, const char *what, const char *file, int line) {
    (void)hipGetLastError();  // clear the sticky launch error, if any
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    g_err = buf;
    return e == hipErrorOutOfMemory ? SPMV_ERR_OOM : SPMV_ERR_HIP;
}

// ---- device block cache.  Plans are built and destroyed around solver
// loops, and hipMalloc / hipFree of their derived formats (hundreds of MB)
// cost more than the kernels that fill them.  Released blocks are kept per
// device, up to kCacheBytes in all, and handed out again for requests of at
// least half their size.  A release waits for the device as hipFree does, so
// a cached block is never handed out while a kernel may still use it; plans
// wait once for their stream(s) and then release all their buffers without
// further waits.  The cache is invisible to other allocators (PyTorch's), so
// it is kept small; spmv_release_cached_blocks empties it.
namespace {
constexpr size_t kCacheBytes = size_t(2) << 30;
constexpr size_t kCacheMaxBlock = size_t(1) << 30;  // larger blocks go straight back
std::mutex g_cache_mu;
std::multimap<std::pair<int, size_t>, void *> g_cache;  // (device, bytes) -> block
size_t g_cache_total = 0;

size_t round_request(size_t n) {
    if (n < 256) return 256;
    const size_t g = n >= (size_t(1) << 20) ? (size_t(1) << 20) : 256;
    return (n + g - 1) / g * g;
}

void cache_trim(int dev, bool all_devices) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
        if (all_devices || it->first.first == dev) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            if (cur != it->first.first) (void)hipSetDevice(it->first.first);
            (void)hipFree(it->second);
            if (cur != it->first.first) (void)hipSetDevice(cur);
            g_cache_total -= it->first.second;
            it = g_cache.erase(it);
        } else {
            ++it;
        }
    }
}
}  // namespace

spmv_status_t DevBuf::alloc(size_t n) {
    if (p && bytes >= n) return SPMV_OK;
    release();
    const size_t want = round_request(n);
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice", __FILE__, __LINE__);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.lower_bound({d, want});
        if (it != g_cache.end() && it->first.first == d && it->first.second / 2 <= want) {
            p = it->second;
            bytes = it->first.second;
            dev = d;
            g_cache_total -= bytes;
            g_cache.erase(it);
            return SPMV_OK;
        }
    }
    e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {  // give the cached blocks back and try once more
        (void)hipGetLastError();
        cache_trim(d, false);
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
        p = nullptr;
        return fail_hip(e, "hipMalloc", __FILE__, __LINE__);
    }
    bytes = want;
    dev = d;
    return SPMV_OK;
}

// Set while a plan whose streams have been synchronised releases its buffers.
static thread_local bool t_streams_synced = false;

void DevBuf::release() {
    if (!p) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    bool kept = false;
    if (t_streams_synced || hipDeviceSynchronize() == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (bytes <= kCacheMaxBlock && g_cache_total + bytes <= kCacheBytes) {
            g_cache.emplace(std::make_pair(dev, bytes), p);
            g_cache_total += bytes;
            kept = true;
        }
    }
    if (!kept) (void)hipFree(p);
    if (cur != dev) (void)hipSetDevice(cur);
    p = nullptr;
    bytes = 0;
}

// ============================================================ process state
namespace {

std::mutex g_mu;
double g_theta[4] = {2.0, 1.2, 1.5, 4.0};

struct Model {
    bool loaded = false;
    std::vector<float> params;  // 5382
    float norm[24];             // mu[12], rho[12]
    float tau = 0.f;
    std::map<int, DevBuf *> dev;  // per-device copy: params then norm
};
Model g_model;

std::map<int, DevBuf *> g_flush;  // 512 MiB eviction buffer per device

// Recycled per-plan buffers: pinned 4 KiB host staging and device scratch,
// so that creating and destroying plans in a loop allocates nothing after
// the first plan on each device.
std::vector<void *> g_pinned_pool;
std::map<int, std::vector<void *>> g_scratch_pool;
constexpr size_t kFlushBytes = 512ull << 20;
constexpr size_t kFlushSink = 256;  // the flush kernel's sink words, after its buffer
constexpr int kNParams = 12 * 64 + 64 + 64 * 64 + 64 + 64 * 6 + 6;

typedef unsigned __int128 u128;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Round an unsigned 128-bit integer to the nearest double (ties to even):
// keep the top 64 bits with every dropped bit folded into a sticky bit, then
// one 64-bit -> double conversion and an exact scaling.
double u128_to_double(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    if (hi == 0) return (double)lo;
    const int sh = 64 - __builtin_clzll(hi);
    const uint64_t top = (uint64_t)(v >> sh);
    const uint64_t sticky = (v & (((u128)1 << sh) - 1)) != 0 ? 1 : 0;
    return ldexp((double)(top | sticky), sh);
}

uint32_t crc32(const unsigned char *p, size_t n) {
    static uint32_t table[256];
    static bool init = false;
    if (!init) {
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
            table[i] = c;
        }
        init = true;
    }
    uint32_t c = 0xFFFFFFFFu;
    for (size_t i = 0; i < n; ++i) c = table[(c ^ p[i]) & 0xFF] ^ (c >> 8);
    return c ^ 0xFFFFFFFFu;
}

int pow2_ceil(double v, int lo, int hi) {
    int w = lo;
    while (w < hi && w < v) w <<= 1;
    return w;
}

int pow2_floor(double v, int lo, int hi) {
    int w = lo;
    while (w * 2 <= hi && w * 2 <= v) w <<= 1;
    return w;
}

hipStream_t S(const spmv_plan *P) { return P->stream; }

spmv_status_t sync(const spmv_plan *P) {
    SPMV_HIP(hipStreamSynchronize(P->stream));
    return SPMV_OK;
}

// scratch layout (bytes)
constexpr size_t kOffFlags = 0;                       // 3 u64
constexpr size_t kOffRec = 256;                       // 16 u64
constexpr size_t kOffSum = 512;                       // 9 u64: a maximum, slice totals
constexpr size_t kOffLong = 640;                      // 1 i64: long-row count
constexpr size_t kOffClf = 768;                       // 80 bytes: classifier output
constexpr size_t kOffMlp = 1024;                      // kSelectRecordBytes
constexpr size_t kOffPart = 4096;                     // kFeatBlocks * 16 u64
constexpr size_t kScratchBytes = kOffPart + kFeatBlocks * 16 * 8;

template <class T> T *scr(const spmv_plan *P, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(P->scratch.p) + off);
}

// ------------------------------------------------------------ features
void finalize_features(const spmv_plan *P, const uint64_t *w, double *f) {
    for (int i = 0; i < 12; ++i) f[i] = 0.0;
    const int64_t n = P->n, nnz = P->nnz;
    if (n == 0) return;
    const double f0 = (double)n, f1 = (double)nnz, nn = f0 * f0;
    const u128 sl2 = w[3], sbw = w[4], sbw2 = ((u128)w[6] << 64) | w[5];
    const u128 sq = w[7], sq2 = ((u128)w[9] << 64) | w[8];
    const int64_t smiss = (int64_t)(w[10] - w[11]);
    f[0] = f0;
    f[1] = f1;
    f[2] = f1 / f0;
    f[3] = sqrt(u128_to_double((u128)n * sl2 - (u128)nnz * (u128)nnz) / nn);
    f[4] = (double)w[1];
    f[5] = (double)w[0];
    f[6] = (double)(uint64_t)sbw / f0;
    f[7] = sqrt(u128_to_double((u128)n * sbw2 - sbw * sbw) / nn);
    f[8] = ((double)(uint64_t)sq / 2147483648.0) / f0;
    f[9] = sqrt(u128_to_double((u128)n * sq2 - sq * sq) / 4611686018427387904.0 / nn);
    f[10] = nnz > 0 ? (double)smiss / f1 : 0.0;
    const int64_t ws = 4 * (n + 1) + (4 + vbytes(P->dtype)) * nnz + xbytes(P->dtype) * P->m +
                       xbytes(P->dtype) * n;
    f[11] = ws <= kLlcBytes ? 1.0 : 0.0;
}

spmv_status_t ensure_features(spmv_plan *P) {
    if (P->have_features) return SPMV_OK;
    uint64_t *rec = scr<uint64_t>(P, kOffRec);
    SPMV_HIP(launch_features(*P, scr<uint64_t>(P, kOffPart), rec, xbytes(P->dtype), S(P)));
    uint64_t *h = static_cast<uint64_t *>(P->h_pinned);
    SPMV_HIP(hipMemcpyAsync(h, rec, 16 * 8, hipMemcpyDeviceToHost, S(P)));
    SPMV_TRY(sync(P));
    uint64_t w[16];
    memcpy(w, h, sizeof w);
    if (P->n == 0) w[0] = 0;
    finalize_features(P, w, P->feats);
    const int64_t smiss = (int64_t)(w[10] - w[11]);
    const uint64_t a[12] = {w[0], w[1], w[2], w[3], w[4], w[5],
                            w[6], w[7], w[8], w[9], (uint64_t)smiss, (uint64_t)P->nnz};
    memcpy(P->acc, a, sizeof a);
    P->have_features = true;
    return SPMV_OK;
}

// delta16 feasibility: every block of d16_rows rows spans at most 65536
// columns.  The block bases are the panel minima; tried first with the
// short_row block height, then with 256-row blocks.
spmv_status_t check_d16(spmv_plan *P) {
    if (P->d16_checked) return SPMV_OK;
    int heights[2] = {P->rs_rows * kBlock, kBlock};
    for (int t = 0; t < 2; ++t) {
        const int H = heights[t];
        if (t == 1 && H == heights[0]) break;
        const int64_t blocks = (P->n + H - 1) / H;
        SPMV_TRY(P->d16_base.alloc((size_t)(blocks > 0 ? blocks : 1) * 4));
        SPMV_TRY(P->d16_cmax.alloc((size_t)(blocks > 0 ? blocks : 1) * 4));
        unsigned long long span = 0;
        if (blocks > 0) {
            SPMV_HIP(launch_panel_windows(*P, H, P->d16_base.as<int32_t>(), P->d16_cmax.as<int32_t>(),
                                          blocks, S(P)));
            auto *d = scr<unsigned long long>(P, kOffSum);
            SPMV_HIP(launch_max_span(P->d16_base.as<int32_t>(), P->d16_cmax.as<int32_t>(), blocks,
                                     d, S(P)));
            SPMV_HIP(hipMemcpyAsync(P->h_pinned, d, 8, hipMemcpyDeviceToHost, S(P)));
            SPMV_TRY(sync(P));
            memcpy(&span, P->h_pinned, 8);
        }
        P->d16_rows = H;
        P->d16_feasible = span <= 65535;
        if (P->d16_feasible) break;
    }
    P->d16_cmax.release();
    P->d16_checked = true;
    P->d16_base_ready = true;
    return SPMV_OK;
}

bool d16_feasible(const spmv_plan *P) { return P->d16_feasible; }

// The block reference columns the delta16 encoder reads: one int32 per block
// of d16_rows rows (the smallest column of the block), computed here when the
// feasibility test took only the spans.
spmv_status_t ensure_d16_base(spmv_plan *P) {
    const int64_t blocks = (P->n + P->d16_rows - 1) / P->d16_rows;
    if (!P->d16_base_ready) {
        SPMV_TRY(P->d16_base.alloc((size_t)(blocks > 0 ? blocks : 1) * 4));
        if (blocks > 0) {
            SPMV_TRY(P->d16_cmax.alloc((size_t)blocks * 4));
            SPMV_HIP(launch_panel_windows(*P, P->d16_rows, P->d16_base.as<int32_t>(),
                                          P->d16_cmax.as<int32_t>(), blocks, S(P)));
            SPMV_TRY(sync(P));
            P->d16_cmax.release();
        }
        P->d16_base_ready = true;
    }
    if (blocks > 0 && (!P->d16_base.p || P->d16_base.bytes < (size_t)blocks * 4))
        return fail(SPMV_ERR_HIP, "delta16: block references missing (%lld blocks of %d rows)",
                    (long long)blocks, P->d16_rows);
    return SPMV_OK;
}

// delta16 layout: the shape of the sliced layout (widths, reference columns,
// slot offsets) decides it; sliced when its slots, padding included, are at
// most kSellMaxPad per nonzero, or kSellMaxPadLong when rows average at least
// 7.5 nonzeros and its offset slices span fewer than kSellMaxSpanLong columns
// (on bands padded to 1.5 slots per nonzero the sliced kernel ran about 10%
// faster than the streamed one with 8 to 16 nonzeros per row, slower with 6,
// and slower across 40000 columns), or when forced.  A
// 64-row slice lies inside one block of the streamed layout, so it is
// feasible whenever that is.
spmv_status_t d16_decide_layout(spmv_plan *P) {
    if (P->d16_layout >= 0) return SPMV_OK;
    SPMV_TRY(check_d16(P));
    if (!d16_feasible(P))
        return fail(SPMV_ERR_INFEASIBLE,
                    "delta16: a block of %d rows spans more than 65536 columns", P->d16_rows);
    if (P->nnz >= (1ll << 30)) {  // beyond the sliced layout's int32 slot arithmetic
        if (P->d16_layout_req == 1)
            return fail(SPMV_ERR_INFEASIBLE, "delta16: the sliced layout needs NNZ < 2^30");
        P->d16_layout = 0;
        return SPMV_OK;
    }
    const int64_t nsl = (P->n + kSellRows - 1) / kSellRows;
    const size_t nb = (size_t)(nsl > 0 ? nsl : 1) * 4;
    SPMV_TRY(P->d16s_width.alloc(nb));
    SPMV_TRY(P->d16s_units.alloc(nb + 4));  // the scan also writes the total after the last slice
    SPMV_TRY(P->d16s_base.alloc(nb));
    SPMV_TRY(P->d16s_kind.alloc(nb));
    SPMV_TRY(P->d16s_diag.alloc(nb * kSellMaxDiag));
    SPMV_TRY(P->d16s_nnz.alloc(nb));
    DevBuf halfw, tmp;
    DevBuf &span = P->d16s_span;
    SPMV_TRY(halfw.alloc(nb));
    SPMV_TRY(span.alloc(nb));
    int64_t units = 0, nnz_off = 0, ndiag = 0, max_span = 0, staged_nnz = 0;
    // the slices' shape (widths, references, kinds, spans) and unit offsets,
    // of the plain layout or, with perm, of the length-sorted one
    auto shape = [&](const int32_t *perm) -> spmv_status_t {
        units = nnz_off = ndiag = max_span = staged_nnz = 0;
        if (nsl == 0) return SPMV_OK;
        SPMV_HIP(launch_sliced_shape(*P, perm, P->d16s_width.as<int32_t>(), halfw.as<int32_t>(),
                                     P->d16s_base.as<int32_t>(), P->d16s_kind.as<int32_t>(),
                                     P->d16s_diag.as<int32_t>(), P->d16s_nnz.as<int32_t>(),
                                     span.as<int32_t>(), S(P)));
        size_t need = 0;
        int64_t *dtot = scr<int64_t>(P, kOffSum);
        SPMV_HIP(launch_exclusive_scan_i32(halfw.as<int32_t>(), P->d16s_units.as<int32_t>(), nsl, 1,
                                           dtot, nullptr, 0, S(P), &need));
        SPMV_TRY(tmp.alloc(need));
        SPMV_HIP(launch_exclusive_scan_i32(halfw.as<int32_t>(), P->d16s_units.as<int32_t>(), nsl, 1,
                                           dtot, tmp.p, tmp.bytes, S(P), nullptr));
        SPMV_HIP(hipMemcpyAsync(P->h_pinned, dtot, 8, hipMemcpyDeviceToHost, S(P)));
        std::vector<int32_t> kinds((size_t)nsl), counts((size_t)nsl), spans((size_t)nsl),
            widths((size_t)nsl);
        SPMV_HIP(hipMemcpyAsync(kinds.data(), P->d16s_kind.p, nb, hipMemcpyDeviceToHost, S(P)));
        SPMV_HIP(hipMemcpyAsync(widths.data(), P->d16s_width.p, nb, hipMemcpyDeviceToHost, S(P)));
        SPMV_HIP(hipMemcpyAsync(counts.data(), P->d16s_nnz.p, nb, hipMemcpyDeviceToHost, S(P)));
        SPMV_HIP(hipMemcpyAsync(spans.data(), span.p, nb, hipMemcpyDeviceToHost, S(P)));
        SPMV_TRY(sync(P));
        memcpy(&units, P->h_pinned, 8);
        for (int64_t k = 0; k < nsl; ++k) {
            if (kinds[k] > 0) {
                ++ndiag;
            } else {
                nnz_off += counts[k];
                if (spans[k] > max_span) max_span = spans[k];
                if (sell_stages_x(spans[k], widths[k])) staged_nnz += counts[k];
            }
        }
        return SPMV_OK;
    };
    SPMV_TRY(shape(nullptr));
    // Length-sorted rows (rows sorted by length inside each 256-row window,
    // as in SELL-C-sigma): taken when requested, or automatically when the
    // plain layout has at most 1% diagonal slices and over 5% of padding,
    // sorting saves at least 5% of its slots, and either the plain layout
    // stages x for under half of its offset nonzeros and sorting saves
    // kSortMinSavedFree slots per row, or sorting keeps at least half of the
    // staging and saves kSortMinSaved slots per row.  The sorted kernel
    // reads a 4-byte row index per row and scatters its y stores over the
    // window, and a sorted slice spans its window's columns, up to 192 more
    // than a plain one, so that it may no longer stage x in LDS: with the
    // staging kept, sorting paid from about 8 saved slots per row; where
    // neither stages, from about 3.  A window lies inside one block of the
    // streamed layout, so its slices stay within 16 bits.
    P->d16_sort = 0;
    P->d16s_perm.release();
    P->d16s_pinv.release();
    const int64_t plain_slots = units * 2 * kSellRows;
    const int64_t staged_plain = staged_nnz, nnz_off_plain = nnz_off;
    const bool consider =
        P->d16_layout_req != 0 &&
        (P->d16_sort_req == 1 ||
         (P->d16_sort_req < 0 && ndiag * 100 <= nsl && plain_slots * 100 > 105 * P->nnz));
    if (consider && P->n > 0) {
        SPMV_TRY(P->d16s_perm.alloc((size_t)P->n * 4));
        SPMV_TRY(P->d16s_pinv.alloc((size_t)P->n * 4));
        SPMV_HIP(launch_sell_perm(*P, P->d16s_perm.as<int32_t>(), P->d16s_pinv.as<int32_t>(), S(P)));
        SPMV_TRY(shape(P->d16s_perm.as<int32_t>()));
        const int64_t saved = plain_slots - units * 2 * kSellRows;
        const bool free_x = 2 * staged_plain < nnz_off_plain;
        if (P->d16_sort_req == 1 ||
            (saved * 20 >= plain_slots &&
             ((free_x && saved >= (int64_t)kSortMinSavedFree * P->n) ||
              (2 * staged_nnz >= staged_plain && saved >= (int64_t)kSortMinSaved * P->n)))) {
            P->d16_sort = 1;
        } else {
            P->d16s_perm.release();
            P->d16s_pinv.release();
            SPMV_TRY(shape(nullptr));
        }
    }
    P->d16_nnz_off = nnz_off;
    P->d16_ndiag = ndiag;
    P->d16_span = max_span;
    P->d16_nsl = nsl;
    P->d16_slots = units * 2 * kSellRows;
    // the unit offsets are int32 (with NNZ < 2^30 every width is too)
    const bool representable = units <= INT32_MAX;
    const double slots = (double)P->d16_slots, nnz = (double)P->nnz;
    const bool padded_ok = slots <= kSellMaxPad * nnz ||
                           (2 * P->nnz >= (int64_t)kSellLongMeanX2 * P->n &&
                            slots <= kSellMaxPadLong * nnz && max_span < kSellMaxSpanLong);
    const int automatic = representable && padded_ok ? 1 : 0;
    if (P->d16_layout_req == 1 && !representable)
        return fail(SPMV_ERR_INFEASIBLE, "delta16: the sliced layout needs under 2^31 slot pairs");
    const int layout = P->d16_layout_req >= 0 ? P->d16_layout_req : automatic;
    // one code width for the whole matrix.  8-bit delta codes escape a gap of
    // 255 or more; a slice spanning fewer columns has none.  Otherwise the
    // escapes are counted, and 8 bits are taken when their area (64 int32
    // entries per unit of the per-slice maximum) costs at most half of the
    // byte per nonzero that the codes save
    int64_t esc_units = 0, nesc = 0;
    std::vector<int32_t> eunits;
    int offw = 16;
    if (layout == 1 && P->d16_offw_req != 16 && (nnz_off > 0 || P->d16_offw_req == 8)) {
        eunits.assign(nb / 4 + 1, 0);  // S + 1 entries (nb covers at least one slice)
        if (max_span >= 255) {
            DevBuf dE, dN;
            SPMV_TRY(dE.alloc(nb));
            SPMV_TRY(dN.alloc(nb));
            SPMV_HIP(launch_sliced_escapes(*P, P->d16s_base.as<int32_t>(), P->d16s_kind.as<int32_t>(),
                                           dE.as<int32_t>(), dN.as<int32_t>(), S(P)));
            std::vector<int32_t> hE((size_t)nsl), hN((size_t)nsl);
            SPMV_HIP(hipMemcpyAsync(hE.data(), dE.p, nb, hipMemcpyDeviceToHost, S(P)));
            SPMV_HIP(hipMemcpyAsync(hN.data(), dN.p, nb, hipMemcpyDeviceToHost, S(P)));
            SPMV_TRY(sync(P));
            for (int64_t k = 0; k < nsl; ++k) {
                eunits[(size_t)k] = (int32_t)esc_units;  // at most one unit per slot pair
                esc_units += hE[(size_t)k];
                nesc += hN[(size_t)k];
            }
            eunits[(size_t)nsl] = (int32_t)esc_units;
        }
        const bool want8 = P->d16_offw_req == 8 || 512 * esc_units <= nnz_off;
        if (want8) offw = 8;
    }
    if (offw == 8) {
        SPMV_TRY(P->d16s_eunits.alloc(nb + 4));
        SPMV_HIP(hipMemcpyAsync(P->d16s_eunits.p, eunits.data(), nb + 4, hipMemcpyHostToDevice,
                                S(P)));
        SPMV_TRY(sync(P));  // the host vector goes out of scope
    } else {
        P->d16s_eunits.release();
        esc_units = nesc = 0;
    }
    P->d16_layout = layout;
    P->d16_offw = offw;
    P->d16_esc_units = esc_units;
    P->d16_nesc = nesc;
    P->d16s_nnz.release();
    if (P->d16_layout == 0) {
        P->d16s_width.release();
        P->d16s_units.release();
        P->d16s_base.release();
        P->d16s_kind.release();
        P->d16s_diag.release();
        P->d16s_span.release();
        P->d16s_perm.release();
        P->d16s_pinv.release();
        P->d16_sort = 0;
    }
    return SPMV_OK;
}

// ------------------------------------------------------------ formats
// x blocking: split the columns into S slices (S <= 8, one XCD group each)
// and store each slice as its own CSR (rowptr per slice, slice-major
// colind/val), with merge-path tiles per slice when a slice row is long, and
// one partial y per slice.
// Slice count: the requested one, else the smallest of 1, 2, 4, 8 (at most
// one slice per XCD) that leaves at most kSliceXEntries columns per slice,
// doubled only while a slice row keeps 0.9 nonzeros on average: with fewer,
// the per-slice row pointers and partial y vectors cost more than the
// smaller windows gain (a sweep of random-row and power-law matrices of 250k
// to 4M rows and 2 to 32 nonzeros per row put the best count there; at 2
// per slice row the count stopped one doubling short on 4M rows, 8-18%
// slower).
int xs_slice_count(const spmv_plan *P) {
    if (P->xs_req > 0) return P->xs_req;
    int ns = 1;
    while (ns < kSlices && P->m > kSliceXEntries * ns &&
           10 * P->nnz >= (int64_t)kSliceMinAvg10 * 2 * ns * P->n)
        ns *= 2;
    return ns;
}

int64_t xs_slice_width(const spmv_plan *P, int ns) {
    return P->m > 0 ? (P->m + ns - 1) / ns : 1;
}

// Rows whose longest slice segment exceeds kSliceStreamMaxLen leave the
// slices (their segments are zeroed in lens) when they hold at most
// kLongMaxShare of the nonzeros; they are then summed from the original CSR
// in chunks of kLongChunk.  Otherwise nothing changes and the slices use
// merge-path tiles.
spmv_status_t split_long_rows(spmv_plan *P, int ns, int32_t *lens) {
    const int64_t n = P->n;
    P->xs_nlong = P->xs_nchunks = P->xs_long_nnz = P->xs_nslots = 0;
    DevBuf flags, pos, tmp, rows, beg, end;
    SPMV_TRY(flags.alloc((size_t)n * 4));
    SPMV_TRY(pos.alloc((size_t)(n + 1) * 4));
    SPMV_HIP(launch_long_flags(n, ns, lens, flags.as<int32_t>(), S(P)));
    size_t need = 0;
    int64_t *dtot = scr<int64_t>(P, kOffLong);
    SPMV_HIP(launch_exclusive_scan_i32(flags.as<int32_t>(), pos.as<int32_t>(), n, 1, dtot, nullptr, 0,
                                       S(P), &need));
    SPMV_TRY(tmp.alloc(need));
    SPMV_HIP(launch_exclusive_scan_i32(flags.as<int32_t>(), pos.as<int32_t>(), n, 1, dtot, tmp.p,
                                       tmp.bytes, S(P), nullptr));
    int64_t *h = static_cast<int64_t *>(P->h_pinned);
    SPMV_HIP(hipMemcpyAsync(h, dtot, 8, hipMemcpyDeviceToHost, S(P)));
    SPMV_TRY(sync(P));
    const int64_t L = h[0];
    if (L == 0) return SPMV_OK;
    SPMV_TRY(rows.alloc((size_t)L * 4));
    SPMV_TRY(beg.alloc((size_t)L * 4));
    SPMV_TRY(end.alloc((size_t)L * 4));
    SPMV_HIP(launch_long_compact(n, flags.as<int32_t>(), pos.as<int32_t>(), P->rowptr,
                                 rows.as<int32_t>(), beg.as<int32_t>(), end.as<int32_t>(), S(P)));
    std::vector<int32_t> hb(L), he(L);
    SPMV_HIP(hipMemcpyAsync(hb.data(), beg.p, (size_t)L * 4, hipMemcpyDeviceToHost, S(P)));
    SPMV_HIP(hipMemcpyAsync(he.data(), end.p, (size_t)L * 4, hipMemcpyDeviceToHost, S(P)));
    SPMV_TRY(sync(P));
    int64_t long_nnz = 0;
    for (int64_t t = 0; t < L; ++t) long_nnz += he[t] - hb[t];
    if ((double)long_nnz > kLongMaxShare * (double)P->nnz) return SPMV_OK;
    // chunks of at most kLongChunk nonzeros, each inside one column slice,
    // in row and column order (the order the finish adds their sums in)
    DevBuf dbnd;
    SPMV_TRY(dbnd.alloc((size_t)L * (ns + 1) * 4));
    SPMV_HIP(launch_long_bounds(L, ns, P->xs_width, P->colind, beg.as<int32_t>(), end.as<int32_t>(),
                                dbnd.as<int32_t>(), S(P)));
    std::vector<int32_t> bnd((size_t)L * (ns + 1));
    SPMV_HIP(hipMemcpyAsync(bnd.data(), dbnd.p, bnd.size() * 4, hipMemcpyDeviceToHost, S(P)));
    SPMV_TRY(sync(P));
    std::vector<int32_t> first(L + 1), ck0, ck1;
    std::vector<std::vector<int32_t>> queue((size_t)ns);
    for (int64_t t = 0; t < L; ++t) {
        first[t] = (int32_t)ck0.size();
        for (int sl = 0; sl < ns; ++sl) {
            const int64_t b0 = bnd[(size_t)t * (ns + 1) + sl], b1 = bnd[(size_t)t * (ns + 1) + sl + 1];
            for (int64_t k = b0; k < b1; k += kLongChunk) {
                queue[(size_t)sl].push_back((int32_t)ck0.size());
                ck0.push_back((int32_t)k);
                ck1.push_back((int32_t)std::min<int64_t>(b1, k + kLongChunk));
            }
        }
    }
    first[L] = (int32_t)ck0.size();
    const int64_t nc = (int64_t)ck0.size();
    // chunk workgroup c of the slice kernel (its grid's slice part is a
    // multiple of 8 workgroups) runs on XCD c mod 8, whose L2 holds slice
    // (c mod 8) mod S: it takes the next chunk of that slice, or none
    std::vector<int32_t> cmap;
    std::vector<size_t> head((size_t)ns, 0);
    for (int64_t c = 0, left = nc; left > 0; ++c) {
        const size_t sl = (size_t)((c % 8) % ns);
        if (head[sl] < queue[sl].size()) {
            cmap.push_back(queue[sl][head[sl]++]);
            --left;
        } else {
            cmap.push_back(-1);
        }
    }
    SPMV_TRY(P->xs_lrows.alloc((size_t)L * 4));
    SPMV_TRY(P->xs_lfirst.alloc((size_t)(L + 1) * 4));
    SPMV_TRY(P->xs_lck0.alloc((size_t)nc * 4));
    SPMV_TRY(P->xs_lck1.alloc((size_t)nc * 4));
    SPMV_TRY(P->xs_lsum.alloc((size_t)nc * 8));
    SPMV_TRY(P->xs_lcmap.alloc(cmap.size() * 4));
    SPMV_TRY(P->xs_lmask.alloc((size_t)((n + 31) / 32) * 4));
    SPMV_HIP(launch_long_mask(n, flags.as<int32_t>(), P->xs_lmask.as<uint32_t>(), S(P)));
    SPMV_HIP(hipMemcpyAsync(P->xs_lrows.p, rows.p, (size_t)L * 4, hipMemcpyDeviceToDevice, S(P)));
    SPMV_HIP(hipMemcpyAsync(P->xs_lfirst.p, first.data(), (size_t)(L + 1) * 4, hipMemcpyHostToDevice, S(P)));
    SPMV_HIP(hipMemcpyAsync(P->xs_lck0.p, ck0.data(), (size_t)nc * 4, hipMemcpyHostToDevice, S(P)));
    SPMV_HIP(hipMemcpyAsync(P->xs_lck1.p, ck1.data(), (size_t)nc * 4, hipMemcpyHostToDevice, S(P)));
    SPMV_HIP(hipMemcpyAsync(P->xs_lcmap.p, cmap.data(), cmap.size() * 4, hipMemcpyHostToDevice, S(P)));
    SPMV_HIP(launch_long_zero(L, ns, n, rows.as<int32_t>(), lens, S(P)));
    SPMV_TRY(sync(P));  // the host vectors above must outlive the copies
    P->xs_nlong = L;
    P->xs_nchunks = nc;
    P->xs_nslots = (int64_t)cmap.size();
    P->xs_long_nnz = long_nnz;
    return SPMV_OK;
}

spmv_status_t build_xslices(spmv_plan *P) {
    if (P->xs_built) return SPMV_OK;
    P->xsc_checked = P->xsc_feasible = P->xsc_built = false;
    const int64_t n = P->n, nnz = P->nnz;
    const int ns = xs_slice_count(P);
    const int64_t cw = xs_slice_width(P, ns);
    P->xs_slices = ns;
    P->xs_width = cw;
    P->xs_nlong = P->xs_nchunks = P->xs_long_nnz = P->xs_nslots = 0;
    P->xs_pj = 0;
    P->xs_pg = 0;
    for (int k = 0; k < kSlices; ++k) P->xs_nnz_off[k] = P->xs_tiles[k] = P->xs_tile_off[k] = 0;
    SPMV_TRY(P->xs_rowptr.alloc((size_t)ns * (n + 1) * 4));
    // slice starts are padded to 8 elements so every slice keeps the
    // 16-byte alignment the vector loads rely on
    SPMV_TRY(P->xs_colind.alloc((size_t)(nnz + 8 * ns) * 4 + 16));
    SPMV_TRY(P->xs_val.alloc((size_t)(nnz + 8 * ns) * vbytes(P->dtype) + 16));
    int64_t snnz[kSlices] = {0};
    // merge-path tiles of the original CSR, walked by the count and scatter kernels
    const int64_t mtiles = (n + nnz + kMergeTile - 1) / kMergeTile;
    DevBuf msr, msn;
    SPMV_TRY(msr.alloc((size_t)(mtiles + 1) * 4));
    SPMV_TRY(msn.alloc((size_t)(mtiles + 1) * 4));
    if (n > 0) {
        SPMV_HIP(launch_merge_splits(P->rowptr, n, nnz, msr.as<int32_t>(), msn.as<int32_t>(), mtiles,
                                     S(P)));
        DevBuf lens, tmp;
        SPMV_TRY(lens.alloc((size_t)ns * n * 4));
        SPMV_HIP(launch_slice_count(*P, cw, msr.as<int32_t>(), msn.as<int32_t>(), mtiles,
                                    lens.as<int32_t>(), S(P)));
        SPMV_TRY(split_long_rows(P, ns, lens.as<int32_t>()));
        size_t need = 0;
        auto *dmax = scr<unsigned long long>(P, kOffSum);  // then the slice totals
        int64_t *dtot = reinterpret_cast<int64_t *>(dmax + 1);
        SPMV_HIP(launch_exclusive_scan_i32(lens.as<int32_t>(), P->xs_rowptr.as<int32_t>(), n,
                                           ns, dtot, nullptr, 0, S(P), &need));
        SPMV_TRY(tmp.alloc(need));
        SPMV_HIP(launch_exclusive_scan_i32(lens.as<int32_t>(), P->xs_rowptr.as<int32_t>(), n,
                                           ns, dtot, tmp.p, tmp.bytes, S(P), nullptr));
        SPMV_HIP(launch_max_i32(lens.as<int32_t>(), (int64_t)ns * n, scr<int32_t>(P, kOffPart),
                                dmax, S(P)));
        int64_t *h = static_cast<int64_t *>(P->h_pinned);
        SPMV_HIP(hipMemcpyAsync(h, dmax, 8 * (1 + ns), hipMemcpyDeviceToHost, S(P)));
        SPMV_TRY(sync(P));
        unsigned long long maxlen = 0;
        memcpy(&maxlen, h, 8);
        for (int k = 0; k < ns; ++k) snnz[k] = h[1 + k];
        // slice rows no longer than a chunk: row-block streaming, else merge path
        if (maxlen <= (unsigned long long)kChunk / 4) {
            const double avg = (double)(nnz - P->xs_long_nnz) / ((double)n * ns);
            P->xs_rows = kBlock * pow2_floor((double)kChunk / (kBlock * (avg > 1e-9 ? avg : 1e-9)),
                                             1, kRowStreamMaxR);
            if (P->xs_nlong == 0) SPMV_HIP(phased_geometry(*P, &P->xs_pj, &P->xs_pg));
        } else {
            P->xs_rows = 0;
        }
    }
    // partial y vectors only for the slice kernels that write them
    if (P->xs_pj == 0) SPMV_TRY(P->xs_y.alloc((size_t)ns * (n > 0 ? n : 1) * xbytes(P->dtype)));
    else P->xs_y.release();
    SliceOffsets so;
    int64_t off = 0, toff = 0;
    int64_t total = 0;
    for (int k = 0; k < kSlices; ++k) so.off[k] = 0;
    for (int k = 0; k < ns; ++k) {
        so.off[k] = off;
        P->xs_nnz_off[k] = off;
        off = (off + snnz[k] + 7) & ~(int64_t)7;
        total += snnz[k];
        P->xs_tiles[k] = n > 0 ? (n + snnz[k] + kMergeTile - 1) / kMergeTile : 0;
        P->xs_tile_off[k] = toff;
        toff += P->xs_tiles[k];
    }
    if (total + P->xs_long_nnz != nnz)
        return fail(SPMV_ERR_HIP, "x-block slices hold %lld of %lld nonzeros (%lld in long rows)",
                    (long long)total, (long long)nnz, (long long)P->xs_long_nnz);
    SPMV_TRY(P->xs_srow.alloc((size_t)(toff + ns) * 4));
    SPMV_TRY(P->xs_snnz.alloc((size_t)(toff + ns) * 4));
    SPMV_TRY(P->xs_crow.alloc((size_t)(toff > 0 ? toff : 1) * 4));
    SPMV_TRY(P->xs_cval.alloc((size_t)(toff > 0 ? toff : 1) * 8));
    if (n > 0) {
        SPMV_HIP(launch_slice_scatter(*P, msr.as<int32_t>(), msn.as<int32_t>(), mtiles,
                                      P->xs_rowptr.as<int32_t>(), so, P->xs_colind.as<int32_t>(),
                                      P->xs_val.p, S(P)));
        for (int k = 0; k < ns && P->xs_rows == 0; ++k)
            SPMV_HIP(launch_merge_splits(P->xs_rowptr.as<int32_t>() + (size_t)k * (n + 1), n, snnz[k],
                                         P->xs_srow.as<int32_t>() + P->xs_tile_off[k] + k,
                                         P->xs_snnz.as<int32_t>() + P->xs_tile_off[k] + k,
                                         P->xs_tiles[k], S(P)));
        SPMV_TRY(sync(P));
    }
    P->xs_built = true;
    return SPMV_OK;
}

// 16-bit codes of the merge-path tiles (splits built): reference = the
// tile's smallest column; feasible when every tile spans < 65536 columns.
spmv_status_t check_merge_codes(spmv_plan *P) {
    if (P->mpc_checked) return SPMV_OK;
    const int64_t tiles = P->mp_tiles;
    SPMV_TRY(P->mpc_base.alloc((size_t)(tiles > 0 ? tiles : 1) * 4));
    DevBuf span;
    SPMV_TRY(span.alloc((size_t)(tiles > 0 ? tiles : 1) * 4));
    int32_t mx = 0;
    if (tiles > 0 && P->nnz > 0) {
        SPMV_HIP(launch_range_ref(tiles, tiles, 1, P->mp_split_nnz.as<int32_t>(), P->colind,
                                  P->mpc_base.as<int32_t>(), span.as<int32_t>(), S(P)));
        auto *d = scr<unsigned long long>(P, kOffSum);
        SPMV_HIP(launch_max_i32(span.as<int32_t>(), tiles, scr<int32_t>(P, kOffPart), d, S(P)));
        SPMV_HIP(hipMemcpyAsync(P->h_pinned, d, 8, hipMemcpyDeviceToHost, S(P)));
        SPMV_TRY(sync(P));
        unsigned long long m = 0;
        memcpy(&m, P->h_pinned, 8);
        mx = (int32_t)m;
    }
    P->mpc_span = mx;
    P->mpc_feasible = mx <= 65535;
    P->mpc_checked = true;
    return SPMV_OK;
}

// 16-bit codes of the x-block slices (slices built, row-streamed): per slice
// and row block of xsc_h rows (256 for the phased walk, else the per-slice
// kernel's block height) the smallest column; feasible when every block's
// segment of every slice spans < 65536 columns.
spmv_status_t check_xblock_codes(spmv_plan *P) {
    if (P->xsc_checked) return SPMV_OK;
    P->xsc_checked = true;
    P->xsc_feasible = false;
    P->xsc_span = 0;
    if (P->xs_rows == 0) return SPMV_OK;  // merge-path slices: no coded form
    const int64_t n = P->n, H = P->xs_pj > 0 ? kBlock : P->xs_rows;
    const int64_t nb = (n + H - 1) / H;
    const int ns = P->xs_slices;
    P->xsc_h = H;
    for (int k = 0; k <= ns; ++k) P->xsc_boff[k] = (int64_t)k * nb;
    SPMV_TRY(P->xsc_base.alloc((size_t)(ns * nb > 0 ? ns * nb : 1) * 4));
    DevBuf span;
    SPMV_TRY(span.alloc((size_t)(ns * nb > 0 ? ns * nb : 1) * 4));
    int32_t mx = 0;
    if (nb > 0) {
        for (int k = 0; k < ns; ++k)
            SPMV_HIP(launch_range_ref(nb, n, H, P->xs_rowptr.as<int32_t>() + (size_t)k * (n + 1),
                                      P->xs_colind.as<int32_t>() + P->xs_nnz_off[k],
                                      P->xsc_base.as<int32_t>() + P->xsc_boff[k],
                                      span.as<int32_t>() + P->xsc_boff[k], S(P)));
        auto *d = scr<unsigned long long>(P, kOffSum);
        SPMV_HIP(launch_max_i32(span.as<int32_t>(), ns * nb, scr<int32_t>(P, kOffPart), d, S(P)));
        SPMV_HIP(hipMemcpyAsync(P->h_pinned, d, 8, hipMemcpyDeviceToHost, S(P)));
        SPMV_TRY(sync(P));
        unsigned long long m = 0;
        memcpy(&m, P->h_pinned, 8);
        mx = (int32_t)m;
    }
    P->xsc_span = mx;
    P->xsc_feasible = mx <= 65535;
    return SPMV_OK;
}

spmv_status_t build_format(spmv_plan *P, int v) {
    const int coded = P->code_of(v);
    if (coded && (v == V_CSR_SCALAR || v == V_CSR_VECTOR))
        return fail(SPMV_ERR_INFEASIBLE, "%s has no coded-index form",
                    v == V_CSR_SCALAR ? "CSR_SCALAR" : "CSR_VECTOR");
    if (v == V_DELTA16 && P->idx_req == 0)
        return fail(SPMV_ERR_INFEASIBLE, "DELTA16 is the coded form: int32 indices requested");
    switch (v) {
    case V_CSR_SCALAR:
    case V_CSR_VECTOR:
        return SPMV_OK;
    case V_SHORT_ROW: {
        if (!coded || P->srow_coded_built) return SPMV_OK;
        // with codes: the rows-streamed delta16 arrays (block references
        // from the feasibility check, 16-bit offsets from them)
        SPMV_TRY(check_d16(P));
        if (!d16_feasible(P))
            return fail(SPMV_ERR_INFEASIBLE, "SHORT_ROW codes: a block of rows spans more than 65536 columns");
        if (!(P->d16_built && P->d16_layout == 0)) {
            SPMV_TRY(P->d16_off.alloc((size_t)(P->nnz > 0 ? P->nnz : 1) * 2 + 16));
            SPMV_TRY(ensure_d16_base(P));
            SPMV_HIP(launch_delta16_encode(*P, P->d16_base.as<int32_t>(),
                                           P->d16_off.as<uint16_t>(), S(P)));
            SPMV_TRY(sync(P));
        }
        P->srow_coded_built = true;
        return SPMV_OK;
    }
    case V_DELTA16: {
        if (P->d16_built) return SPMV_OK;
        SPMV_TRY(d16_decide_layout(P));
        if (P->d16_layout == 1) {
            const size_t slots = (size_t)P->d16_slots;
            const bool d8 = P->d16_offw == 8;
            // 8-bit codes: one byte per slot plus a spare unit per slice
            const size_t cbytes = d8 ? slots + (size_t)(2 * kSellRows) * P->d16_nsl : slots * 2;
            SPMV_TRY(P->d16s_off.alloc(cbytes + 16));
            SPMV_TRY(P->d16s_val.alloc(slots * vbytes(P->dtype) + 16));
            const size_t mbytes = (size_t)(P->n > 0 ? P->n : 1) * 4;
            SPMV_TRY(P->d16s_mask.alloc(mbytes));
            SPMV_HIP(hipMemsetAsync(P->d16s_off.p, 0, cbytes + 16, S(P)));
            SPMV_HIP(hipMemsetAsync(P->d16s_val.p, 0, slots * vbytes(P->dtype) + 16, S(P)));
            SPMV_HIP(launch_sliced_scatter(*P, P->d16s_units.as<int32_t>(), P->d16s_base.as<int32_t>(),
                                           P->d16s_kind.as<int32_t>(), P->d16s_diag.as<int32_t>(),
                                           d8 ? nullptr : P->d16s_off.as<uint16_t>(),
                                           d8 ? P->d16s_off.as<uint8_t>() : nullptr, P->d16s_val.p,
                                           P->d16s_mask.as<uint32_t>(), S(P)));
            if (d8) {
                const size_t eb = (size_t)P->d16_esc_units * kSellRows * 4 + 16;
                SPMV_TRY(P->d16s_esc.alloc(eb));
                SPMV_HIP(hipMemsetAsync(P->d16s_esc.p, 0, eb, S(P)));
                if (P->d16_esc_units > 0)
                    SPMV_HIP(launch_sliced_escape_cols(*P, P->d16s_base.as<int32_t>(),
                                                       P->d16s_kind.as<int32_t>(),
                                                       P->d16s_eunits.as<int32_t>(),
                                                       P->d16s_esc.as<int32_t>(), S(P)));
            } else {
                P->d16s_esc.release();
            }
            SPMV_TRY(sync(P));
            P->d16s_pinv.release();  // the scatter's; the layout is decided again before any rebuild
            P->d16_built = true;
            return SPMV_OK;
        }
        SPMV_TRY(P->d16_off.alloc((size_t)(P->nnz > 0 ? P->nnz : 1) * 2 + 16));
        SPMV_TRY(ensure_d16_base(P));
        SPMV_HIP(launch_delta16_encode(*P, P->d16_base.as<int32_t>(), P->d16_off.as<uint16_t>(),
                                       S(P)));
        SPMV_TRY(sync(P));
        P->d16_built = true;
        return SPMV_OK;
    }
    case V_MERGE_PATH: {
        if (P->mp_built && (!coded || P->mpc_built)) return SPMV_OK;
        if (P->mp_built) {  // splits there, codes wanted
            SPMV_TRY(check_merge_codes(P));
            if (!P->mpc_feasible)
                return fail(SPMV_ERR_INFEASIBLE, "MERGE_PATH codes: a tile spans %d columns (> 65535)",
                            (int)P->mpc_span);
            SPMV_TRY(P->mpc_off.alloc((size_t)(P->nnz > 0 ? P->nnz : 1) * 2 + 16));
            SPMV_HIP(launch_range_encode(P->mp_tiles, P->mp_tiles, 1, P->mp_split_nnz.as<int32_t>(),
                                         P->colind, P->mpc_base.as<int32_t>(), P->mpc_off.as<uint16_t>(),
                                         S(P)));
            SPMV_TRY(sync(P));
            P->mpc_built = true;
            return SPMV_OK;
        }
        const int64_t tiles = (P->n + P->nnz + kMergeTile - 1) / kMergeTile;
        P->mp_tiles = tiles;
        SPMV_TRY(P->mp_split_row.alloc((size_t)(tiles + 1) * 4));
        SPMV_TRY(P->mp_split_nnz.alloc((size_t)(tiles + 1) * 4));
        SPMV_TRY(P->mp_carry_row.alloc((size_t)(tiles > 0 ? tiles : 1) * 4));
        SPMV_TRY(P->mp_carry_val.alloc((size_t)(tiles > 0 ? tiles : 1) * 8));
        SPMV_HIP(launch_merge_splits(P->rowptr, P->n, P->nnz, P->mp_split_row.as<int32_t>(),
                                     P->mp_split_nnz.as<int32_t>(), tiles, S(P)));
        SPMV_TRY(sync(P));
        P->mp_built = true;
        return coded ? build_format(P, v) : SPMV_OK;
    }
    case V_XBLOCK_LDS: {
        SPMV_TRY(build_xslices(P));
        if (!coded || P->xsc_built) return SPMV_OK;
        SPMV_TRY(check_xblock_codes(P));
        if (!P->xsc_feasible)
            return fail(SPMV_ERR_INFEASIBLE, P->xs_rows == 0
                        ? "XBLOCK_LDS codes: the slices use merge-path tiles (no coded form)"
                        : "XBLOCK_LDS codes: a row block of a slice spans %d columns (> 65535)",
                        (int)P->xsc_span);
        const size_t len = (size_t)(P->nnz + 8 * P->xs_slices);
        SPMV_TRY(P->xsc_off.alloc(len * 2 + 16));
        SPMV_HIP(hipMemsetAsync(P->xsc_off.p, 0, len * 2 + 16, S(P)));
        const int64_t n = P->n, H = P->xsc_h, nb = (n + H - 1) / H;
        for (int k = 0; k < P->xs_slices && nb > 0; ++k)
            SPMV_HIP(launch_range_encode(nb, n, H, P->xs_rowptr.as<int32_t>() + (size_t)k * (n + 1),
                                         P->xs_colind.as<int32_t>() + P->xs_nnz_off[k],
                                         P->xsc_base.as<int32_t>() + P->xsc_boff[k],
                                         P->xsc_off.as<uint16_t>() + P->xs_nnz_off[k], S(P)));
        SPMV_TRY(sync(P));
        P->xsc_built = true;
        return SPMV_OK;
    }
    default:
        return fail(SPMV_ERR_ARG, "unknown variant %d", v);
    }
}

// 1 if variant v (format built) sums every row from +0 in increasing column
// order, one product at a time: Algorithm 1's order, so FP64 results equal
// the sequential sum bit for bit.
int column_order(const spmv_plan *P, int v) {
    switch (v) {
    case V_CSR_SCALAR:
    case V_SHORT_ROW:
    case V_DELTA16: return 1;
    case V_XBLOCK_LDS: return P->xs_pj > 0 ? 1 : 0;
    default: return 0;
    }
}

// Variants that can run this matrix under the plan's index-coding request
// (coded forms: their 16-bit codes must fit; building their base format to
// find out).
spmv_status_t feasible_mask(spmv_plan *P, uint32_t *bits) {
    SPMV_TRY(check_d16(P));
    uint32_t b = 0;
    if (P->idx_req != 1) {
        b = (1u << V_CSR_SCALAR) | (1u << V_CSR_VECTOR) | (1u << V_MERGE_PATH) |
            (1u << V_SHORT_ROW) | (1u << V_XBLOCK_LDS);
        if (d16_feasible(P) && P->idx_req != 0) b |= 1u << V_DELTA16;
    } else {
        if (d16_feasible(P)) b |= (1u << V_DELTA16) | (1u << V_SHORT_ROW);
        if (!P->mp_built) {
            const int req = P->idx_req;
            P->idx_req = 0;  // the splits alone
            const spmv_status_t st = build_format(P, V_MERGE_PATH);
            P->idx_req = req;
            SPMV_TRY(st);
        }
        SPMV_TRY(check_merge_codes(P));
        if (P->mpc_feasible) b |= 1u << V_MERGE_PATH;
        SPMV_TRY(build_xslices(P));
        SPMV_TRY(check_xblock_codes(P));
        if (P->xsc_feasible) b |= 1u << V_XBLOCK_LDS;
    }
    *bits = b;
    return SPMV_OK;
}


spmv_status_t ensure_timing_vectors(spmv_plan *P) {
    const size_t xb = xbytes(P->dtype);
    SPMV_TRY(P->tx.alloc((size_t)(P->m > 0 ? P->m : 1) * xb));
    SPMV_TRY(P->ty.alloc((size_t)(P->n > 0 ? P->n : 1) * xb));
    SPMV_HIP(hipMemsetAsync(P->tx.p, 0, P->tx.bytes, S(P)));
    return SPMV_OK;
}

spmv_status_t flush_cache(hipStream_t s) {
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    DevBuf *b;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_flush.find(dev);
        if (it == g_flush.end()) it = g_flush.emplace(dev, new DevBuf()).first;
        b = it->second;
        if (!b->p) {
            SPMV_TRY(b->alloc(kFlushBytes + kFlushSink));
            SPMV_HIP(hipMemset(b->p, 0, kFlushBytes + kFlushSink));
        }
    }
    SPMV_HIP(launch_flush(b->p, kFlushBytes, s));  // (its sink words follow the buffer)
    return SPMV_OK;
}

double median(std::vector<double> v) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const size_t k = v.size();
    return k % 2 ? v[k / 2] : 0.5 * (v[k / 2 - 1] + v[k / 2]);
}

spmv_status_t time_runs(spmv_plan *P, int reps, bool cold,
                        const std::function<spmv_status_t()> &run, std::vector<double> *out) {
    hipEvent_t a, b;
    SPMV_HIP(hipEventCreate(&a));
    SPMV_HIP(hipEventCreate(&b));
    spmv_status_t st = SPMV_OK;
    for (int r = 0; r < reps && st == SPMV_OK; ++r) {
        if (cold) st = flush_cache(S(P));
        if (st != SPMV_OK) break;
        if (hipEventRecord(a, S(P)) != hipSuccess) { st = fail(SPMV_ERR_HIP, "event"); break; }
        st = run();
        if (st != SPMV_OK) break;
        if (hipEventRecord(b, S(P)) != hipSuccess) { st = fail(SPMV_ERR_HIP, "event"); break; }
        if (hipEventSynchronize(b) != hipSuccess) { st = fail(SPMV_ERR_HIP, "event sync"); break; }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, a, b) != hipSuccess) { st = fail(SPMV_ERR_HIP, "event time"); break; }
        out->push_back(ms * 1e-3);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

// ------------------------------------------------------------ profiling
spmv_status_t profile_measure(spmv_plan *P, int reps, double meas[5]) {
    for (int i = 0; i < 5; ++i) meas[i] = 0.0;
    if (P->n == 0) return SPMV_OK;
    if (!P->part_built) {
        SPMV_TRY(P->part_bounds.alloc((size_t)(P->parts + 1) * 4));
        SPMV_HIP(launch_partition(P->rowptr, P->n, P->parts, P->part_bounds.as<int32_t>(), S(P)));
        P->part_built = true;
    }
    SPMV_TRY(ensure_timing_vectors(P));
    DevBuf stamps, rowcols, rp64, ci64;  // rowcols: every index of row i is i mod M
    SPMV_TRY(stamps.alloc((size_t)P->parts * 16));
    SPMV_TRY(rowcols.alloc((size_t)(P->nnz > 0 ? P->nnz : 1) * 4));
    SPMV_TRY(rp64.alloc((size_t)(P->n + 1) * 8));
    SPMV_TRY(ci64.alloc((size_t)(P->nnz > 0 ? P->nnz : 1) * 8));
    SPMV_HIP(launch_row_columns(*P, rowcols.as<int32_t>(), S(P)));
    SPMV_HIP(launch_widen(P->rowptr, rp64.as<int64_t>(), P->n + 1, S(P)));
    SPMV_HIP(launch_widen(P->colind, ci64.as<int64_t>(), P->nnz, S(P)));
    const int32_t *bounds = P->part_bounds.as<int32_t>();
    auto *st = stamps.as<unsigned long long>();
    auto base = [&]() -> spmv_status_t {
        SPMV_HIP(launch_csr_part(*P, bounds, P->rowptr, P->colind, nullptr, nullptr, P->tx.p,
                                 P->ty.p, st, S(P)));
        return SPMV_OK;
    };
    auto nox = [&]() -> spmv_status_t {
        SPMV_HIP(launch_csr_part(*P, bounds, P->rowptr, rowcols.as<int32_t>(), nullptr, nullptr,
                                 P->tx.p, P->ty.p, st, S(P)));
        return SPMV_OK;
    };
    auto inf = [&]() -> spmv_status_t {
        SPMV_HIP(launch_csr_part(*P, bounds, nullptr, nullptr, rp64.as<int64_t>(),
                                 ci64.as<int64_t>(), P->tx.p, P->ty.p, st, S(P)));
        return SPMV_OK;
    };
    // warm-up of each kind
    SPMV_TRY(base());
    SPMV_TRY(nox());
    SPMV_TRY(inf());
    std::vector<double> tb, tn, ti, dmax, dmean;
    std::vector<unsigned long long> h((size_t)P->parts * 2);
    for (int r = 0; r < reps; ++r) {
        SPMV_TRY(time_runs(P, 1, false, base, &tb));
        SPMV_HIP(hipMemcpyAsync(h.data(), st, h.size() * 8, hipMemcpyDeviceToHost, S(P)));
        SPMV_TRY(sync(P));
        double mx = 0.0, sum = 0.0;
        for (int p = 0; p < P->parts; ++p) {
            const double d = (double)(h[2 * p + 1] - h[2 * p]);
            mx = d > mx ? d : mx;
            sum += d;
        }
        dmax.push_back(mx);
        dmean.push_back(sum / P->parts);
    }
    SPMV_TRY(time_runs(P, reps, false, nox, &tn));
    SPMV_TRY(time_runs(P, reps, false, inf, &ti));
    // balance score of the median baseline run
    std::vector<std::pair<double, int>> order;
    for (int r = 0; r < reps; ++r) order.push_back({dmax[r] / (dmean[r] > 0 ? dmean[r] : 1), r});
    std::sort(order.begin(), order.end());
    const int rm = order[order.size() / 2].second;
    meas[0] = median(tb);
    meas[1] = median(tn);
    meas[2] = median(ti);
    meas[3] = dmax[rm];
    meas[4] = dmean[rm];
    return SPMV_OK;
}

double ratio(double a, double b) { return b > 0 ? a / b : 0.0; }

}  // namespace

// Table 2 on the GPU: the optimisation for a bottleneck class.
int class_variant(int k, const double feats[12], const double th[4], uint32_t feas) {
    if (k == K_CML) return (feas >> V_XBLOCK_LDS) & 1 ? V_XBLOCK_LDS : V_CSR_VECTOR;
    if (k == K_MB) return (feas >> V_DELTA16) & 1 ? V_DELTA16 : V_CSR_VECTOR;
    if (k == K_IMB) return V_MERGE_PATH;
    return feats[2] <= th[3] ? V_SHORT_ROW : V_CSR_VECTOR;
}

// One SpMV with variant v (its format must be built).
spmv_status_t run_variant(const spmv_plan *P, int v, const void *x, void *y, hipStream_t s) {
    const int coded = P->code_of(v);
    if ((v == V_DELTA16 && !P->d16_built) || (v == V_MERGE_PATH && !P->mp_built) ||
        (v == V_XBLOCK_LDS && !P->xs_built) || (coded && v == V_MERGE_PATH && !P->mpc_built) ||
        (coded && v == V_XBLOCK_LDS && !P->xsc_built) || (coded && v == V_SHORT_ROW && !P->srow_coded_built))
        return fail(SPMV_ERR_ARG, "variant %d has no prepared format", v);
    if (coded && (v == V_CSR_SCALAR || v == V_CSR_VECTOR))
        return fail(SPMV_ERR_INFEASIBLE, "variant %d has no coded-index form", v);
    switch (v) {
    case V_CSR_SCALAR: SPMV_HIP(launch_csr_scalar(*P, x, y, s)); break;
    case V_CSR_VECTOR: SPMV_HIP(launch_csr_vector(*P, x, y, s)); break;
    case V_MERGE_PATH: SPMV_HIP(launch_merge_path(*P, x, y, s)); break;
    case V_DELTA16:
        if (P->d16_layout == 1) SPMV_HIP(launch_sliced_d16(*P, x, y, s));
        else SPMV_HIP(launch_rowstream(*P, true, x, y, s));
        break;
    case V_XBLOCK_LDS: SPMV_HIP(launch_xblock(*P, x, y, s)); break;
    case V_SHORT_ROW: SPMV_HIP(launch_rowstream(*P, coded == 1, x, y, s)); break;
    default: return fail(SPMV_ERR_ARG, "unknown variant %d", v);
    }
    return SPMV_OK;
}

namespace {

void cascade(const double meas[5], const double feats[12], const double th[4], uint32_t feas,
             int32_t *variant, int32_t *klass, double scores[3]) {
    const double s[3] = {ratio(meas[0], meas[1]), ratio(meas[2], meas[0]), ratio(meas[3], meas[4])};
    int order[3] = {0, 1, 2};
    std::stable_sort(order, order + 3, [&](int a, int b) { return s[a] > s[b]; });
    int k = K_CMP;
    for (int i = 0; i < 3; ++i) {
        const int b = order[i];
        if (s[b] > th[b]) {
            k = b == 0 ? K_CML : b == 1 ? K_MB : K_IMB;
            break;
        }
    }
    *variant = class_variant(k, feats, th, feas);
    *klass = k;
    if (scores)
        for (int i = 0; i < 3; ++i) scores[i] = s[i];
}

// ------------------------------------------------------------ MLP on device
spmv_status_t model_device(const float **params, const float **norm) {
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_model.loaded) return fail(SPMV_ERR_NO_MODEL, "no MLP model loaded");
    auto it = g_model.dev.find(dev);
    if (it == g_model.dev.end()) {
        DevBuf *b = new DevBuf();
        spmv_status_t st = b->alloc((kNParams + 24) * 4);
        if (st != SPMV_OK) { delete b; return st; }
        std::vector<float> host(g_model.params);
        host.insert(host.end(), g_model.norm, g_model.norm + 24);
        hipError_t e = hipMemcpy(b->p, host.data(), host.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) { delete b; return fail_hip(e, "hipMemcpy(model)", __FILE__, __LINE__); }
        it = g_model.dev.emplace(dev, b).first;
    }
    *params = it->second->as<float>();
    *norm = it->second->as<float>() + kNParams;
    return SPMV_OK;
}

spmv_status_t mlp_predict(const double f[12], uint32_t feas, hipStream_t s, float *d_out,
                          float *h_out, int32_t *variant, float *margin, int32_t *fallback,
                          float *logits, float *z) {
    const float *dp, *dn;
    SPMV_TRY(model_device(&dp, &dn));
    float tau;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        tau = g_model.tau;
    }
    SPMV_HIP(launch_mlp_infer(dp, dn, f, feas, tau, d_out, s));
    SPMV_HIP(hipMemcpyAsync(h_out, d_out, 32 * 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    int32_t v;
    memcpy(&v, &h_out[0], 4);
    if (variant) *variant = v;
    if (margin) *margin = h_out[1];
    if (fallback) *fallback = h_out[2] != 0.f;
    if (logits) memcpy(logits, h_out + 3, 6 * 4);
    if (z) memcpy(z, h_out + 9, 12 * 4);
    return SPMV_OK;
}

// The one-pass path of the learned selectors (MLP, CART, naive Bayes) for a
// plan with neither features nor the delta16 test yet, under automatic
// index coding: one kernel takes the feature sums and the delta16 block
// spans at both block heights in one pass over the rows, a second reduces
// them, finalises the features on the device and runs the selector, writing
// the record straight into pinned host memory; one wait, no allocation.
// Returns SPMV_ERR_NO_MODEL (error cleared) without launching anything when
// the selector has no model.  variant: the pick (for class labels mapped
// through Table 2 with thresholds th); margin and logits: the MLP's.
spmv_status_t select_onepass(spmv_plan *P, int32_t selector, const double th[4], uint32_t *feas,
                             int32_t *variant, float *margin, int32_t *fallback, float *logits) {
    const float *dp = nullptr, *dn = nullptr;
    float tau = 0.f;
    const int which = selector == SEL_DTREE ? 0 : 1;
    if (selector == SEL_MLP) {
        const spmv_status_t st = model_device(&dp, &dn);
        if (st == SPMV_ERR_NO_MODEL) { clear_error(); return st; }
        SPMV_TRY(st);
        std::lock_guard<std::mutex> lk(g_mu);
        tau = g_model.tau;
    } else if (!classic_loaded(which)) {
        return SPMV_ERR_NO_MODEL;
    }
    const hipStream_t s = S(P);
    // spans at the heights check_d16 tries: H0 = the short_row block, then H1 = kBlock
    const int R = P->rs_rows, H0 = R * kBlock, H1 = kBlock;
    hipError_t e = hipSuccess;
    const int parts = launch_select_pass(*P, R, scr<uint64_t>(P, kOffPart), xbytes(P->dtype), s, &e);
    SPMV_HIP(e);  // hipErrorInvalidValue for a row count per thread other than 1, 2, 4, 8
    char *h = static_cast<char *>(P->h_pinned) + 2048;
    void *hd = static_cast<char *>(P->h_pinned_dev) + 2048;
    const uint32_t base_bits = (1u << V_CSR_SCALAR) | (1u << V_CSR_VECTOR) |
                               (1u << V_MERGE_PATH) | (1u << V_SHORT_ROW) | (1u << V_XBLOCK_LDS);
    int label_kind = 0;
    if (selector == SEL_MLP) {
        SPMV_HIP(launch_mlp_select(dp, dn, scr<uint64_t>(P, kOffPart), parts, P->n, P->m, P->nnz,
                                   vbytes(P->dtype), xbytes(P->dtype), R > 1 ? 1 : 0, base_bits,
                                   tau, static_cast<float *>(hd), s));
    } else {
        const spmv_status_t st =
            classic_select_launch(which, scr<uint64_t>(P, kOffPart), parts, P->n, P->m, P->nnz,
                                  vbytes(P->dtype), xbytes(P->dtype), R > 1 ? 1 : 0, base_bits, hd,
                                  s, &label_kind);
        if (st == SPMV_ERR_NO_MODEL) {  // unloaded meanwhile: the pass only wrote scratch
            clear_error();
            return st;
        }
        SPMV_TRY(st);
    }
    SPMV_TRY(sync(P));
    double f[12];
    uint64_t w[16];
    memcpy(feas, h + 128, 4);
    memcpy(f, h + 192, sizeof f);
    memcpy(w, h + 288, sizeof w);
    // delta16: the first height whose blocks fit 16-bit offsets
    const bool ok0 = w[12] <= 65535, ok1 = R > 1 && w[13] <= 65535;
    P->d16_feasible = ok0 || ok1;
    P->d16_rows = ok0 || R == 1 ? H0 : H1;
    P->d16_checked = true;
    P->d16_base_ready = false;
    memcpy(P->feats, f, sizeof f);
    const int64_t smiss = (int64_t)(w[10] - w[11]);
    const uint64_t a[12] = {w[0], w[1], w[2], w[3], w[4], w[5],
                            w[6], w[7], w[8], w[9], (uint64_t)smiss, (uint64_t)P->nnz};
    memcpy(P->acc, a, sizeof a);
    P->have_features = true;
    if (selector == SEL_MLP) {
        float hf[9];
        memcpy(hf, h, sizeof hf);
        memcpy(variant, &hf[0], 4);
        *margin = hf[1];
        *fallback = hf[2] != 0.f;
        memcpy(logits, hf + 3, 6 * 4);
    } else {
        int32_t hi[3];
        memcpy(hi, h, sizeof hi);
        *fallback = hi[2];
        *variant = label_kind == 0 ? hi[0] : class_variant(hi[0], f, th, *feas);
    }
    return SPMV_OK;
}

// Return the plan's recycled buffers to the pools and free the rest, after
// one wait for the plan's stream (or for the device, if the plan ran on
// other streams too) instead of a device wait per buffer.
void release_plan(spmv_plan *P) {
    const bool ok = P->other_streams ? hipDeviceSynchronize() == hipSuccess
                                     : hipStreamSynchronize(P->stream) == hipSuccess;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (P->h_pinned) g_pinned_pool.push_back(P->h_pinned);
        if (P->scratch.p && P->scratch.bytes == kScratchBytes) {
            g_scratch_pool[P->device].push_back(P->scratch.p);
            P->scratch.p = nullptr;
            P->scratch.bytes = 0;
        }
    }
    P->h_pinned = nullptr;
    t_streams_synced = ok;
    delete P;
    t_streams_synced = false;
}

}  // namespace
}  // namespace spmvsel

using namespace spmvsel;

// ============================================================ C ABI
extern "C" {

const char *spmv_last_error(void) { return g_err.c_str(); }

spmv_status_t spmv_plan_create(spmv_plan_t *out, int64_t n_rows, int64_t n_cols, int64_t nnz,
                               const int32_t *d_rowptr, const int32_t *d_colind,
                               const void *d_val, int32_t val_dtype, void *stream,
                               uint32_t flags) {
    clear_error();
    if (!out) return fail(SPMV_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_rows < 0 || n_cols < 0 || nnz < 0)
        return fail(SPMV_ERR_ARG, "negative size");
    if (n_rows >= INT32_MAX || n_cols > INT32_MAX)
        return fail(SPMV_ERR_ARG, "sizes must be below 2^31");
    // the kernels step int32 nonzero indices up to a chunk (2048) past a
    // row's or a tile's end, so NNZ keeps that much headroom below 2^31
    if (nnz >= kMaxNnz) return fail(SPMV_ERR_ARG, "NNZ must be below 2^31 - 2^16");
    if (val_dtype < SPMV_F64 || val_dtype > SPMV_BF16)
        return fail(SPMV_ERR_ARG, "unknown value dtype %d", val_dtype);
    if (!d_rowptr) return fail(SPMV_ERR_ARG, "rowptr is NULL");
    if (nnz > 0 && (!d_colind || !d_val)) return fail(SPMV_ERR_ARG, "colind or val is NULL");
    if (nnz > 0 && n_rows == 0) return fail(SPMV_ERR_CSR_ROWPTR, "nonzeros without rows");
    if (((uintptr_t)d_rowptr & 3) || (nnz > 0 && (((uintptr_t)d_colind & 15) || ((uintptr_t)d_val & 15))))
        return fail(SPMV_ERR_ARG, "arrays must be 16-byte aligned (rowptr 4-byte)");
    spmv_plan *P = new (std::nothrow) spmv_plan();
    if (!P) return fail(SPMV_ERR_OOM, "host allocation failed");
    P->n = n_rows;
    P->m = n_cols;
    P->nnz = nnz;
    P->dtype = val_dtype;
    P->stream = (hipStream_t)stream;
    P->flags = flags;
    P->rowptr = d_rowptr;
    P->colind = d_colind;
    P->val = d_val;
    auto bail = [&](spmv_status_t st) {
        release_plan(P);
        return st;
    };
    spmv_status_t st;
#define BAIL_HIP(expr)                                                      \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) return bail(fail_hip(e_, #expr, __FILE__, __LINE__)); \
    } while (0)
#define BAIL(expr)                                                          \
    do {                                                                    \
        if ((st = (expr)) != SPMV_OK) return bail(st);                      \
    } while (0)
    BAIL_HIP(hipGetDevice(&P->device));
    BAIL_HIP(hipDeviceGetAttribute(&P->num_cus, hipDeviceAttributeMultiprocessorCount, P->device));
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_pinned_pool.empty()) {
            P->h_pinned = g_pinned_pool.back();
            g_pinned_pool.pop_back();
        }
        auto &sp = g_scratch_pool[P->device];
        if (!sp.empty()) {
            P->scratch.p = sp.back();
            P->scratch.bytes = kScratchBytes;
            sp.pop_back();
        }
    }
    if (!P->h_pinned) BAIL_HIP(hipHostMalloc(&P->h_pinned, 4096, hipHostMallocDefault));
    BAIL_HIP(hipHostGetDevicePointer(&P->h_pinned_dev, P->h_pinned, 0));
    BAIL(P->scratch.alloc(kScratchBytes));
    if (flags & SPMV_COPY_INPUTS) {
        const size_t vb = vbytes(val_dtype);
        BAIL(P->own_rowptr.alloc((size_t)(n_rows + 1) * 4));
        BAIL(P->own_colind.alloc((size_t)(nnz > 0 ? nnz : 1) * 4 + 16));
        BAIL(P->own_val.alloc((size_t)(nnz > 0 ? nnz : 1) * vb + 16));
        BAIL_HIP(hipMemcpyAsync(P->own_rowptr.p, d_rowptr, (size_t)(n_rows + 1) * 4,
                                hipMemcpyDeviceToDevice, P->stream));
        if (nnz > 0) {
            BAIL_HIP(hipMemcpyAsync(P->own_colind.p, d_colind, (size_t)nnz * 4,
                                    hipMemcpyDeviceToDevice, P->stream));
            BAIL_HIP(hipMemcpyAsync(P->own_val.p, d_val, (size_t)nnz * vb,
                                    hipMemcpyDeviceToDevice, P->stream));
        }
        P->rowptr = P->own_rowptr.as<int32_t>();
        P->colind = P->own_colind.as<int32_t>();
        P->val = P->own_val.p;
    }
    // launch parameters from the mean row length
    const double avg = n_rows > 0 ? (double)nnz / (double)n_rows : 0.0;
    P->vec_width = pow2_ceil(avg, 2, 64);
    P->rs_rows = pow2_floor((double)kChunk / (kBlock * (avg > 1e-9 ? avg : 1e-9)), 1, kRowStreamMaxR);
    P->parts = P->num_cus * 8;
    if (!(flags & SPMV_SKIP_VALIDATE)) {
        uint64_t *f = scr<uint64_t>(P, kOffFlags);
        static_assert(kFeatBlocks * 16 >= kValGrid * 3, "validation partials fit the scratch");
        BAIL_HIP(launch_validate(*P, f, scr<uint64_t>(P, kOffPart), P->stream));
        BAIL_HIP(hipMemcpyAsync(P->h_pinned, f, 24, hipMemcpyDeviceToHost, P->stream));
        BAIL_HIP(hipStreamSynchronize(P->stream));
        uint64_t h[3];
        memcpy(h, P->h_pinned, 24);
        if (h[0] & 1) return bail(fail(SPMV_ERR_CSR_ROWPTR, "invalid rowptr"));
        if (h[0] & 2) return bail(fail(SPMV_ERR_CSR_COL_RANGE, "column index outside [0, %lld)", (long long)n_cols));
        if (h[1] != h[2])
            return bail(fail(SPMV_ERR_CSR_UNSORTED, "columns not strictly increasing in %llu places",
                             (unsigned long long)(h[1] - h[2])));
    } else {
        BAIL_HIP(hipStreamSynchronize(P->stream));
    }
#undef BAIL
#undef BAIL_HIP
    *out = P;
    return SPMV_OK;
}

spmv_status_t spmv_plan_destroy(spmv_plan_t P) {
    if (!P) return SPMV_OK;
    release_plan(P);
    return SPMV_OK;
}

spmv_status_t spmv_features(spmv_plan_t P, double out[12], uint64_t acc[12]) {
    clear_error();
    if (!P || !out) return fail(SPMV_ERR_ARG, "NULL argument");
    SPMV_TRY(ensure_features(P));
    memcpy(out, P->feats, sizeof P->feats);
    if (acc) memcpy(acc, P->acc, sizeof P->acc);
    return SPMV_OK;
}

spmv_status_t spmv_execute(spmv_plan_t P, const void *d_x, void *d_y, void *stream) {
    if (!P) return fail(SPMV_ERR_ARG, "plan is NULL");
    if (P->n > 0 && !d_y) return fail(SPMV_ERR_ARG, "y is NULL");
    if (P->nnz > 0 && !d_x) return fail(SPMV_ERR_ARG, "x is NULL");
    if ((hipStream_t)stream != P->stream) P->other_streams = true;
    return run_variant(P, P->variant, d_x, d_y, (hipStream_t)stream);
}

spmv_status_t spmv_set_variant(spmv_plan_t P, int32_t v) {
    clear_error();
    if (!P) return fail(SPMV_ERR_ARG, "plan is NULL");
    if (v < 0 || v >= SPMV_N_VARIANTS) return fail(SPMV_ERR_ARG, "unknown variant %d", v);
    SPMV_TRY(build_format(P, v));
    P->variant = v;
    return SPMV_OK;
}

spmv_status_t spmv_set_index_coding(spmv_plan_t P, int32_t coding) {
    clear_error();
    if (!P) return fail(SPMV_ERR_ARG, "plan is NULL");
    if (coding < -1 || coding > 1)
        return fail(SPMV_ERR_ARG, "index coding must be -1 (each variant's own), 0 (int32) or 1 (16-bit codes)");
    if (coding == P->idx_req) return SPMV_OK;
    P->idx_req = coding;
    // the current variant's format under the new coding, when it has one
    const spmv_status_t st = build_format(P, P->variant);
    if (st == SPMV_ERR_INFEASIBLE) {
        clear_error();
        return SPMV_OK;
    }
    return st;
}

spmv_status_t spmv_set_kahan_min_len(spmv_plan_t P, int32_t len) {
    clear_error();
    if (!P) return fail(SPMV_ERR_ARG, "plan is NULL");
    if (len < 1) return fail(SPMV_ERR_ARG, "length must be at least 1 (INT32_MAX: no compensation)");
    P->kahan_min = len;
    return SPMV_OK;
}

spmv_status_t spmv_get_variant(spmv_plan_t P, int32_t *v) {
    if (!P || !v) return fail(SPMV_ERR_ARG, "NULL argument");
    *v = P->variant;
    return SPMV_OK;
}

spmv_status_t spmv_variant_mask(spmv_plan_t P, uint32_t *bits) {
    clear_error();
    if (!P || !bits) return fail(SPMV_ERR_ARG, "NULL argument");
    return feasible_mask(P, bits);
}

spmv_status_t spmv_bytes(spmv_plan_t P, int32_t v, int64_t *bytes) {
    if (!P || !bytes) return fail(SPMV_ERR_ARG, "NULL argument");
    if (v < 0 || v >= SPMV_N_VARIANTS) return fail(SPMV_ERR_ARG, "unknown variant %d", v);
    const int64_t vb = vbytes(P->dtype), xb = xbytes(P->dtype);
    const int coded = P->code_of(v);
    const int64_t ib = coded ? 2 : 4;
    int64_t extra = 0;
    if (coded && v == V_MERGE_PATH) extra = 4 * ((P->n + P->nnz + kMergeTile - 1) / kMergeTile);
    if (coded && v == V_XBLOCK_LDS) {  // a reference column per slice and row block
        SPMV_TRY(build_xslices(P));
        const int64_t H = P->xs_pj > 0 ? kBlock : (P->xs_rows > 0 ? P->xs_rows : kBlock);
        extra = 4 * (int64_t)P->xs_slices * ((P->n + H - 1) / H);
    }
    if (coded && v == V_SHORT_ROW) {  // the rows-streamed delta16 layout
        SPMV_TRY(check_d16(P));
        extra = 4 * ((P->n + P->d16_rows - 1) / P->d16_rows);
    }
    if (v == V_DELTA16) {  // also defined where the variant is infeasible
        SPMV_TRY(check_d16(P));
        if (d16_feasible(P)) SPMV_TRY(d16_decide_layout(P));
        if (d16_feasible(P) && P->d16_layout == 1) {
            // offsets only in offset slices; width, units, base and kind per
            // slice, the column span per offset slice, 32 diagonals per
            // diagonal slice; a row's mask replaces its row pointer in
            // diagonal slices
            // 8-bit codes: 4 bytes per escaped column and 4 per offset slice
            // (its first escape unit, read only there)
            const bool d8 = P->d16_offw == 8;
            const int64_t n_off = P->d16_nsl - P->d16_ndiag;
            *bytes = 4 * (P->n + 1) + vb * P->nnz + (d8 ? 1 : 2) * P->d16_nnz_off +
                     (d8 ? 4 * P->d16_nesc + 4 * n_off : 0) + xb * P->m + xb * P->n +
                     16 * P->d16_nsl + 4 * n_off + 4 * kSellMaxDiag * P->d16_ndiag +
                     (P->d16_sort ? 4 * P->n : 0);  // the sorted layout's row index per row
            return SPMV_OK;
        }
        extra = 4 * ((P->n + P->d16_rows - 1) / P->d16_rows);
    }
    *bytes = 4 * (P->n + 1) + (ib + vb) * P->nnz + xb * P->m + xb * P->n + extra;
    return SPMV_OK;
}

spmv_status_t spmv_time_variant(spmv_plan_t P, int32_t v, int32_t reps, int32_t cold,
                                double *t_med, double *t_min) {
    clear_error();
    if (!P || reps < 1) return fail(SPMV_ERR_ARG, "bad argument");
    SPMV_TRY(build_format(P, v));
    SPMV_TRY(ensure_timing_vectors(P));
    auto run = [&]() { return run_variant(P, v, P->tx.p, P->ty.p, S(P)); };
    SPMV_TRY(run());
    SPMV_TRY(run());
    std::vector<double> t;
    SPMV_TRY(time_runs(P, reps, cold != 0, run, &t));
    if (t_med) *t_med = median(t);
    if (t_min) *t_min = *std::min_element(t.begin(), t.end());
    return SPMV_OK;
}

spmv_status_t spmv_time_variant_batch(spmv_plan_t P, int32_t v, int32_t launches, int32_t reps,
                                      double *t_med, double *t_min) {
    clear_error();
    if (!P || reps < 1 || launches < 1 || launches > 100000) return fail(SPMV_ERR_ARG, "bad argument");
    SPMV_TRY(build_format(P, v));
    SPMV_TRY(ensure_timing_vectors(P));
    auto one = [&]() { return run_variant(P, v, P->tx.p, P->ty.p, S(P)); };
    auto batch = [&]() -> spmv_status_t {
        for (int i = 0; i < launches; ++i) SPMV_TRY(one());
        return SPMV_OK;
    };
    SPMV_TRY(one());
    SPMV_TRY(one());
    std::vector<double> t;
    SPMV_TRY(time_runs(P, reps, false, batch, &t));
    for (double &u : t) u /= launches;
    if (t_med) *t_med = median(t);
    if (t_min) *t_min = *std::min_element(t.begin(), t.end());
    return SPMV_OK;
}

spmv_status_t spmv_plan_query(spmv_plan_t P, int32_t key, int64_t *value) {
    clear_error();
    if (!P || !value) return fail(SPMV_ERR_ARG, "NULL argument");
    switch (key) {
    case 0: *value = P->variant; break;
    case 1: *value = P->vec_width; break;
    case 2: *value = P->rs_rows * kBlock; break;
    case 3: *value = kMergeTile; break;
    case 4: *value = (P->n + P->nnz + kMergeTile - 1) / kMergeTile; break;
    case 5: *value = xs_slice_width(P, xs_slice_count(P)); break;
    case 6: SPMV_TRY(build_xslices(P)); *value = P->xs_tile_off[P->xs_slices - 1] + P->xs_tiles[P->xs_slices - 1]; break;
    case 7: *value = xs_slice_count(P); break;
    case 12: SPMV_TRY(build_xslices(P)); *value = P->xs_rows; break;
    case 13: SPMV_TRY(build_xslices(P)); *value = P->xs_nlong; break;
    case 16: SPMV_TRY(build_xslices(P)); *value = P->xs_pj; break;
    case 8: *value = P->parts; break;
    case 9: SPMV_TRY(check_d16(P)); *value = d16_feasible(P); break;
    case 11: SPMV_TRY(check_d16(P)); *value = P->d16_rows; break;
    case 14:
        SPMV_TRY(check_d16(P));
        if (!d16_feasible(P)) { *value = -1; break; }
        SPMV_TRY(d16_decide_layout(P));
        *value = P->d16_layout;
        break;
    case 15: SPMV_TRY(d16_decide_layout(P)); *value = P->d16_slots; break;
    case 17:
    case 18:
    case 19:
    case 20:
        SPMV_TRY(check_d16(P));
        if (!d16_feasible(P)) { *value = -1; break; }
        SPMV_TRY(d16_decide_layout(P));
        *value = key == 17 ? P->d16_offw : key == 18 ? P->d16_span
                 : key == 19 ? P->d16_esc_units : P->d16_nesc;
        break;
    case 10: *value = 1; break;
    case 21: SPMV_TRY(build_format(P, P->variant)); *value = column_order(P, P->variant); break;
    case 22: *value = P->code_of(P->variant); break;
    case 23: {  // merge-path codes feasible (tiles of the splits)
        if (!P->mp_built) {
            const int req = P->idx_req;
            P->idx_req = 0;
            const spmv_status_t st = build_format(P, V_MERGE_PATH);
            P->idx_req = req;
            SPMV_TRY(st);
        }
        SPMV_TRY(check_merge_codes(P));
        *value = P->mpc_feasible;
        break;
    }
    case 24:
        SPMV_TRY(build_xslices(P));
        SPMV_TRY(check_xblock_codes(P));
        *value = P->xsc_feasible;
        break;
    case 25: SPMV_TRY(build_xslices(P)); SPMV_TRY(check_xblock_codes(P)); *value = P->xsc_h; break;
    case 26:
        SPMV_TRY(check_d16(P));
        if (!d16_feasible(P)) { *value = -1; break; }
        SPMV_TRY(d16_decide_layout(P));
        *value = P->d16_layout == 1 ? P->d16_sort : 0;
        break;
    default: return fail(SPMV_ERR_ARG, "unknown key %d", key);
    }
    return SPMV_OK;
}

spmv_status_t spmv_plan_copy_format(spmv_plan_t P, int32_t which, void *dst, int64_t bytes) {
    clear_error();
    if (!P || (!dst && bytes > 0)) return fail(SPMV_ERR_ARG, "NULL argument");
    const void *src = nullptr;
    int64_t want = 0;
    switch (which) {
    case 8: case 9: case 10: case 11: case 12: case 13: case 14: case 15: case 16: case 17: case 22:
        SPMV_TRY(build_format(P, V_DELTA16));
        if (P->d16_layout != 1) return fail(SPMV_ERR_ARG, "delta16 is not in the sliced layout");
        switch (which) {
        case 8: src = P->d16s_width.p; want = 4 * P->d16_nsl; break;
        case 9: src = P->d16s_units.p; want = 4 * P->d16_nsl; break;
        case 10: src = P->d16s_base.p; want = 4 * P->d16_nsl; break;
        case 11:
            src = P->d16s_off.p;
            want = P->d16_offw == 8 ? P->d16_slots + 2 * kSellRows * P->d16_nsl : 2 * P->d16_slots;
            break;
        case 16: src = P->d16s_esc.p; want = 4 * kSellRows * P->d16_esc_units; break;
        case 17: src = P->d16s_eunits.p; want = P->d16_offw == 8 ? 4 * P->d16_nsl : 0; break;
        case 12: src = P->d16s_val.p; want = vbytes(P->dtype) * P->d16_slots; break;
        case 13: src = P->d16s_kind.p; want = 4 * P->d16_nsl; break;
        case 14: src = P->d16s_diag.p; want = 4 * kSellMaxDiag * P->d16_nsl; break;
        case 22: src = P->d16s_perm.p; want = P->d16_sort ? 4 * P->n : 0; break;
        default: src = P->d16s_mask.p; want = 4 * P->n; break;
        }
        break;
    case 0: case 1:
        SPMV_TRY(build_format(P, V_DELTA16));
        if (P->d16_layout != 0) return fail(SPMV_ERR_ARG, "delta16 is not in the streamed layout");
        if (which == 0) SPMV_TRY(ensure_d16_base(P));
        src = which == 0 ? P->d16_base.p : P->d16_off.p;
        want = which == 0 ? 4 * ((P->n + P->d16_rows - 1) / P->d16_rows) : 2 * P->nnz;
        break;
    case 2: case 3:
        SPMV_TRY(build_format(P, V_MERGE_PATH));
        src = which == 2 ? P->mp_split_row.p : P->mp_split_nnz.p;
        want = 4 * (P->mp_tiles + 1);
        break;
    case 4: case 5:
        SPMV_TRY(build_xslices(P));
        if (which == 5) {  // the slices without their alignment padding
            const int64_t want5 = 4 * (P->nnz - P->xs_long_nnz);
            if (bytes != want5) return fail(SPMV_ERR_ARG, "array 5 has %lld bytes", (long long)want5);
            int64_t done = 0;
            for (int k = 0; k < P->xs_slices; ++k) {
                int32_t last = 0;
                SPMV_HIP(hipMemcpy(&last, P->xs_rowptr.as<int32_t>() + (size_t)k * (P->n + 1) + P->n, 4,
                                   hipMemcpyDeviceToHost));
                if (last > 0)
                    SPMV_HIP(hipMemcpy(static_cast<int32_t *>(dst) + done,
                                       P->xs_colind.as<int32_t>() + P->xs_nnz_off[k], (size_t)last * 4,
                                       hipMemcpyDeviceToHost));
                done += last;
            }
            return SPMV_OK;
        }
        src = P->xs_rowptr.p;
        want = 4 * P->xs_slices * (P->n + 1);
        break;
    case 6:
        if (!P->part_built) {
            SPMV_TRY(P->part_bounds.alloc((size_t)(P->parts + 1) * 4));
            SPMV_HIP(launch_partition(P->rowptr, P->n, P->parts, P->part_bounds.as<int32_t>(), S(P)));
            P->part_built = true;
        }
        src = P->part_bounds.p;
        want = 4 * (P->parts + 1);
        break;
    case 7:
        SPMV_TRY(build_xslices(P));
        src = P->xs_lrows.p;
        want = 4 * P->xs_nlong;
        break;
    case 18: case 19: {  // coded merge path
        const int req = P->idx_req;
        P->idx_req = 1;
        const spmv_status_t st = build_format(P, V_MERGE_PATH);
        P->idx_req = req;
        SPMV_TRY(st);
        src = which == 18 ? P->mpc_base.p : P->mpc_off.p;
        want = which == 18 ? 4 * P->mp_tiles : 2 * P->nnz;
        break;
    }
    case 20: case 21: {  // coded x blocking
        const int req = P->idx_req;
        P->idx_req = 1;
        const spmv_status_t st = build_format(P, V_XBLOCK_LDS);
        P->idx_req = req;
        SPMV_TRY(st);
        if (which == 21) {  // the codes of the slices without their alignment padding
            const int64_t want21 = 2 * (P->nnz - P->xs_long_nnz);
            if (bytes != want21) return fail(SPMV_ERR_ARG, "array 21 has %lld bytes", (long long)want21);
            int64_t done = 0;
            for (int k = 0; k < P->xs_slices; ++k) {
                int32_t last = 0;
                SPMV_HIP(hipMemcpy(&last, P->xs_rowptr.as<int32_t>() + (size_t)k * (P->n + 1) + P->n, 4,
                                   hipMemcpyDeviceToHost));
                if (last > 0)
                    SPMV_HIP(hipMemcpy(static_cast<uint16_t *>(dst) + done,
                                       P->xsc_off.as<uint16_t>() + P->xs_nnz_off[k], (size_t)last * 2,
                                       hipMemcpyDeviceToHost));
                done += last;
            }
            return SPMV_OK;
        }
        src = P->xsc_base.p;
        want = 4 * P->xsc_boff[P->xs_slices];
        break;
    }
    default: return fail(SPMV_ERR_ARG, "unknown array %d", which);
    }
    if (bytes != want) return fail(SPMV_ERR_ARG, "array %d has %lld bytes, not %lld", which,
                                   (long long)want, (long long)bytes);
    if (want > 0) SPMV_HIP(hipMemcpyAsync(dst, src, (size_t)want, hipMemcpyDeviceToHost, S(P)));
    return sync(P);
}

spmv_status_t spmv_profile_measure(spmv_plan_t P, int32_t reps, double meas[5]) {
    clear_error();
    if (!P || !meas || reps < 1) return fail(SPMV_ERR_ARG, "bad argument");
    return profile_measure(P, reps, meas);
}

spmv_status_t spmv_profile_decide(const double meas[5], const double feats[12],
                                  const double theta[4], uint32_t feas, int32_t *variant,
                                  int32_t *klass) {
    clear_error();
    if (!meas || !feats || !theta || !variant || !klass) return fail(SPMV_ERR_ARG, "NULL argument");
    cascade(meas, feats, theta, feas, variant, klass, nullptr);
    return SPMV_OK;
}

spmv_status_t spmv_set_thresholds(const double theta[4]) {
    if (!theta) return fail(SPMV_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_mu);
    memcpy(g_theta, theta, sizeof g_theta);
    return SPMV_OK;
}

spmv_status_t spmv_get_thresholds(double theta[4]) {
    if (!theta) return fail(SPMV_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_mu);
    memcpy(theta, g_theta, sizeof g_theta);
    return SPMV_OK;
}

spmv_status_t spmv_select(spmv_plan_t P, int32_t selector, spmv_select_info_t *info) {
    clear_error();
    if (!P) return fail(SPMV_ERR_ARG, "plan is NULL");
    if (selector < SEL_PROFILING || selector > SEL_GNB)
        return fail(SPMV_ERR_ARG, "unknown selector %d", selector);
    spmv_select_info_t I;
    memset(&I, 0, sizeof I);
    I.klass = -1;
    double th[4];
    spmv_get_thresholds(th);
    const double t0 = now_s();
    uint32_t feas = 0;
    int32_t v = V_CSR_VECTOR;
    int used = selector;
    bool onepass = false;
    const bool learned = selector == SEL_MLP || selector == SEL_DTREE || selector == SEL_GNB;
    if (learned && !P->have_features && !P->d16_checked && P->idx_req < 0 && P->n > 0) {
        int32_t fb = 1;
        const spmv_status_t st = select_onepass(P, selector, th, &feas, &v, &I.margin, &fb, I.logits);
        if (st == SPMV_OK) {
            onepass = true;
            if (fb || v < 0 || !((feas >> v) & 1)) {
                I.fell_back = 1;
                used = SEL_PROFILING;
            }
        } else if (st != SPMV_ERR_NO_MODEL) {
            return st;
        }
    }
    if (!onepass) {
        SPMV_TRY(ensure_features(P));
        SPMV_TRY(feasible_mask(P, &feas));
    }
    const double t1 = now_s();
    I.t_features_s = t1 - t0;
    I.feasible = feas;
    memcpy(I.features, P->feats, sizeof I.features);
    if (selector == SEL_MLP && !onepass) {
        int32_t fb = 1;
        spmv_status_t st = mlp_predict(P->feats, feas, S(P), scr<float>(P, kOffMlp),
                                       static_cast<float *>(P->h_pinned) + 512, &v, &I.margin,
                                       &fb, I.logits, nullptr);
        if (st == SPMV_ERR_NO_MODEL) { fb = 1; clear_error(); }
        else if (st != SPMV_OK) return st;
        I.t_decide_s = now_s() - t1;
        if (fb || v < 0) {
            I.fell_back = 1;
            used = SEL_PROFILING;
        }
    } else if ((selector == SEL_DTREE || selector == SEL_GNB) && !onepass) {
        int32_t fb = 1, lab = -1;
        spmv_status_t st = classic_predict(selector == SEL_DTREE ? 0 : 1, P->feats, feas, th, S(P),
                                           scr<char>(P, kOffClf), &v, &lab, &fb);
        if (st == SPMV_ERR_NO_MODEL) { fb = 1; clear_error(); }
        else if (st != SPMV_OK) return st;
        I.t_decide_s = now_s() - t1;
        if (fb || v < 0 || !((feas >> v) & 1)) {
            I.fell_back = 1;
            used = SEL_PROFILING;
        }
    }
    if (used == SEL_PROFILING) {
        const double tp = now_s();
        SPMV_TRY(profile_measure(P, 3, I.meas));
        const double tq = now_s();
        I.t_profile_s = tq - tp;
        cascade(I.meas, P->feats, th, feas, &v, &I.klass, I.scores);
        I.t_decide_s += now_s() - tq;
    } else if (used == SEL_EXHAUSTIVE) {
        double best = 0;
        v = -1;
        for (int k = 0; k < SPMV_N_VARIANTS; ++k) {
            if (!((feas >> k) & 1)) continue;
            double tm = 0;
            SPMV_TRY(spmv_time_variant(P, k, 10, 0, &tm, nullptr));
            I.variant_times_s[k] = tm;
            if (v < 0 || tm < best) { best = tm; v = k; }
        }
        I.t_decide_s = now_s() - t1;
    }
    I.t_total_s = now_s() - t0;
    I.selector = used;
    const double tp0 = now_s();
    SPMV_TRY(build_format(P, v));
    I.t_prepare_s = now_s() - tp0;
    P->variant = v;
    I.variant = v;
    if (info) *info = I;
    return SPMV_OK;
}

spmv_status_t spmv_model_load(const char *path) {
    clear_error();
    if (!path) return fail(SPMV_ERR_ARG, "NULL path");
    FILE *fp = fopen(path, "rb");
    if (!fp) return fail(SPMV_ERR_NO_MODEL, "cannot open %s", path);
    std::vector<unsigned char> buf;
    unsigned char tmp[65536];
    size_t got;
    while ((got = fread(tmp, 1, sizeof tmp, fp)) > 0) buf.insert(buf.end(), tmp, tmp + got);
    fclose(fp);
    const size_t want = 8 + 4 + 4 + 24 * 4 + 4 + (size_t)kNParams * 4 + 4;
    if (buf.size() != want) return fail(SPMV_ERR_NO_MODEL, "%s: %zu bytes, expected %zu", path, buf.size(), want);
    if (memcmp(buf.data(), "SPMVMLP1", 8) != 0) return fail(SPMV_ERR_NO_MODEL, "%s: bad magic", path);
    uint32_t ver, np, crc;
    memcpy(&ver, &buf[8], 4);
    memcpy(&np, &buf[12], 4);
    memcpy(&crc, &buf[want - 4], 4);
    if (ver != 1 || np != (uint32_t)kNParams) return fail(SPMV_ERR_NO_MODEL, "%s: bad header", path);
    if (crc32(buf.data(), want - 4) != crc) return fail(SPMV_ERR_NO_MODEL, "%s: CRC mismatch", path);
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_model.dev) delete kv.second;
    g_model.dev.clear();
    memcpy(g_model.norm, &buf[16], 24 * 4);
    memcpy(&g_model.tau, &buf[16 + 96], 4);
    g_model.params.resize(kNParams);
    memcpy(g_model.params.data(), &buf[16 + 96 + 4], (size_t)kNParams * 4);
    g_model.loaded = true;
    return SPMV_OK;
}

spmv_status_t spmv_model_unload(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_model.dev) delete kv.second;
    g_model.dev.clear();
    g_model.loaded = false;
    return SPMV_OK;
}

spmv_status_t spmv_mlp_predict(const double features[12], uint32_t feas, int32_t *variant,
                               float *margin, int32_t *fallback, float logits[6], float z[12]) {
    clear_error();
    if (!features) return fail(SPMV_ERR_ARG, "NULL features");
    DevBuf out;
    SPMV_TRY(out.alloc(256));
    float h[32];
    spmv_status_t st = mlp_predict(features, feas, nullptr, out.as<float>(), h, variant, margin,
                                   fallback, logits, z);
    return st;
}

spmv_status_t spmv_mlp_forward_backward(const float *params, const float *Z, const int32_t *labels,
                                        const uint8_t *mask, int32_t B, float *grads, float *loss,
                                        void *stream) {
    clear_error();
    if (!params || !Z || !labels || !mask || !grads || !loss || B < 1 || B > 1024)
        return fail(SPMV_ERR_ARG, "bad argument");
    SPMV_HIP(launch_mlp_fwd_bwd(params, Z, labels, nullptr, mask, B, grads, loss,
                                (hipStream_t)stream));
    return SPMV_OK;
}

spmv_status_t spmv_mlp_forward_backward_sets(const float *params, const float *Z,
                                             const uint8_t *accept, const uint8_t *mask, int32_t B,
                                             float *grads, float *loss, void *stream) {
    clear_error();
    if (!params || !Z || !accept || !mask || !grads || !loss || B < 1 || B > 1024)
        return fail(SPMV_ERR_ARG, "bad argument");
    SPMV_HIP(launch_mlp_fwd_bwd(params, Z, nullptr, accept, mask, B, grads, loss,
                                (hipStream_t)stream));
    return SPMV_OK;
}

spmv_status_t spmv_mlp_adam_step(float *p, const float *g, float *m, float *v, int32_t n,
                                 int32_t step, float lr, float b1, float b2, float eps,
                                 void *stream) {
    clear_error();
    if (!p || !g || !m || !v || n < 0 || step < 1) return fail(SPMV_ERR_ARG, "bad argument");
    SPMV_HIP(launch_mlp_adam(p, g, m, v, n, step, lr, b1, b2, eps, (hipStream_t)stream));
    return SPMV_OK;
}

spmv_status_t spmv_quantize(const double *in, void *out, int64_t n, int32_t to, void *stream) {
    clear_error();
    if (n < 0 || (n > 0 && (!in || !out)) || (to != SPMV_F32 && to != SPMV_BF16))
        return fail(SPMV_ERR_ARG, "bad argument");
    SPMV_HIP(launch_quantize(in, out, n, to, (hipStream_t)stream));
    return SPMV_OK;
}

spmv_status_t spmv_set_xblock_slices(spmv_plan_t P, int32_t slices) {
    clear_error();
    if (!P) return fail(SPMV_ERR_ARG, "NULL plan");
    if (slices != 0 && slices != 1 && slices != 2 && slices != 4 && slices != 8)
        return fail(SPMV_ERR_ARG, "x-block slices must be 0 (automatic), 1, 2, 4 or 8, not %d", slices);
    if (slices == P->xs_req) return SPMV_OK;
    P->xs_req = slices;
    if (P->xs_built && xs_slice_count(P) != P->xs_slices) {
        SPMV_TRY(sync(P));
        P->xs_built = false;
        if (P->variant == V_XBLOCK_LDS) SPMV_TRY(build_xslices(P));  // else on next use
    }
    return SPMV_OK;
}

// Drops every delta16 array so that the next use builds the format again.
static void release_d16(spmv_plan *P) {
    P->d16_layout = -1;
    P->d16_built = false;
    P->srow_coded_built = false;
    P->d16_off.release();
    P->d16s_width.release();
    P->d16s_units.release();
    P->d16s_base.release();
    P->d16s_off.release();
    P->d16s_val.release();
    P->d16s_kind.release();
    P->d16s_diag.release();
    P->d16s_span.release();
    P->d16s_mask.release();
    P->d16s_esc.release();
    P->d16s_eunits.release();
    P->d16s_perm.release();
    P->d16s_pinv.release();
    P->d16_sort = 0;
}

spmv_status_t spmv_set_delta16_layout(spmv_plan_t P, int32_t layout) {
    clear_error();
    if (!P) return fail(SPMV_ERR_ARG, "NULL plan");
    if (layout < -1 || layout > 1)
        return fail(SPMV_ERR_ARG, "delta16 layout must be -1 (automatic), 0 or 1, not %d", layout);
    if (layout == P->d16_layout_req) return SPMV_OK;
    SPMV_TRY(sync(P));
    P->d16_layout_req = layout;
    release_d16(P);
    if (P->variant == V_DELTA16) SPMV_TRY(build_format(P, V_DELTA16));  // else on next use
    return SPMV_OK;
}

spmv_status_t spmv_set_delta16_sort(spmv_plan_t P, int32_t mode) {
    clear_error();
    if (!P) return fail(SPMV_ERR_ARG, "NULL plan");
    if (mode < -1 || mode > 1)
        return fail(SPMV_ERR_ARG, "delta16 row sorting must be -1 (automatic), 0 or 1, not %d", mode);
    if (mode == P->d16_sort_req) return SPMV_OK;
    SPMV_TRY(sync(P));
    P->d16_sort_req = mode;
    release_d16(P);
    if (P->variant == V_DELTA16) SPMV_TRY(build_format(P, V_DELTA16));
    return SPMV_OK;
}

spmv_status_t spmv_set_delta16_offset_bits(spmv_plan_t P, int32_t bits) {
    clear_error();
    if (!P) return fail(SPMV_ERR_ARG, "NULL plan");
    if (bits != 0 && bits != 8 && bits != 16)
        return fail(SPMV_ERR_ARG, "delta16 offset bits must be 0 (automatic), 8 or 16, not %d", bits);
    if (bits == P->d16_offw_req) return SPMV_OK;
    SPMV_TRY(sync(P));
    P->d16_offw_req = bits;
    P->d16_layout = -1;  // decided again, with the new width
    P->d16_built = false;
    P->d16s_off.release();
    P->d16s_val.release();
    P->d16s_mask.release();
    P->d16s_esc.release();
    P->d16s_eunits.release();
    if (P->variant == V_DELTA16) SPMV_TRY(build_format(P, V_DELTA16));  // else on next use
    return SPMV_OK;
}

spmv_status_t spmv_release_cached_blocks(void) {
    clear_error();
    cache_trim(0, true);
    return SPMV_OK;
}

spmv_status_t spmv_cache_flush(void *stream) {
    clear_error();
    return flush_cache((hipStream_t)stream);
}

spmv_status_t spmv_hbm_probe(int64_t bytes, double *read_gbs, double *copy_gbs) {
    clear_error();
    if (bytes < (1 << 20)) return fail(SPMV_ERR_ARG, "buffer too small");
    bytes &= ~(int64_t)4095;
    DevBuf a, b, sink;
    SPMV_TRY(a.alloc((size_t)bytes));
    SPMV_TRY(b.alloc((size_t)bytes));
    SPMV_TRY(sink.alloc(4096 * 8));
    SPMV_HIP(hipMemset(a.p, 1, (size_t)bytes));
    SPMV_HIP(hipMemset(b.p, 0, (size_t)bytes));
    hipEvent_t e0, e1;
    SPMV_HIP(hipEventCreate(&e0));
    SPMV_HIP(hipEventCreate(&e1));
    std::vector<double> tr, tc;
    for (int r = 0; r < 6; ++r) {
        float ms;
        SPMV_HIP(hipEventRecord(e0, nullptr));
        SPMV_HIP(launch_read_probe(a.p, (size_t)bytes, sink.as<double>(), nullptr));
        SPMV_HIP(hipEventRecord(e1, nullptr));
        SPMV_HIP(hipEventSynchronize(e1));
        SPMV_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (r) tr.push_back(ms * 1e-3);
        SPMV_HIP(hipEventRecord(e0, nullptr));
        SPMV_HIP(launch_copy_probe(a.p, b.p, (size_t)bytes, nullptr));
        SPMV_HIP(hipEventRecord(e1, nullptr));
        SPMV_HIP(hipEventSynchronize(e1));
        SPMV_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (r) tc.push_back(ms * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (read_gbs) *read_gbs = (double)bytes / median(tr) * 1e-9;
    if (copy_gbs) *copy_gbs = 2.0 * (double)bytes / median(tc) * 1e-9;
    return SPMV_OK;
}

spmv_status_t spmv_gather_probe(int64_t window_elems, int32_t elem_bytes, int32_t windows,
                                int64_t gathers, double *t_median_s) {
    return spmv_gather_probe2(window_elems, elem_bytes, windows, gathers, 0, t_median_s);
}

spmv_status_t spmv_gather_probe2(int64_t window_elems, int32_t elem_bytes, int32_t windows,
                                 int64_t gathers, int32_t indexed, double *t_median_s) {
    clear_error();
    if (!t_median_s) return fail(SPMV_ERR_ARG, "NULL argument");
    if (elem_bytes != 4 && elem_bytes != 8) return fail(SPMV_ERR_ARG, "elem_bytes must be 4 or 8");
    if (windows != 1 && windows != 2 && windows != 4 && windows != 8)
        return fail(SPMV_ERR_ARG, "windows must be 1, 2, 4 or 8");
    if (window_elems < 1 || window_elems > UINT32_MAX ||
        window_elems * elem_bytes * windows > (int64_t)kFlushBytes)
        return fail(SPMV_ERR_ARG, "the windows must fit the %lld-byte probe buffer",
                    (long long)kFlushBytes);
    if (gathers < 8 || gathers > ((int64_t)1 << 34)) return fail(SPMV_ERR_ARG, "gathers out of range");
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    DevBuf *b;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_flush.find(dev);
        if (it == g_flush.end()) it = g_flush.emplace(dev, new DevBuf()).first;
        b = it->second;
        if (!b->p) {
            SPMV_TRY(b->alloc(kFlushBytes + kFlushSink));
            SPMV_HIP(hipMemset(b->p, 0, kFlushBytes + kFlushSink));
        }
    }
    DevBuf sink, col, val;
    SPMV_TRY(sink.alloc((size_t)((gathers + 2047) / 2048 + 1) * 8));
    if (indexed) {  // the streamed columns and values of the indexed form
        SPMV_TRY(col.alloc((size_t)gathers * 4));
        SPMV_TRY(val.alloc((size_t)gathers * elem_bytes));
        SPMV_HIP(launch_fill_cols(col.as<int32_t>(), gathers, window_elems, nullptr));
        SPMV_HIP(hipMemsetAsync(val.p, 0, (size_t)gathers * elem_bytes, nullptr));
    }
    hipEvent_t e0, e1;
    SPMV_HIP(hipEventCreate(&e0));
    SPMV_HIP(hipEventCreate(&e1));
    std::vector<double> t;
    spmv_status_t st = SPMV_OK;
    for (int r = 0; r < 7 && st == SPMV_OK; ++r) {
        float ms = 0.f;
        hipError_t e = hipEventRecord(e0, nullptr);
        if (e == hipSuccess)
            e = indexed ? launch_indexed_probe(col.as<int32_t>(), val.p, b->p, window_elems, elem_bytes,
                                               windows, gathers, sink.as<unsigned long long>(), nullptr)
                        : launch_gather_probe(b->p, window_elems, elem_bytes, windows, gathers,
                                              sink.as<unsigned long long>(), nullptr);
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) st = fail_hip(e, "gather probe", __FILE__, __LINE__);
        else if (r >= 2) t.push_back(ms * 1e-3);  // two warm-ups
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    SPMV_TRY(st);
    *t_median_s = median(t);
    return SPMV_OK;
}

spmv_status_t spmv_generate(int32_t family, const int64_t *params, int32_t n_params, uint64_t seed,
                            int32_t *d_rowptr, int32_t *d_colind, double *d_val, int64_t *nnz_out,
                            void *stream) {
    clear_error();
    static const int need[9] = {2, 2, 2, 2, 3, 3, 2, 4, 1};
    if (family < 0 || family > 8) return fail(SPMV_ERR_ARG, "unknown family %d", family);
    if (!params || n_params < need[family] || n_params > 6 || !d_rowptr)
        return fail(SPMV_ERR_ARG, "bad generator arguments");
    int64_t p[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < n_params; ++i) p[i] = params[i];
    for (int i = 0; i < need[family]; ++i)
        if (p[i] < 0) return fail(SPMV_ERR_ARG, "negative generator parameter");
    int64_t n;
    if (family <= 1) n = p[0] * p[0];
    else if (family <= 3) n = p[0] * p[0] * p[0];
    else n = p[0];
    if (p[0] > (1 << 24) * 128ll || n >= INT32_MAX) return fail(SPMV_ERR_ARG, "too many rows");
    if (family == 4 && (p[1] < 1 || p[1] >= INT32_MAX)) return fail(SPMV_ERR_ARG, "bad column count");
    if ((family == 5 || family == 6) && (p[1] < 1 || p[1] > (1 << 20)))
        return fail(SPMV_ERR_ARG, "d16 out of range");
    if (family == 7 && (p[1] < 1 || p[1] >= (1 << 16) || p[2] < 1 || p[2] >= (1 << 21)))
        return fail(SPMV_ERR_ARG, "power-law parameters out of range");
    hipStream_t s = (hipStream_t)stream;
    if (!d_colind) {
        DevBuf lens, tmp;
        size_t need_tmp = 0;
        SPMV_TRY(lens.alloc((size_t)(n > 0 ? n : 1) * 4));
        SPMV_HIP(launch_gen_lengths(family, p, seed, n, lens.as<int32_t>(), s));
        SPMV_HIP(launch_exclusive_scan_i32(lens.as<int32_t>(), d_rowptr, n, 1, nullptr, nullptr, 0, s, &need_tmp));
        SPMV_TRY(tmp.alloc(need_tmp));
        SPMV_HIP(launch_exclusive_scan_i32(lens.as<int32_t>(), d_rowptr, n, 1, nullptr, tmp.p, tmp.bytes, s, nullptr));
        int64_t total = 0;
        const int64_t nb = (int64_t)need_tmp / 8 - 1;
        SPMV_HIP(hipMemcpyAsync(&total, tmp.as<int64_t>() + nb, 8, hipMemcpyDeviceToHost, s));
        SPMV_HIP(hipStreamSynchronize(s));
        if (total >= INT32_MAX) return fail(SPMV_ERR_ARG, "generated matrix has %lld >= 2^31 nonzeros", (long long)total);
        if (nnz_out) *nnz_out = total;
        return SPMV_OK;
    }
    if (!d_val) return fail(SPMV_ERR_ARG, "val is NULL");
    SPMV_HIP(launch_gen_fill(family, p, seed, n, d_rowptr, d_colind, d_val, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

spmv_status_t spmv_generate_vector(int64_t n, uint64_t seed, double *d_x, void *stream) {
    clear_error();
    if (n < 0 || (n > 0 && !d_x)) return fail(SPMV_ERR_ARG, "bad argument");
    SPMV_HIP(launch_gen_vector(n, seed, d_x, (hipStream_t)stream));
    return SPMV_OK;
}

}  // extern "C"
