// Internal declarations of libspmvsel (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <type_traits>
#include <utility>
#include <string>
#include <vector>

#include "spmvsel.h"

namespace spmvsel {

// ---------------------------------------------------------------- constants
constexpr int kBlock = 256;           // threads per workgroup for every SpMV kernel
constexpr int kRunLen = 8;            // nonzeros per thread run in the streaming kernels
constexpr int kChunk = kBlock * kRunLen;  // nonzeros staged per LDS chunk
constexpr int kRowStreamMaxR = 8;     // rows per thread (max) in short_row / delta16
constexpr int kMergeIpt = 8;          // merge-path items per thread
constexpr int64_t kMaxNnz = (1ll << 31) - (1ll << 16);  // NNZ below this: int32 index headroom
constexpr int kMergeTile = kBlock * kMergeIpt;
constexpr int kSlices = 8;            // x-block column slices at most (one per XCD)
constexpr int64_t kSliceXEntries = 256ll << 10;  // x entries per slice the automatic count aims at
constexpr int kSliceMinAvg10 = 9;     // ... keeping at least this many tenths of a nonzero per slice row
constexpr int kSliceStreamMaxLen = 128;  // longest slice segment for row streaming
constexpr int kLongChunk = 256;       // nonzeros per block of the long-row sums
constexpr double kLongMaxShare = 0.25;  // long rows leave the slices up to this share of NNZ
constexpr int kKahanMinLen = 257;     // FP32 rows longer than 256 use Kahan sums
constexpr int kSellRows = 64;         // rows per slice of the sliced delta16 layout (one per lane)
constexpr double kSellMaxPad = 1.35;  // ... taken when its slots are at most this many per nonzero,
constexpr double kSellMaxPadLong = 1.6;  // or this many when rows average at least
constexpr int kSellLongMeanX2 = 15;      // 7.5 nonzeros (twice the mean, in integers)
constexpr int kSellMaxSpanLong = 8192;   // and its offset slices span fewer columns
constexpr int kSortMinSaved = 8;         // slots per row that sorting rows by length must save,
constexpr int kSortMinSavedFree = 4;     // or this many where the plain layout stages little x
constexpr int kSellMaxDiag = 32;         // diagonals a diagonal slice can hold (mask bits)
constexpr int kSellXWindow = 512;        // x entries an offset slice can stage in LDS
// An offset slice of width w whose columns lie within kSellXWindow of its
// reference column and whose gathers number at least twice its column span
// reads x from a copy of that window in LDS.
__host__ __device__ inline bool sell_stages_x(int span, int w) {
    return span < kSellXWindow && 2 * (span + 1) <= kSellRows * w;
}
constexpr int kLineBytes = 128;       // cache line assumed by the miss feature
constexpr int64_t kLlcBytes = 256ll << 20;
constexpr int kFeatBlocks = 1024;     // feature kernel partial records
constexpr int kValGrid = 2048;        // validation blocks (one partial each)

// ---------------------------------------------------------------- errors
spmv_status_t fail(spmv_status_t st, const char *fmt, ...);
spmv_status_t fail_hip(hipError_t e, const char *what, const char *file, int line);
void clear_error();

#define SPMV_HIP(expr)                                                          \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) return ::spmvsel::fail_hip(e_, #expr, __FILE__, __LINE__); \
    } while (0)

#define SPMV_TRY(expr)                                                          \
    do {                                                                        \
        spmv_status_t s_ = (expr);                                              \
        if (s_ != SPMV_OK) return s_;                                           \
    } while (0)

// ---------------------------------------------------------------- device buffer
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int dev = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    spmv_status_t alloc(size_t n);        // no-op if already >= n bytes
    void release();
    void swap(DevBuf &o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(dev, o.dev);
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

inline int vbytes(int dtype) { return dtype == SPMV_F64 ? 8 : dtype == SPMV_F32 ? 4 : 2; }
inline int xbytes(int dtype) { return dtype == SPMV_F64 ? 8 : 4; }

// ---------------------------------------------------------------- plan
struct SliceOffsets {  // first nonzero of each column slice in the slice-major arrays
    int64_t off[kSlices];
};

}  // namespace spmvsel

struct spmv_plan {
    int64_t n = 0, m = 0, nnz = 0;
    const int32_t *rowptr = nullptr;
    const int32_t *colind = nullptr;
    const void *val = nullptr;
    int dtype = SPMV_F64;
    hipStream_t stream = nullptr;
    bool other_streams = false;  // spmv_execute ran on a stream other than `stream`
    uint32_t flags = 0;
    int device = 0;
    int num_cus = 256;
    int variant = V_CSR_SCALAR;
    // FP32/BF16 plans: rows of at least this many nonzeros use Kahan sums
    // (INT32_MAX: no compensation anywhere, for measuring what it buys)
    int kahan_min = spmvsel::kKahanMinLen;

    spmvsel::DevBuf own_rowptr, own_colind, own_val;  // SPMV_COPY_INPUTS
    spmvsel::DevBuf scratch;     // small: flags, feature partials, records
    void *h_pinned = nullptr;    // pinned host staging (4 KiB)

    // features
    bool have_features = false;
    double feats[12] = {0};
    uint64_t acc[12] = {0};

    // launch parameters
    int vec_width = 2;           // csr_vector sub-wave width
    int rs_rows = 1;             // rows per thread in the streaming kernels
    int parts = 2048;            // profiling partitions

    // derived formats (lazy)
    bool d16_checked = false, d16_feasible = false, d16_built = false;
    // d16_base holds the block references at d16_rows (the one-pass
    // selection takes only the spans; the references follow at preparation)
    bool d16_base_ready = false;
    void *h_pinned_dev = nullptr;  // h_pinned's device address
    int d16_rows = 256;          // rows per block sharing one reference column
    spmvsel::DevBuf d16_base, d16_off, d16_cmax;
    // delta16 layout: 0 rows streamed (d16_base/d16_off), 1 sliced (64-row
    // slices stored column-major in pairs, one reference column per slice)
    int d16_layout = -1;         // -1: not decided yet
    int d16_layout_req = -1;     // forced layout, -1 automatic
    // bits per column code in the sliced layout's offset slices (one width
    // per matrix): 16 = offsets from the slice's reference column, 8 = deltas
    // from the row's previous column with an escape code (255) for a gap
    // that does not fit, the escaped column stored in d16s_esc
    int d16_offw = 16;
    int d16_offw_req = 0;        // forced width, 0 automatic
    int64_t d16_span = 0;        // largest column span of an offset slice
    int64_t d16_esc_units = 0, d16_nesc = 0;  // sum of per-slice max escapes; escapes
    spmvsel::DevBuf d16s_eunits, d16s_esc;    // per slice: first escape unit; escapes
    int64_t d16_nsl = 0, d16_slots = 0;
    int64_t d16_nnz_off = 0, d16_ndiag = 0;  // nonzeros of offset slices; diagonal slices
    spmvsel::DevBuf d16s_width, d16s_units, d16s_base, d16s_off, d16s_val;
    // per slice: 0 for an offset slice, 1 + D for a diagonal slice of D
    // diagonals (listed in d16s_diag[32 s .. 32 s + D)); one mask per row
    spmvsel::DevBuf d16s_kind, d16s_diag, d16s_mask, d16s_nnz;
    spmvsel::DevBuf d16s_span;  // per slice: largest offset from its reference column
    // length-sorted sliced layout: the row at each position (perm) and the
    // position of each row (pinv, until the layout is built); requested
    // -1 automatic, 0 plain, 1 sorted
    spmvsel::DevBuf d16s_perm, d16s_pinv;
    int d16_sort_req = -1, d16_sort = 0;
    bool mp_built = false;
    int64_t mp_tiles = 0;
    spmvsel::DevBuf mp_split_row, mp_split_nnz, mp_carry_row, mp_carry_val;
    bool xs_built = false;       // x blocking: column slices (slice s on XCDs s, s+S, ...)
    int xs_req = 0;              // requested slice count (0: from the size of x)
    int xs_slices = 0;           // slice count S of the built format (1, 2, 4 or 8)
    int64_t xs_width = 0;        // columns per slice
    int xs_rows = 0;             // >0: row-streaming per slice with this block height; 0: merge path
    int64_t xs_nnz_off[spmvsel::kSlices] = {0}, xs_tiles[spmvsel::kSlices] = {0},
            xs_tile_off[spmvsel::kSlices] = {0};
    spmvsel::DevBuf xs_rowptr, xs_colind, xs_val, xs_srow, xs_snnz, xs_crow, xs_cval, xs_y;
    // rows with a slice segment longer than kSliceStreamMaxLen, taken out of
    // the slices and summed from the original CSR in chunks of kLongChunk
    // inside one column slice each; xs_lcmap gives the chunk of each chunk
    // workgroup of the slice kernel (-1: none), xs_nslots of them
    int64_t xs_nlong = 0, xs_nchunks = 0, xs_long_nnz = 0, xs_nslots = 0;
    spmvsel::DevBuf xs_lrows, xs_lfirst, xs_lck0, xs_lck1, xs_lsum, xs_lcmap;
    spmvsel::DevBuf xs_lmask;    // one bit per row: set for the long rows
    // phased row streaming (no partial y): row blocks per workgroup and
    // workgroups; 0 when the slices use the partial-y kernels
    int xs_pj = 0;
    int64_t xs_pg = 0;
    bool part_built = false;
    spmvsel::DevBuf part_bounds;

    // index coding (spmv_set_index_coding): -1 each variant's own (DELTA16
    // coded, the rest int32), 0 int32 column indices, 1 16-bit column codes
    int idx_req = -1;
    // 1 if variant v reads 16-bit column codes under the current request
    int code_of(int v) const { return v == V_DELTA16 ? 1 : (idx_req == 1 ? 1 : 0); }
    // coded merge path: per tile its smallest column (mpc_base) and 16-bit
    // offsets from it (mpc_off), feasible when every tile spans < 65536
    bool mpc_checked = false, mpc_feasible = false, mpc_built = false;
    int32_t mpc_span = 0;
    spmvsel::DevBuf mpc_base, mpc_off;
    // coded x blocking: per slice and row block of xsc_h rows (the slice
    // kernel's block) its smallest column (xsc_base from xsc_boff[s]) and
    // 16-bit offsets at the positions of the slice-major columns (xsc_off)
    bool xsc_checked = false, xsc_feasible = false, xsc_built = false;
    int32_t xsc_span = 0;
    int64_t xsc_h = 0, xsc_boff[spmvsel::kSlices + 1] = {0};
    spmvsel::DevBuf xsc_base, xsc_off;
    // SHORT_ROW with codes runs the rows-streamed delta16 kernel on these
    bool srow_coded_built = false;

    // timing helpers (lazy)
    spmvsel::DevBuf tx, ty;      // x and y used by spmv_time_variant / profiling
};

namespace spmvsel {

// ---------------------------------------------------------------- launchers
// validation (k_validate.hip): writes flags[0] (bit0 rowptr, bit1 col range),
// counts[1] = descending pairs, counts[2] = descending pairs at row starts
// d_part: kValGrid * 3 u64 of device scratch for per-block partials
// One SpMV y = A x with variant v on stream s (SPMV_ERR_ARG if v's format is
// not built).
spmv_status_t run_variant(const spmv_plan *P, int v, const void *x, void *y, hipStream_t s);
// Table 2 on the GPU: the variant for bottleneck class k (K_CML ... K_CMP).
int class_variant(int k, const double feats[12], const double th[4], uint32_t feas);
// Device inference of the CART (which 0) or naive Bayes (1) selector; d_out
// needs 80 bytes of device memory.  SPMV_ERR_NO_MODEL if none is loaded.
// One-pass selection with a classifier (0 tree, 1 naive Bayes): whether a
// model is loaded; launching its selection kernel on the partials of the
// selection pass (the record of kSelectRecordBytes at out: int32 label,
// leaf, fallback, then the common part at the MLP's offsets); label_kind
// tells how to read the label (0 variant, 1 bottleneck class).
bool classic_loaded(int which);
spmv_status_t classic_select_launch(int which, const uint64_t *d_partials, int nparts, int64_t n,
                                    int64_t m, int64_t nnz, int vb, int xb, int two_heights,
                                    uint32_t feas_base, void *out, hipStream_t s,
                                    int *label_kind);
spmv_status_t classic_predict(int which, const double f[12], uint32_t feas, const double th[4],
                              hipStream_t s, void *d_out, int32_t *variant, int32_t *label,
                              int32_t *fallback);
hipError_t launch_validate(const spmv_plan &P, uint64_t *d_flags, uint64_t *d_part,
                           hipStream_t s);

// features (k_features.hip): final record -> d_rec (16 words)
hipError_t launch_features(const spmv_plan &P, uint64_t *d_partials, uint64_t *d_rec,
                           int xb, hipStream_t s);

// SpMV variants (k_spmv.hip)
hipError_t launch_csr_scalar(const spmv_plan &P, const void *x, void *y, hipStream_t s);
hipError_t launch_csr_vector(const spmv_plan &P, const void *x, void *y, hipStream_t s);
hipError_t launch_rowstream(const spmv_plan &P, bool d16, const void *x, void *y, hipStream_t s);
hipError_t launch_sliced_d16(const spmv_plan &P, const void *x, void *y, hipStream_t s);
hipError_t phased_geometry(const spmv_plan &P, int *blocks_per_group, int64_t *groups);
hipError_t launch_merge_path(const spmv_plan &P, const void *x, void *y, hipStream_t s);
// merge path on explicit buffers: splits srow/snnz [tiles + 1], carries
// crow [tiles] and cval [tiles] of the accumulation type (tiles =
// ceil((n + nnz) / kMergeTile)); every carry is written before it is read
hipError_t launch_merge_path_raw(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                                 const void *val, int dtype, const void *x, void *y,
                                 const int32_t *srow, const int32_t *snnz, int32_t *crow,
                                 void *cval, int kmin, hipStream_t s,
                                 const uint16_t *off = nullptr, const int32_t *tbase = nullptr);
hipError_t launch_xblock(const spmv_plan &P, const void *x, void *y, hipStream_t s);

// format preparation (k_prep.hip)
hipError_t launch_delta16_encode(const spmv_plan &P, const int32_t *base, uint16_t *off,
                                 hipStream_t s);
// Sliced delta16 layout: per slice of kSellRows rows its width (longest row
// rounded up to even), half width and reference column (smallest column);
// then, with the scanned half widths (units of 128 slots), the scatter of
// offsets and values into the zero-filled slot arrays.
// Diagonal slices: a slice whose rows' values of c - r, D distinct ones, fit
// kSellMaxDiag and, rounded up to even, its offset width, lists them in
// diag[32 s ..] (kind = 1 + D) and sets bit k of a row's mask for each
// diagonal k the row has; its positions follow the diagonals, not the row.
hipError_t launch_sliced_shape(const spmv_plan &P, const int32_t *perm, int32_t *width,
                               int32_t *halfw, int32_t *base, int32_t *kind, int32_t *diag,
                               int32_t *snnz, int32_t *span, hipStream_t s);
// the row order of the length-sorted sliced layout (windows of kBlock rows)
hipError_t launch_sell_perm(const spmv_plan &P, int32_t *perm, int32_t *pinv, hipStream_t s);
// values, masks, and the 16-bit offsets or the 8-bit codes (off or codes
// null: not written)
hipError_t launch_sliced_scatter(const spmv_plan &P, const int32_t *units, const int32_t *base,
                                 const int32_t *kind, const int32_t *diag, uint16_t *off,
                                 uint8_t *codes, void *vals, uint32_t *mask, hipStream_t s);
// per offset slice: the most escapes of one of its rows (E) and their sum
hipError_t launch_sliced_escapes(const spmv_plan &P, const int32_t *base, const int32_t *kind,
                                 int32_t *E, int32_t *nesc, hipStream_t s);
// the escaped columns of the 8-bit codes (eunits: S + 1 prefix sums of E)
hipError_t launch_sliced_escape_cols(const spmv_plan &P, const int32_t *base, const int32_t *kind,
                                    const int32_t *eunits, int32_t *esc, hipStream_t s);
// 16-bit codes over ranges of a column array: range k covers positions
// [bnd[min(k H, nb)], bnd[min((k + 1) H, nb)]); base[k] = its smallest
// column (0 if empty), span[k] = largest - smallest; then off = ci - base
hipError_t launch_range_ref(int64_t nranges, int64_t nb, int64_t H, const int32_t *bnd,
                            const int32_t *ci, int32_t *base, int32_t *span, hipStream_t s);
hipError_t launch_range_encode(int64_t nranges, int64_t nb, int64_t H, const int32_t *bnd,
                               const int32_t *ci, const int32_t *base, uint16_t *off, hipStream_t s);
hipError_t launch_max_span(const int32_t *cmin, const int32_t *cmax, int64_t panels,
                           unsigned long long *d_max, hipStream_t s);
hipError_t launch_merge_splits(const int32_t *rowptr, int64_t n, int64_t nnz, int32_t *srow,
                               int32_t *snnz, int64_t tiles, hipStream_t s);
// Long rows of the x-block split: flags[i] = 1 if a slice segment of row i
// exceeds kSliceStreamMaxLen; then, from the scanned flags, the row list with
// its [start, end) nonzero range.
hipError_t launch_long_flags(int64_t n, int ns, const int32_t *lens, int32_t *flags, hipStream_t s);
hipError_t launch_long_compact(int64_t n, const int32_t *flags, const int32_t *pos,
                               const int32_t *rp, int32_t *rows, int32_t *beg, int32_t *end,
                               hipStream_t s);
hipError_t launch_long_bounds(int64_t L, int ns, int64_t cw, const int32_t *ci, const int32_t *beg,
                              const int32_t *end, int32_t *bounds, hipStream_t s);
hipError_t launch_long_zero(int64_t L, int ns, int64_t n, const int32_t *rows, int32_t *lens,
                            hipStream_t s);
// mask[w] bit b = flags[32 w + b] != 0
hipError_t launch_long_mask(int64_t n, const int32_t *flags, uint32_t *mask, hipStream_t s);
hipError_t launch_slice_count(const spmv_plan &P, int64_t cw, const int32_t *srow,
                              const int32_t *snnz, int64_t tiles, int32_t *lens, hipStream_t s);
// d_part: 2048 int32 of device scratch for per-block maxima
hipError_t launch_max_i32(const int32_t *a, int64_t n, int32_t *d_part,
                          unsigned long long *d_max, hipStream_t s);
hipError_t launch_slice_scatter(const spmv_plan &P, const int32_t *srow, const int32_t *snnz,
                                int64_t tiles, const int32_t *srp, const SliceOffsets &so,
                                int32_t *xci, void *xval, hipStream_t s);
hipError_t launch_panel_windows(const spmv_plan &P, int rows_per_panel, int32_t *cmin,
                                int32_t *cmax, int64_t panels, hipStream_t s);
hipError_t launch_partition(const int32_t *rowptr, int64_t n, int parts, int32_t *bounds,
                            hipStream_t s);
hipError_t launch_widen(const int32_t *in, int64_t *out, int64_t n, hipStream_t s);
hipError_t launch_row_columns(const spmv_plan &P, int32_t *out, hipStream_t s);
hipError_t launch_quantize(const double *in, void *out, int64_t n, int to, hipStream_t s);

// profiling micro-benchmarks (k_profile.hip)
hipError_t launch_csr_part(const spmv_plan &P, const int32_t *bounds, const int32_t *rp32,
                           const int32_t *ci32, const int64_t *rp64, const int64_t *ci64,
                           const void *x, void *y, unsigned long long *stamps, hipStream_t s);

// MLP (k_mlp.hip)
hipError_t launch_mlp_infer(const float *d_params, const float *d_norm, const double *feats,
                            uint32_t feasible, float tau, float *d_out, hipStream_t s);
// One-pass MLP selection: k_select_pass<R> (feature sums and the largest
// delta16 block spans at heights 256 R and 256 into the partial records at
// d_partials; returns the partial count, 0 on a bad R),
// then k_mlp_select (reduction, device finalisation of the features,
// feasibility, network and decision in one workgroup).  out:
// kSelectRecordBytes (the inference record in floats 0..31, feasibility bits
// at byte 128, features as doubles from byte 192, the reduced record as 16
// words from byte 288, with the spans in its words 12 and 13).
constexpr size_t kSelectRecordBytes = 416;
int launch_select_pass(const spmv_plan &P, int R, uint64_t *d_partials, int xb, hipStream_t s,
                       hipError_t *err);
hipError_t launch_mlp_select(const float *d_params, const float *d_norm, const uint64_t *d_partials,
                             int nparts, int64_t n, int64_t m, int64_t nnz, int vb, int xb,
                             int two_heights, uint32_t feas_base, float tau, float *out,
                             hipStream_t s);
hipError_t launch_mlp_fwd_bwd(const float *params, const float *Z, const int32_t *labels,
                              const uint8_t *accept, const uint8_t *mask, int B, float *grads,
                              float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *p, const float *g, float *m, float *v, int n, int step,
                           float lr, float b1, float b2, float eps, hipStream_t s);

// generator and utilities (k_gen.hip, k_util.hip)
hipError_t launch_gen_lengths(int family, const int64_t *prm, uint64_t seed, int64_t n,
                              int32_t *lens, hipStream_t s);
hipError_t launch_gen_fill(int family, const int64_t *prm, uint64_t seed, int64_t n,
                           const int32_t *rowptr, int32_t *colind, double *val, hipStream_t s);
hipError_t launch_gen_vector(int64_t n, uint64_t seed, double *x, hipStream_t s);
hipError_t launch_exclusive_scan_i32(const int32_t *lens, int32_t *rowptr, int64_t n, int segs,
                                     int64_t *totals, void *tmp, size_t tmp_bytes, hipStream_t s,
                                     size_t *tmp_needed);
// reads buf[0, bytes) (evicting the caches); 256 sink bytes must follow it
hipError_t launch_flush(void *buf, size_t bytes, hipStream_t s);
hipError_t launch_read_probe(const void *buf, size_t bytes, double *sink, hipStream_t s);
hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t s);
// random gathers from ns windows of w elements (elem_bytes 4 or 8); sink
// needs ceil(gathers / 2048) words
hipError_t launch_gather_probe(const void *buf, int64_t w, int elem_bytes, int ns,
                               int64_t gathers, unsigned long long *sink, hipStream_t s);
// the indexed form: stream col[nnz] and val[nnz], gather from the windows
hipError_t launch_fill_cols(int32_t *col, int64_t nnz, int64_t w, hipStream_t s);
hipError_t launch_indexed_probe(const int32_t *col, const void *val, const void *buf, int64_t w,
                                int elem_bytes, int ns, int64_t nnz, unsigned long long *sink,
                                hipStream_t s);

}  // namespace spmvsel
