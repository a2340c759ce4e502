// y = A x by the merge-path variant without a plan and without allocating:
// the merge-path splits and the per-tile carries live in a file-scope
// device array instead of plan-owned buffers.  For callers that cannot call
// hipMalloc (code under HIP graph capture, tight serving loops, harnesses
// that forbid allocation).  The kernels are the plan path's merge-path
// kernels; only where their scratch lives differs.
#include <mutex>

#include "internal.h"

namespace spmvsel {

// Room for the splits (2 x (tiles + 1) int32) and the carries (tiles int32
// rows and tiles values of up to 8 bytes) of up to kNoAllocMaxTiles tiles.
constexpr int64_t kNoAllocScratchBytes = 8ll << 20;
constexpr int64_t kNoAllocMaxTiles = (kNoAllocScratchBytes - 1024) / 20;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code this name is
// a host-side stand-in for the symbol, not a device address: kernels get the
// address from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_noalloc_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

// The scratch array's device address on the current device, looked up once
// per device with that device current.
static spmv_status_t noalloc_scratch(void **out) {
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SPMV_ERR_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        SPMV_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(SPMV_ERR_HIP, "hipGetSymbolAddress returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SPMV_OK;
}

}  // namespace spmvsel

using namespace spmvsel;

extern "C" spmv_status_t spmv_merge_path_noalloc(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                                 const int32_t *d_rowptr, const int32_t *d_colind,
                                                 const void *d_val, int32_t val_dtype,
                                                 const void *d_x, void *d_y, void *stream) {
    clear_error();
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(SPMV_ERR_ARG, "negative size");
    if (n_rows >= INT32_MAX || n_cols >= INT32_MAX || nnz >= kMaxNnz)
        return fail(SPMV_ERR_ARG, "size beyond the int32 index limits");
    if (val_dtype != SPMV_F64 && val_dtype != SPMV_F32 && val_dtype != SPMV_BF16)
        return fail(SPMV_ERR_ARG, "unknown value dtype %d", val_dtype);
    const int64_t tiles = (n_rows + nnz + kMergeTile - 1) / kMergeTile;
    if (tiles > kNoAllocMaxTiles)
        return fail(SPMV_ERR_ARG,
                    "N + NNZ = %lld exceeds the allocation-free limit of %lld items "
                    "(a %lld-byte static scratch array)",
                    (long long)(n_rows + nnz), (long long)(kNoAllocMaxTiles * kMergeTile),
                    (long long)kNoAllocScratchBytes);
    if (n_rows == 0) return SPMV_OK;
    if (!d_rowptr || !d_y || (nnz > 0 && (!d_colind || !d_val || !d_x)))
        return fail(SPMV_ERR_ARG, "NULL array");
    void *base = nullptr;
    SPMV_TRY(noalloc_scratch(&base));
    // layout: carry values (8-byte aligned) | split rows | split nonzeros | carry rows
    char *p = static_cast<char *>(base);
    void *cval = p;
    int32_t *srow = reinterpret_cast<int32_t *>(p + 8 * tiles);
    int32_t *snnz = srow + (tiles + 1);
    int32_t *crow = snnz + (tiles + 1);
    const hipStream_t s = (hipStream_t)stream;
    SPMV_HIP(launch_merge_splits(d_rowptr, n_rows, nnz, srow, snnz, tiles, s));
    SPMV_HIP(launch_merge_path_raw(n_rows, nnz, d_rowptr, d_colind, d_val, val_dtype, d_x, d_y,
                                   srow, snnz, crow, cval, kKahanMinLen, s));
    return SPMV_OK;
}
