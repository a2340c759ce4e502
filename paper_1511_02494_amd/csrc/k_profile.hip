// Micro-benchmarks of the profiling-based classifier (Section 3.2.1).
//
// Baseline CSR under the paper's default partitioning: a static set of
// contiguous row ranges with equal nonzeros, one range per wavefront (the
// GPU's independent instruction stream, the analogue of a CPU thread).  The
// wavefront walks its range with a sub-wavefront of W lanes per row (W from
// the mean row length, as csr_vector).  The same kernel runs the `noxmiss`
// benchmark (every column index of row i replaced by i mod M, which removes
// the irregular x accesses: the paper's all-zero indices would make every
// lane of every wavefront read one cache line on a GPU) and the `inflate`
// benchmark (64-bit row pointers and column indices).  Each wavefront stamps the device
// real-time clock at its start and end for the `balance` benchmark.
#include "dev.h"
#include "internal.h"

namespace spmvsel {

template <class V, class I, int W>
__global__ __launch_bounds__(kBlock) void k_csr_part(const int32_t *__restrict__ bounds,
                                                     const I *__restrict__ rp,
                                                     const I *__restrict__ ci,
                                                     const V *__restrict__ val,
                                                     const typename VT<V>::A *__restrict__ x,
                                                     typename VT<V>::A *__restrict__ y,
                                                     unsigned long long *__restrict__ stamps) {
    using A = typename VT<V>::A;
    const int64_t w = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int sub = lane / W, sl = lane & (W - 1);
    const unsigned long long t0 = wall_clock64();
    const int64_t b0 = bounds[w], b1 = bounds[w + 1];
    for (int64_t i = b0 + sub; i < b1; i += 64 / W) {
        const I a = rp[i], b = rp[i + 1];
        const bool comp = is_f32<A>() && (int64_t)(b - a) >= kKahanMinLen;
        Sum<A> s;
        for (I k = a + sl; k < b; k += W) s.add(VT<V>::cvt(val[k]) * x[ci[k]], comp);
        const A t = group_sum<W>(s.s);
        if (sl == 0) y[i] = t;
    }
    const unsigned long long t1 = wall_clock64();
    if (lane == 0) {
        stamps[2 * w] = t0;
        stamps[2 * w + 1] = t1;
    }
}

hipError_t launch_csr_part(const spmv_plan &P, const int32_t *bounds, const int32_t *rp32,
                           const int32_t *ci32, const int64_t *rp64, const int64_t *ci64,
                           const void *x, void *y, unsigned long long *stamps, hipStream_t s) {
    const unsigned g = (unsigned)((P.parts * 64 + kBlock - 1) / kBlock);
    auto go = [&](auto vtag) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(vtag)>>;
        using A = typename VT<V>::A;
#define PART(WW)                                                                                 \
    case WW:                                                                                     \
        if (rp64)                                                                                \
            hipLaunchKernelGGL((k_csr_part<V, int64_t, WW>), dim3(g), dim3(kBlock), 0, s, bounds, \
                               rp64, ci64, (const V *)P.val, (const A *)x, (A *)y, stamps);      \
        else                                                                                     \
            hipLaunchKernelGGL((k_csr_part<V, int32_t, WW>), dim3(g), dim3(kBlock), 0, s, bounds, \
                               rp32, ci32, (const V *)P.val, (const A *)x, (A *)y, stamps);      \
        break;
        switch (P.vec_width) {
            PART(2) PART(4) PART(8) PART(16) PART(32) PART(64)
        default: return hipErrorInvalidValue;
        }
#undef PART
        return hipGetLastError();
    };
    switch (P.dtype) {
    case SPMV_F64: return go((const double *)nullptr);
    case SPMV_F32: return go((const float *)nullptr);
    default: return go((const uint16_t *)nullptr);
    }
}

}  // namespace spmvsel
