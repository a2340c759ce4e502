// Conjugate gradients (Hestenes and Stiefel 1952) on a plan's matrix with its
// selected SpMV variant: the solver loop whose SpMVs repay the selection.
//
//   r = b - A x;  p = r;  rr = r.r
//   repeat: q = A p;  alpha = rr / p.q;  x += alpha p;  r -= alpha q;
//           rr' = r.r;  stop when sqrt(rr') <= rtol ||b|| or after max_iters;
//           p = r + (rr' / rr) p;  rr = rr'
//
// Dot products are two-stage (per-block tree sums over a fixed grid, then one
// block folds the partials in a fixed order), so a solve is deterministic.
// The scalars live in device memory; rr alternates between two slots so no
// kernel reads a value another kernel of the same iteration writes.
#include <math.h>

#include "dev.h"
#include "internal.h"

namespace spmvsel {
namespace {

constexpr int kDotGrid = 1024;
enum { SC_RR0 = 0, SC_RR1 = 1, SC_PQ = 2, SC_BB = 3 };

__device__ inline void block_sum_to(double v, double *part) {
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_dot_part(int64_t n, const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ part) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        s = s + a[i] * b[i];
    block_sum_to(s, part);
}

__global__ __launch_bounds__(kBlock) void k_dot_final(const double *__restrict__ part, int np,
                                                      double *__restrict__ out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += kBlock) s = s + part[i];
    block_sum_to(s, out);  // one block: writes out[0]
}

// r = b - q; p = r; partial sums of r.r
__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t n, const double *__restrict__ b,
                                                    const double *__restrict__ q,
                                                    double *__restrict__ r, double *__restrict__ p,
                                                    double *__restrict__ part) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double ri = b[i] - q[i];
        r[i] = ri;
        p[i] = ri;
        s = s + ri * ri;
    }
    block_sum_to(s, part);
}

// x += alpha p; r -= alpha q with alpha = sc[rr] / sc[PQ]; partial sums of r.r
__global__ __launch_bounds__(kBlock) void k_cg_xr(int64_t n, double *__restrict__ x,
                                                  double *__restrict__ r,
                                                  const double *__restrict__ p,
                                                  const double *__restrict__ q,
                                                  const double *__restrict__ sc, int rr,
                                                  double *__restrict__ part) {
    const double alpha = sc[rr] / sc[SC_PQ];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        x[i] = x[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        s = s + ri * ri;
    }
    block_sum_to(s, part);
}

// p = r + beta p with beta = sc[rr_new] / sc[rr_old]
__global__ __launch_bounds__(kBlock) void k_cg_p(int64_t n, double *__restrict__ p,
                                                 const double *__restrict__ r,
                                                 const double *__restrict__ sc, int rr_new,
                                                 int rr_old) {
    const double beta = sc[rr_new] / sc[rr_old];
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = r[i] + beta * p[i];
}

}  // namespace
}  // namespace spmvsel

using namespace spmvsel;

extern "C" spmv_status_t spmv_cg(spmv_plan_t P, const double *d_b, double *d_x, int32_t max_iters,
                                 double rtol, void *stream, int32_t *iters, double *rel_resid) {
    clear_error();
    if (!P || !d_b || !d_x) return fail(SPMV_ERR_ARG, "NULL argument");
    if (P->dtype != SPMV_F64) return fail(SPMV_ERR_ARG, "CG needs an FP64 plan");
    if (P->n != P->m) return fail(SPMV_ERR_ARG, "CG needs a square matrix");
    if (max_iters < 0 || !(rtol >= 0.0)) return fail(SPMV_ERR_ARG, "bad max_iters or rtol");
    hipStream_t s = (hipStream_t)stream;
    if (s != P->stream) P->other_streams = true;  // destroy then waits for the device
    const int64_t n = P->n;
    if (iters) *iters = 0;
    if (rel_resid) *rel_resid = 0.0;
    if (n == 0) return SPMV_OK;
    DevBuf r, p, q, part, sc;
    SPMV_TRY(r.alloc((size_t)n * 8));
    SPMV_TRY(p.alloc((size_t)n * 8));
    SPMV_TRY(q.alloc((size_t)n * 8));
    SPMV_TRY(part.alloc(kDotGrid * 8));
    SPMV_TRY(sc.alloc(8 * 8));
    int64_t gb = (n + kBlock - 1) / kBlock;
    const unsigned g = (unsigned)(gb < kDotGrid ? gb : kDotGrid);
    double *dsc = sc.as<double>(), *dpart = part.as<double>();
    double *h = static_cast<double *>(P->h_pinned);
    auto dot_final = [&](int slot) -> hipError_t {
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, s, dpart, (int)g, dsc + slot);
        return hipGetLastError();
    };
    auto read = [&](int slot, double *v) -> spmv_status_t {
        SPMV_HIP(hipMemcpyAsync(h, dsc + slot, 8, hipMemcpyDeviceToHost, s));
        SPMV_HIP(hipStreamSynchronize(s));
        *v = h[0];
        return SPMV_OK;
    };
    // ||b||
    hipLaunchKernelGGL(k_dot_part, dim3(g), dim3(kBlock), 0, s, n, d_b, d_b, dpart);
    SPMV_HIP(dot_final(SC_BB));
    double bb;
    SPMV_TRY(read(SC_BB, &bb));
    const double nb = sqrt(bb);
    // r = b - A x
    SPMV_TRY(run_variant(P, P->variant, d_x, q.p, s));
    hipLaunchKernelGGL(k_cg_init, dim3(g), dim3(kBlock), 0, s, n, d_b, q.as<double>(),
                       r.as<double>(), p.as<double>(), dpart);
    int cur = SC_RR0, nxt = SC_RR1;
    SPMV_HIP(dot_final(cur));
    double rr;
    SPMV_TRY(read(cur, &rr));
    int it = 0;
    double rel = nb > 0 ? sqrt(rr) / nb : 0.0;
    if (nb > 0 && !(sqrt(rr) <= rtol * nb)) {
        while (it < max_iters) {
            SPMV_TRY(run_variant(P, P->variant, p.p, q.p, s));
            hipLaunchKernelGGL(k_dot_part, dim3(g), dim3(kBlock), 0, s, n, p.as<double>(),
                               q.as<double>(), dpart);
            SPMV_HIP(dot_final(SC_PQ));
            hipLaunchKernelGGL(k_cg_xr, dim3(g), dim3(kBlock), 0, s, n, d_x, r.as<double>(),
                               p.as<double>(), q.as<double>(), dsc, cur, dpart);
            SPMV_HIP(dot_final(nxt));
            double rr_new;
            SPMV_TRY(read(nxt, &rr_new));
            ++it;
            rel = sqrt(rr_new) / nb;
            if (sqrt(rr_new) <= rtol * nb || !(rr_new == rr_new)) break;
            hipLaunchKernelGGL(k_cg_p, dim3(g), dim3(kBlock), 0, s, n, p.as<double>(),
                               r.as<double>(), dsc, nxt, cur);
            SPMV_HIP(hipGetLastError());
            const int t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    SPMV_HIP(hipStreamSynchronize(s));
    if (iters) *iters = it;
    if (rel_resid) *rel_resid = rel;
    return SPMV_OK;
}
