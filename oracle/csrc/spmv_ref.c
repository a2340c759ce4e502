/* Plain CSR SpMV (Algorithm 1 of the paper, with the accumulation the
 * printed listing drops): y[i] = sum over j in [rowptr[i], rowptr[i+1]) of
 * val[j] * x[colind[j]], summed in increasing j from +0.0.
 *
 * TEST INFRASTRUCTURE: host timing of the oracle loop.  Built with
 * -O2 -ffp-contract=off so that every multiply and add rounds separately,
 * exactly like the Python oracle.  Shares no code with the HIP library.
 *
 * spmv_ref_f64      single thread.
 * spmv_ref_f64_omp  the same loop over the paper's default static partition
 *                   (contiguous row ranges with equal nonzeros per thread,
 *                   Section 3.2.1), one range per OpenMP thread.
 */
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void spmv_ref_f64(int64_t n, const int32_t *rowptr, const int32_t *colind,
                  const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = rowptr[i]; j < rowptr[i + 1]; ++j)
            s = s + val[j] * x[colind[j]];
        y[i] = s;
    }
}

static int64_t lower_bound(const int32_t *a, int64_t n, int64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

int spmv_ref_f64_omp(int64_t n, const int32_t *rowptr, const int32_t *colind,
                     const double *val, const double *x, double *y)
{
    int used = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
        int t = omp_get_thread_num(), P = omp_get_num_threads();
        int64_t nnz = rowptr[n];
        int64_t lo = t == 0 ? 0 : lower_bound(rowptr, n + 1, (t * nnz + P - 1) / P);
        int64_t hi = t == P - 1 ? n : lower_bound(rowptr, n + 1, ((t + 1) * nnz + P - 1) / P);
        for (int64_t i = lo; i < hi; ++i) {
            double s = 0.0;
            for (int64_t j = rowptr[i]; j < rowptr[i + 1]; ++j)
                s = s + val[j] * x[colind[j]];
            y[i] = s;
        }
        if (t == 0) used = P;
    }
#else
    spmv_ref_f64(n, rowptr, colind, val, x, y);
#endif
    return used;
}
