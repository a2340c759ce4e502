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
 * spmv_ref_dot2     the accuracy reference: every row's dot product by
 *                   Dot2 (Ogita, Rump and Oishi, "Accurate sum and dot
 *                   product", SIAM J. Sci. Comput. 26(6), 2005), i.e. as if
 *                   computed in twice the working precision and rounded
 *                   once, plus the row's scale sum |a_ij| |x_j|.
 */
#include <math.h>
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

/* Error-free transformations (Knuth's TwoSum; TwoProduct by one fused
 * multiply-add, exact barring overflow and underflow).  The -ffp-contract=off
 * build keeps every other operation a separately rounded one. */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void two_product(double a, double b, double *p, double *e)
{
    double q = a * b;
    *e = __builtin_fma(a, b, -q);
    *p = q;
}

/* y_ref[i] = Dot2 over the row's products val[j] * x[colind[j]] in
 * increasing j: the running sum p with its error terms accumulated in s,
 * result p + s.  Its error is at most u |y_i| + gamma_L^2 scale[i]
 * (u = 2^-53, L the row length), so below 1e-20 scale[i] for any row
 * shorter than 10^6.  scale[i] = sum |val[j]| |x[colind[j]]| (plain sum: it
 * only sizes the tolerance).  Rows run in parallel when OpenMP is on. */
void spmv_ref_dot2(int64_t n, const int32_t *rowptr, const int32_t *colind,
                   const double *val, const double *x, double *y_ref, double *scale)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4096)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double p = 0.0, s = 0.0, sc = 0.0;
        int64_t a = rowptr[i], b = rowptr[i + 1];
        if (a < b) {
            two_product(val[a], x[colind[a]], &p, &s);
            sc = fabs(val[a]) * fabs(x[colind[a]]);
        }
        for (int64_t j = a + 1; j < b; ++j) {
            double h, r, q;
            two_product(val[j], x[colind[j]], &h, &r);
            two_sum(p, h, &p, &q);
            s = s + (q + r);
            sc = sc + fabs(val[j]) * fabs(x[colind[j]]);
        }
        y_ref[i] = p + s;
        scale[i] = sc;
    }
}

/* The plain sequential loop of spmv_ref_f64 with OpenMP over rows (the
 * result does not depend on the thread count: each row is one thread's
 * sequential sum). */
void spmv_ref_seq_par(int64_t n, const int32_t *rowptr, const int32_t *colind,
                      const double *val, const double *x, double *y)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4096)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double t = 0.0;
        for (int64_t j = rowptr[i]; j < rowptr[i + 1]; ++j)
            t = t + val[j] * x[colind[j]];
        y[i] = t;
    }
}
