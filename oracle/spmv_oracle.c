/*
 * Plain FP64 CPU oracle for the sparse matrix-vector product (test
 * infrastructure only: used by the tests and the CPU baseline, never by the
 * GPU library).
 *
 * Computes y = alpha * A * x + beta * y, the product Y = A X of the paper's
 * SpMV background section extended with the BLAS scaling factors. Each row is
 * summed in FP64 in increasing column order, exactly as the CSR arrays list
 * it (Popular SpMV Formats, CSR paragraph). When beta == 0 the old y is not
 * read, so a NaN there does not propagate.
 */
#include <stdint.h>

void oracle_spmv_csr_f64(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                         const double *val, const double *x, double alpha, double beta,
                         double *y, int n_threads)
{
    if (n_threads < 1)
        n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1024) num_threads(n_threads)
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += val[k] * x[col[k]];
        double r = alpha * s;
        if (beta != 0.0)
            r += beta * y[i];
        y[i] = r;
    }
}

/* Same product, one row at a time, for sampled checks at full size. */
void oracle_spmv_rows_f64(int64_t n_sample, const int64_t *rows, const int64_t *row_ptr,
                          const int32_t *col, const double *val, const double *x, double alpha,
                          double beta, const double *y_in, double *y_out, double *denom)
{
    for (int64_t t = 0; t < n_sample; ++t) {
        int64_t i = rows[t];
        double s = 0.0, d = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            double p = val[k] * x[col[k]];
            s += p;
            d += p < 0 ? -p : p;
        }
        double r = alpha * s;
        double dy = 0.0;
        if (beta != 0.0) {
            r += beta * y_in[i];
            dy = beta * y_in[i];
            dy = dy < 0 ? -dy : dy;
        }
        y_out[t] = r;
        denom[t] = (alpha < 0 ? -alpha : alpha) * d + dy;
    }
}

int oracle_abi_version(void) { return 1; }
