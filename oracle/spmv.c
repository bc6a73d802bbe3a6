/* Plain CSR sparse matrix-vector product y = A x in FP64, rows split over
 * OpenMP threads.  TEST INFRASTRUCTURE ONLY: the benchmark's CPU baseline
 * times the oracle's assembled operator with it.  No SIMD intrinsics, no
 * blocking: one row after the other, entries in stored order.
 *
 * indptr[n_rows + 1], indices[nnz], data[nnz], x[n_cols], y[n_rows].
 * Returns the number of threads the parallel region ran with. */
#include <stdint.h>
#include <omp.h>

int oracle_csr_spmv(int64_t n_rows, const int64_t *indptr, const int32_t *indices,
                    const double *data, const double *x, double *y) {
  int used = 1;
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
      double s = 0.0;
      for (int64_t q = indptr[i]; q < indptr[i + 1]; ++q) s += data[q] * x[indices[q]];
      y[i] = s;
    }
  }
  return used;
}
