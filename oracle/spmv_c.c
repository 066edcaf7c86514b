/* Plain CSR sparse matrix-vector product y = A x (complex double), OpenMP
 * over rows.  Test infrastructure: times the oracle's assembled HEOMLS on
 * all host cores beside the GPU apply. */
#include <complex.h>
#include <omp.h>
#include <stdint.h>

void csr_spmv_z(int64_t n_rows, const int64_t *indptr, const int64_t *indices, const double complex *data,
                const double complex *x, double complex *y) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n_rows; ++r) {
    double complex acc = 0;
    for (int64_t p = indptr[r]; p < indptr[r + 1]; ++p) acc += data[p] * x[indices[p]];
    y[r] = acc;
  }
}

int csr_threads(void) { return omp_get_max_threads(); }
