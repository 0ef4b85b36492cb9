/*
 * Multi-core CSR sparse matrix-vector product y = A x (OpenMP, FP64).
 *
 * Test infrastructure: it times the oracle's assembled operator on all host
 * cores, beside the single-threaded scipy product.  Rows are split statically
 * over the threads; each row is summed in storage order, as scipy does.
 */
#include <omp.h>
#include <stdint.h>

void oracle_csr_spmv(int32_t n, const int32_t* indptr, const int32_t* indices, const double* data,
                     const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t k = indptr[i]; k < indptr[i + 1]; ++k) s += data[k] * x[indices[k]];
    y[i] = s;
  }
}

int oracle_csr_threads(void) { return omp_get_max_threads(); }
