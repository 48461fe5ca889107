/* Sparse matrix-vector product y = A x in CSR form on all host cores
 * (oracle, test infrastructure only: the matrix-based CPU baseline beside the
 * GPU operator).  Row-parallel with OpenMP, static schedule; the row loop is
 * the plain definition y_i = sum_k val[k] x[col[k]].
 * row_ptr: n + 1 int64, col: nnz int32 (scipy's index type), val: nnz double. */
#include <omp.h>
#include <stdint.h>

int oracle_spmv_threads(void) { return omp_get_max_threads(); }

void oracle_spmv(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val, const double* x,
                 double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * x[col[k]];
    y[i] = s;
  }
}
