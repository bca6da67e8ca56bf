// Products with the dense operators of the statistical workloads (kernel PCA:
// A = K; sample covariance: A = scale X^T X), as rocBLAS GEMMs, which run on
// the MFMA units.  The callers' blocks are row-major n x k; a row-major block
// is the column-major k x n matrix with the same leading dimension, so
// Y = A X becomes Y^T = X^T A (A symmetric) with no transposition of data.
#include <rocblas/rocblas.h>

#include "kernels.h"

namespace rafeast {

namespace {

hipError_t to_hip(rocblas_status s) {
  switch (s) {
    case rocblas_status_success: return hipSuccess;
    case rocblas_status_memory_error: return hipErrorOutOfMemory;
    case rocblas_status_invalid_size:
    case rocblas_status_invalid_pointer:
    case rocblas_status_invalid_value:
    case rocblas_status_invalid_handle: return hipErrorInvalidValue;
    default: return hipErrorUnknown;
  }
}

bool fits_int(int64_t v) { return v >= 0 && v < ((int64_t)1 << 31); }

}  // namespace

hipError_t dense_create_handle(void** blas) {
  rocblas_handle h = nullptr;
  const rocblas_status s = rocblas_create_handle(&h);
  *blas = s == rocblas_status_success ? (void*)h : nullptr;
  return to_hip(s);
}

void dense_destroy_handle(void* blas) {
  if (blas) (void)rocblas_destroy_handle((rocblas_handle)blas);
}

hipError_t dense_apply_f64(const DenseOp& A, hipStream_t st, int k, const double* X, int ldx,
                           double* Y, int ldy, double alpha, double beta) {
  if (k == 0) return hipSuccess;
  if (k < 0 || !A.blas || !fits_int(A.n) || !fits_int(A.rows) || ldx < k || ldy < k)
    return hipErrorInvalidValue;
  rocblas_handle h = (rocblas_handle)A.blas;
  rocblas_status s = rocblas_set_stream(h, st);
  if (s != rocblas_status_success) return to_hip(s);
  const int n = (int)A.n;
  if (A.kind == 1) {
    // Y^T (k x n) = alpha X^T K + beta Y^T
    s = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, k, n, n, &alpha, X, ldx,
                      A.a64, n, &beta, Y, ldy);
    return to_hip(s);
  }
  if (A.kind != 2 || k > A.tcols) return hipErrorInvalidValue;
  const int rows = (int)A.rows;
  const double one = 1.0, zero = 0.0, as = alpha * A.scale;
  // T^T (k x rows) = X^T Xd^T, then Y^T = alpha scale T^T Xd + beta Y^T
  s = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, k, rows, n, &one, X,
                    ldx, A.a64, rows, &zero, A.t64, k);
  if (s != rocblas_status_success) return to_hip(s);
  s = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, k, n, rows, &as, A.t64, k,
                    A.a64, rows, &beta, Y, ldy);
  return to_hip(s);
}

hipError_t dense_apply_f32(const DenseOp& A, hipStream_t st, int k, const float* X, int ldx,
                           float* Y, int ldy) {
  if (k == 0) return hipSuccess;
  if (k < 0 || !A.blas || !fits_int(A.n) || !fits_int(A.rows) || ldx < k || ldy < k)
    return hipErrorInvalidValue;
  rocblas_handle h = (rocblas_handle)A.blas;
  rocblas_status s = rocblas_set_stream(h, st);
  if (s != rocblas_status_success) return to_hip(s);
  const int n = (int)A.n;
  const float one = 1.0f, zero = 0.0f;
  if (A.kind == 1) {
    s = rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_none, k, n, n, &one, X, ldx,
                      A.a32, n, &zero, Y, ldy);
    return to_hip(s);
  }
  if (A.kind != 2 || k > A.tcols) return hipErrorInvalidValue;
  const int rows = (int)A.rows;
  const float sc = (float)A.scale;
  s = rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_transpose, k, rows, n, &one, X,
                    ldx, A.a32, rows, &zero, A.t32, k);
  if (s != rocblas_status_success) return to_hip(s);
  s = rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_none, k, n, rows, &sc, A.t32, k,
                    A.a32, rows, &zero, Y, ldy);
  return to_hip(s);
}

hipError_t dense_axpy(const DenseOp& A, hipStream_t st, int64_t count, double a, const double* x,
                      double* y) {
  if (count == 0) return hipSuccess;
  if (!A.blas || !fits_int(count)) return hipErrorInvalidValue;
  rocblas_handle h = (rocblas_handle)A.blas;
  rocblas_status s = rocblas_set_stream(h, st);
  if (s != rocblas_status_success) return to_hip(s);
  return to_hip(rocblas_daxpy(h, (int)count, &a, x, 1, y, 1));
}

}  // namespace rafeast
