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

// T^T (k x rows, leading dimension k) = X^T Xd^T for the covariance form.
// Its output is small and its inner dimension n long, so a single GEMM
// fills only a few tiles of the chip: with split > 1 the inner dimension is
// cut into split equal chunks (and a remainder), their products formed as
// one strided-batched GEMM into the partial slabs after T, and summed by a
// GEMV with a vector of ones.
template <typename R, typename Gemm, typename Batched, typename Gemv>
rocblas_status xvt(const DenseOp& A, rocblas_handle h, int k, const R* X, int ldx, const R* Xd,
                   R* T, const R* ones, Gemm gemm, Batched batched, Gemv gemv) {
  const int n = (int)A.n, rows = (int)A.rows;
  const R one = 1, zero = 0;
  if (A.split <= 1 || (int64_t)k * rows >= ((int64_t)1 << 31))
    return gemm(h, rocblas_operation_none, rocblas_operation_transpose, k, rows, n, &one, X, ldx,
                Xd, rows, &zero, T, k);
  const int S = A.split, c = n / S, rem = n - S * c;
  const size_t slab = (size_t)k * rows;
  R* part = T + (size_t)rows * A.tcols;
  rocblas_status s = batched(h, rocblas_operation_none, rocblas_operation_transpose, k, rows, c,
                             &one, X, ldx, (rocblas_stride)c * ldx, Xd, rows,
                             (rocblas_stride)c * rows, &zero, part, k, (rocblas_stride)slab, S);
  if (s != rocblas_status_success) return s;
  if (rem > 0) {
    s = gemm(h, rocblas_operation_none, rocblas_operation_transpose, k, rows, rem, &one,
             X + (size_t)S * c * ldx, ldx, Xd + (size_t)S * c * rows, rows, &zero,
             part + (size_t)S * slab, k);
    if (s != rocblas_status_success) return s;
  }
  return gemv(h, rocblas_operation_none, (int)slab, S + (rem > 0 ? 1 : 0), &one, part, (int)slab,
              ones, 1, &zero, T, 1);
}

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
  const double as = alpha * A.scale;
  // T^T (k x rows) = X^T Xd^T, then Y^T = alpha scale T^T Xd + beta Y^T
  s = xvt<double>(A, h, k, X, ldx, A.a64, A.t64, A.ones64, rocblas_dgemm,
                  rocblas_dgemm_strided_batched, rocblas_dgemv);
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
  s = xvt<float>(A, h, k, X, ldx, A.a32, A.t32, A.ones32, rocblas_sgemm,
                 rocblas_sgemm_strided_batched, rocblas_sgemv);
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
