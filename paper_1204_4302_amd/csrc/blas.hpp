// Type-overloaded rocBLAS GEMM entry points (FP32 / FP64), column-major.
#pragma once
#include <rocblas/rocblas.h>

namespace demag {

inline rocblas_status gemm_sb(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                       const float* al, const float* A, int lda, rocblas_stride sa, const float* B, int ldb,
                       rocblas_stride sb, const float* be, float* C, int ldc, rocblas_stride sc, int batch) {
    return rocblas_sgemm_strided_batched(h, ta, tb, m, n, k, al, A, lda, sa, B, ldb, sb, be, C, ldc, sc, batch);
}
inline rocblas_status gemm_sb(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                       const double* al, const double* A, int lda, rocblas_stride sa, const double* B, int ldb,
                       rocblas_stride sb, const double* be, double* C, int ldc, rocblas_stride sc, int batch) {
    return rocblas_dgemm_strided_batched(h, ta, tb, m, n, k, al, A, lda, sa, B, ldb, sb, be, C, ldc, sc, batch);
}
inline rocblas_status gemm_b(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                      const float* al, const float* const* A, int lda, const float* const* B, int ldb,
                      const float* be, float* const* C, int ldc, int batch) {
    return rocblas_sgemm_batched(h, ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc, batch);
}
inline rocblas_status gemm_b(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                      const double* al, const double* const* A, int lda, const double* const* B, int ldb,
                      const double* be, double* const* C, int ldc, int batch) {
    return rocblas_dgemm_batched(h, ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc, batch);
}
inline rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                    const float* al, const float* A, int lda, const float* B, int ldb, const float* be, float* C,
                    int ldc) {
    return rocblas_sgemm(h, ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc);
}
inline rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                    const double* al, const double* A, int lda, const double* B, int ldb, const double* be,
                    double* C, int ldc) {
    return rocblas_dgemm(h, ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc);
}
inline rocblas_status gemv_sb(rocblas_handle h, rocblas_operation ta, int m, int n, const float* al, const float* A,
                              int lda, rocblas_stride sa, const float* x, int incx, rocblas_stride sx, const float* be,
                              float* y, int incy, rocblas_stride sy, int batch) {
    return rocblas_sgemv_strided_batched(h, ta, m, n, al, A, lda, sa, x, incx, sx, be, y, incy, sy, batch);
}
inline rocblas_status gemv_sb(rocblas_handle h, rocblas_operation ta, int m, int n, const double* al, const double* A,
                              int lda, rocblas_stride sa, const double* x, int incx, rocblas_stride sx, const double* be,
                              double* y, int incy, rocblas_stride sy, int batch) {
    return rocblas_dgemv_strided_batched(h, ta, m, n, al, A, lda, sa, x, incx, sx, be, y, incy, sy, batch);
}

}  // namespace demag
