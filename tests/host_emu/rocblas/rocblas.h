// CPU stand-in for the rocBLAS declarations the library uses (host-emulation
// and host-logic tests only).
#pragma once
#include <cstdint>
typedef int32_t rocblas_int;
typedef int64_t rocblas_stride;
typedef enum { rocblas_status_success = 0, rocblas_status_invalid_value = 3 } rocblas_status;
typedef enum {
    rocblas_operation_none = 111,
    rocblas_operation_transpose = 112,
    rocblas_operation_conjugate_transpose = 113
} rocblas_operation;
struct MockBlas;
typedef MockBlas* rocblas_handle;
struct rocblas_float_complex {
    float x, y;
    rocblas_float_complex(float a = 0.0f, float b = 0.0f) : x(a), y(b) {}
};
struct rocblas_double_complex {
    double x, y;
    rocblas_double_complex(double a = 0.0, double b = 0.0) : x(a), y(b) {}
};
struct MockStream;
rocblas_status rocblas_create_handle(rocblas_handle* h);
rocblas_status rocblas_destroy_handle(rocblas_handle h);
rocblas_status rocblas_set_stream(rocblas_handle h, MockStream* s);
rocblas_status rocblas_cgemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, rocblas_int m, rocblas_int n,
                             rocblas_int k, const rocblas_float_complex* alpha, const rocblas_float_complex* A,
                             rocblas_int lda, const rocblas_float_complex* B, rocblas_int ldb,
                             const rocblas_float_complex* beta, rocblas_float_complex* C, rocblas_int ldc);
rocblas_status rocblas_zgemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, rocblas_int m, rocblas_int n,
                             rocblas_int k, const rocblas_double_complex* alpha, const rocblas_double_complex* A,
                             rocblas_int lda, const rocblas_double_complex* B, rocblas_int ldb,
                             const rocblas_double_complex* beta, rocblas_double_complex* C, rocblas_int ldc);
rocblas_status rocblas_cgemm_strided_batched(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, rocblas_int m,
                                             rocblas_int n, rocblas_int k, const rocblas_float_complex* alpha,
                                             const rocblas_float_complex* A, rocblas_int lda, rocblas_stride sa,
                                             const rocblas_float_complex* B, rocblas_int ldb, rocblas_stride sb,
                                             const rocblas_float_complex* beta, rocblas_float_complex* C,
                                             rocblas_int ldc, rocblas_stride sc, rocblas_int batch);
rocblas_status rocblas_zgemm_strided_batched(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, rocblas_int m,
                                             rocblas_int n, rocblas_int k, const rocblas_double_complex* alpha,
                                             const rocblas_double_complex* A, rocblas_int lda, rocblas_stride sa,
                                             const rocblas_double_complex* B, rocblas_int ldb, rocblas_stride sb,
                                             const rocblas_double_complex* beta, rocblas_double_complex* C,
                                             rocblas_int ldc, rocblas_stride sc, rocblas_int batch);
