// Dense building blocks shared by the build stages (row-major storage).
#pragma once
#include "gbs_common.h"

// C = alpha * op(A) * op(B) + beta * C for `batch` strided problems.
// op: 0 = as stored, 1 = transpose, 2 = conjugate transpose.  op(A) is M x K,
// op(B) is K x N, C is M x N; lda/ldb/ldc are row strides of the stored arrays.
template <typename C>
hipError_t zgemm(hipStream_t st, int M, int N, int K, C alpha, const C* A, long lda, long sA, int opA, const C* B,
                 long ldb, long sB, int opB, C beta, C* Cm, long ldc, long sC, int batch);

// Batched Hermitian eigensolver (FP64 Jacobi).  Matrix b: size dims[b] (or ld
// when dims == NULL), leading dimension ld, batch stride sA.  Writes
// eigenvalues (descending) to w[b*ld + k] and eigenvectors as columns of Vout.
// A and Vtmp are overwritten.
hipError_t jacobi_herm(hipStream_t st, cplx64* A, cplx64* Vtmp, double* w, const int* dims, long ld, long sA,
                       int batch, int* err, cplx64* Vout);

// Same problem, faster for large batches: rotations are logged (log_stride
// entries per matrix, see jacobi_log_entries) and the eigenvectors rebuilt by
// a replay pass spread over many workgroups.  nsw: per-matrix sweep counts.
long jacobi_log_entries(int n, int max_sweeps);
hipError_t jacobi_herm_logged(hipStream_t st, cplx64* A, cplx64* Vtmp, double* w, const int* dims, int nmax, long ld,
                              long sA, int batch, int* err, cplx64* Vout, double2* logz, long log_stride,
                              int* nsw, int max_sweeps);
