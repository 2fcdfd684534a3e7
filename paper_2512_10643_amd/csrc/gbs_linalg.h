// Dense building blocks shared by the build stages (row-major storage).
#pragma once
#include "gbs_common.h"

// C = alpha * op(A) * op(B) + beta * C for `batch` strided problems.
// op: 0 = as stored, 1 = transpose, 2 = conjugate transpose.  op(A) is M x K,
// op(B) is K x N, C is M x N; lda/ldb/ldc are row strides of the stored arrays.
// ws (optional, ws_elems elements): lets a long-K product with few output
// tiles split K over workgroups (partials summed in a fixed order).
template <typename C>
hipError_t zgemm(hipStream_t st, int M, int N, int K, C alpha, const C* A, long lda, long sA, int opA, const C* B,
                 long ldb, long sB, int opB, C beta, C* Cm, long ldc, long sC, int batch, C* ws = nullptr,
                 long ws_elems = 0);

// The same product for complex FP32 data by split-BF16x3 products on the BF16
// matrix cores (relative error of order 2^-16 per real product).
hipError_t zgemm_bf16x3(hipStream_t st, int M, int N, int K, cplx32 alpha, const cplx32* A, long lda, long sA,
                        int opA, const cplx32* B, long ldb, long sB, int opB, cplx32 beta, cplx32* Cm, long ldc,
                        long sC, int batch, cplx32* ws = nullptr, long ws_elems = 0);

// Batched Hermitian eigensolver (FP64 Jacobi).  Matrix b: size dims[b] (or ld
// when dims == NULL), leading dimension ld, batch stride sA.  Writes
// eigenvalues (descending) to w[b*ld + k] and eigenvectors as columns of Vout.
// A and Vtmp are overwritten.
hipError_t jacobi_herm(hipStream_t st, cplx64* A, cplx64* Vtmp, double* w, const int* dims, long ld, long sA,
                       int batch, int* err, cplx64* Vout);

// Same problem by blocked Jacobi (32 x 32 subproblems per round, see the
// kernels): workspace Vs of jacobi_blocked_ws_elems(nmax, batch) complex,
// `active` (batch ints), `vid` (jacobi_blocked_ws_elems / 1024 ints) and `dm`
// (batch doubles).  Runs sweeps until a whole
// sweep needs no rotation or max_sweeps is reached; synchronises `st` once per
// sweep.  *sweeps_done receives the number of sweeps run, or -1 when the
// last allowed sweep still rotated (not converged).
long jacobi_blocked_ws_elems(int nmax, int batch);
hipError_t jacobi_herm_blocked(hipStream_t st, cplx64* A, cplx64* Vtmp, double* w, const int* dims, int nmax,
                               long ld, long sA, int batch, int* err, cplx64* Vout, cplx64* Vs, int* active,
                               int* vid, double* dm, int max_sweeps, int* sweeps_done);
