// Dense building blocks: complex GEMM (FP32/FP64) and batched Hermitian
// Jacobi eigensolver (FP64), both row-major.
#include "gbs_linalg.h"

#include <algorithm>

// ---------------------------------------------------------------------------
// Complex GEMM  C = alpha * op(A) * op(B) + beta * C, strided-batched, on the
// matrix cores (v_mfma_f64_16x16x4f64 for FP64, v_mfma_f32_16x16x4f32 for
// FP32).  op: 0 = none, 1 = transpose, 2 = conjugate transpose.
//
// A workgroup owns a 32 x 32 complex output tile; its four waves split K in
// four contiguous ranges and each accumulates the whole tile over its range
// (the chain contractions have K = d chi >> M, N), then the four partial tiles
// are summed through LDS in a fixed order, so results are deterministic.
// A wave stages 16-deep K blocks of op(A) (32 x 16) and op(B) (16 x 32)
// through its own LDS region with coalesced loads (the next block is held in
// registers while the current one is multiplied).  Each complex product is
// four real MFMAs: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
// MFMA 16x16x4 operand layout (both types): A[i = lane % 16][k = lane / 16],
// B[k = lane / 16][j = lane % 16].  Accumulator v of a lane holds
// D[4 (lane / 16) + v][lane % 16] for FP32 and D[4 v + lane / 16][lane % 16]
// for FP64 (mma_traits::row).
template <typename C> struct mma_traits;
template <> struct mma_traits<cplx64> {
  typedef double R;
  typedef double R4 __attribute__((ext_vector_type(4)));
  typedef double2 V2;
  static __device__ R4 mma(R a, R b, R4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct mma_traits<cplx32> {
  typedef float R;
  typedef float R4 __attribute__((ext_vector_type(4)));
  typedef float2 V2;
  static __device__ R4 mma(R a, R b, R4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

namespace {
constexpr int kGT = 32;   // output tile (complex) per workgroup
constexpr int kGK = 16;   // K block per stage
}  // namespace

template <typename C>
__global__ __launch_bounds__(256) void zgemm_mfma_kernel(int M, int N, int K, C alpha, const C* __restrict__ A,
                                                         long lda, long sA, int opA, const C* __restrict__ B,
                                                         long ldb, long sB, int opB, C beta, C* __restrict__ Cm,
                                                         long ldc, long sC) {
  typedef mma_traits<C> T;
  typedef typename T::R R;
  typedef typename T::R4 R4;
  typedef typename T::V2 V2;
  // per wave: As[kGK][kGT] and Bs[kGK][kGT]; reused for the 4 partial tiles
  __shared__ V2 lds[4 * 2 * kGK * kGT];
  const int bz = blockIdx.z;
  A += (long)bz * sA;
  B += (long)bz * sB;
  Cm += (long)bz * sC;
  const int i0 = blockIdx.y * kGT, j0 = blockIdx.x * kGT;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  V2* As = lds + w * 2 * kGK * kGT;
  V2* Bs = As + kGK * kGT;
  // this wave's K range
  const int kq = ((K + 4 * kGK - 1) / (4 * kGK)) * kGK;
  const int kb = w * kq, ke = min(K, kb + kq);
  R4 cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = R4{0, 0, 0, 0};
      cim[a][b] = R4{0, 0, 0, 0};
    }
  // staging: 512 complex of each operand per block, 8 per lane
  V2 ra[8], rb[8];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = lane + 64 * r;
      int ii, kk;
      if (opA == 0) { ii = e / kGK; kk = e % kGK; } else { kk = e / kGT; ii = e % kGT; }
      const int gi = i0 + ii, gk = k0 + kk;
      V2 v;
      v.x = 0;
      v.y = 0;
      if (gi < M && gk < ke) {
        const C z = opA == 0 ? A[(long)gi * lda + gk] : A[(long)gk * lda + gi];
        v.x = z.re;
        v.y = opA == 2 ? -z.im : z.im;
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = lane + 64 * r;
      int jj, kk;
      if (opB == 0) { kk = e / kGT; jj = e % kGT; } else { jj = e / kGK; kk = e % kGK; }
      const int gj = j0 + jj, gk = k0 + kk;
      V2 v;
      v.x = 0;
      v.y = 0;
      if (gj < N && gk < ke) {
        const C z = opB == 0 ? B[(long)gk * ldb + gj] : B[(long)gj * ldb + gk];
        v.x = z.re;
        v.y = opB == 2 ? -z.im : z.im;
      }
      rb[r] = v;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = lane + 64 * r;
      int ii, kk;
      if (opA == 0) { ii = e / kGK; kk = e % kGK; } else { kk = e / kGT; ii = e % kGT; }
      As[kk * kGT + ii] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = lane + 64 * r;
      int jj, kk;
      if (opB == 0) { kk = e / kGT; jj = e % kGT; } else { jj = e / kGK; kk = e % kGK; }
      Bs[kk * kGT + jj] = rb[r];
    }
  };
  if (kb < ke) fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += kGK) {
    stage();
    // the wave's own LDS writes complete before its lanes read each other's
    // entries (lgkmcnt(0); the loop trip count differs between waves, so no
    // workgroup barrier here)
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    if (k0 + kGK < ke) fetch(k0 + kGK);
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      V2 av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = As[kk * kGT + 16 * t + (lane & 15)];
        bv[t] = Bs[kk * kGT + 16 * t + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cre[a][b] = T::mma(av[a].x, bv[b].x, cre[a][b]);
          cre[a][b] = T::mma(-av[a].y, bv[b].y, cre[a][b]);
          cim[a][b] = T::mma(av[a].x, bv[b].y, cim[a][b]);
          cim[a][b] = T::mma(av[a].y, bv[b].x, cim[a][b]);
        }
    }
    __builtin_amdgcn_wave_barrier();  // keep this block's reads before the next block's stage
  }
  // sum the four partial tiles in a fixed order
  __syncthreads();
  V2* part = lds + w * kGT * kGT;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = 16 * a + T::row(lane, v), jj = 16 * b + (lane & 15);
        V2 z;
        z.x = cre[a][b][v];
        z.y = cim[a][b][v];
        part[ii * kGT + jj] = z;
      }
  __syncthreads();
  for (int e = tid; e < kGT * kGT; e += 256) {
    const int ii = e / kGT, jj = e % kGT;
    const int gi = i0 + ii, gj = j0 + jj;
    if (gi >= M || gj >= N) continue;
    R sr = 0, si = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const V2 z = lds[q * kGT * kGT + e];
      sr += z.x;
      si += z.y;
    }
    C v = cmul(alpha, cmake<C>(sr, si));
    if (beta.re != (R)0 || beta.im != (R)0) v = cadd(v, cmul(beta, Cm[(long)gi * ldc + gj]));
    Cm[(long)gi * ldc + gj] = v;
  }
}

template <typename C>
hipError_t zgemm(hipStream_t st, int M, int N, int K, C alpha, const C* A, long lda, long sA, int opA, const C* B,
                 long ldb, long sB, int opB, C beta, C* Cm, long ldc, long sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT, batch);
  hipLaunchKernelGGL(zgemm_mfma_kernel<C>, grid, dim3(256), 0, st, M, N, K, alpha, A, lda, sA, opA, B, ldb, sB, opB,
                     beta, Cm, ldc, sC);
  return hipGetLastError();
}
template hipError_t zgemm<cplx64>(hipStream_t, int, int, int, cplx64, const cplx64*, long, long, int, const cplx64*,
                                  long, long, int, cplx64, cplx64*, long, long, int);
template hipError_t zgemm<cplx32>(hipStream_t, int, int, int, cplx32, const cplx32*, long, long, int, const cplx32*,
                                  long, long, int, cplx32, cplx32*, long, long, int);

// ---------------------------------------------------------------------------
// Batched Hermitian Jacobi (FP64), one 1024-thread workgroup per matrix.
// Matrix b has size n = dims[b] (<= ld), stored at A + b*sA with leading
// dimension ld.  On exit: w[b*ld + k] eigenvalues in descending order,
// V[b*sA + i*ld + k] the matching eigenvectors as columns.  A is destroyed.
// Parallel cyclic ordering (round robin), two-sided rotations on 2x2 blocks.
__device__ inline void rr_pair(int npad, int s, int i, int& p, int& q) {
  int m = npad - 1;
  if (i == 0) {
    p = 0;
    q = 1 + (s % m);
  } else {
    p = 1 + ((s + i) % m);
    q = 1 + (((s - i) % m + m) % m);
  }
}

// Largest |a_ii| of an n x n matrix, reduced over the workgroup (<= 1024
// threads).  Sets the absolute floor below which the Hermitian Jacobi kernels
// leave an off-diagonal entry alone: dropping entries of size <= 1e-18 max|a_ii|
// moves no eigenvalue by more than n * 1e-18 max|a_ii|, far below the FP64
// error of the matrices they receive, and rank-deficient matrices (whose
// tiny diagonal entries make the relative test 1e-15 sqrt(|a_pp a_qq|)
// unreachable at the rounding floor) then converge.
__device__ double diag_absmax(const cplx64* a, long ld, int n, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double m = 0.0;
  for (int i = tid; i < n; i += nt) m = fmax(m, fabs(a[(long)i * ld + i].re));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < (nt + 63) / 64; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(1024) void jacobi_herm_batched(cplx64* __restrict__ A, cplx64* __restrict__ V,
                                                            double* __restrict__ w, const int* __restrict__ dims,
                                                            long ld, long sA, int max_sweeps, double tol,
                                                            int* __restrict__ err, cplx64* __restrict__ Vout) {
  const int b = blockIdx.x;
  const int n = dims ? dims[b] : (int)ld;
  cplx64* a = A + (long)b * sA;
  cplx64* v = V + (long)b * sA;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double rc[GBS_CHI_MAX / 2 + 1], rs[GBS_CHI_MAX / 2 + 1];
  __shared__ cplx64 rph[GBS_CHI_MAX / 2 + 1];
  __shared__ int rp[GBS_CHI_MAX / 2 + 1], rq[GBS_CHI_MAX / 2 + 1];
  __shared__ int any_rot;
  if (n <= 0) return;
  for (long e = tid; e < (long)n * n; e += nt) {
    long i = e / n, j = e % n;
    v[i * ld + j] = cmake<cplx64>(i == j ? 1.0 : 0.0, 0.0);
  }
  // make the diagonal exactly real
  for (int i = tid; i < n; i += nt) a[(long)i * ld + i].im = 0.0;
  __syncthreads();
  __shared__ double red[16];
  const double floor_abs = fmax(1e-18 * diag_absmax(a, ld, n, red), 1e-300);
  const int npad = n + (n & 1);
  const int half = npad / 2;
  bool converged = (n == 1);
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int s = 0; s < npad - 1; ++s) {
      for (int i = tid; i < half; i += nt) {
        int p, q;
        rr_pair(npad, s, i, p, q);
        double c = 1.0, sn = 0.0;
        cplx64 ph = cmake<cplx64>(1.0, 0.0);
        if (p < n && q < n) {
          double app = a[(long)p * ld + p].re, aqq = a[(long)q * ld + q].re;
          cplx64 bpq = a[(long)p * ld + q];
          double ab = sqrt(cabs2(bpq));
          if (ab > tol * sqrt(fabs(app * aqq)) && ab > floor_abs) {
            ph = cmake<cplx64>(bpq.re / ab, bpq.im / ab);
            double th = (aqq - app) / (2.0 * ab);
            double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
            any_rot = 1;
          }
        }
        rp[i] = p;
        rq[i] = q;
        rc[i] = c;
        rs[i] = sn;
        rph[i] = ph;
      }
      __syncthreads();
      // 2x2 block updates (P <= Q) and eigenvector updates.
      const long nblk = (long)half * (half + 1) / 2;
      for (long e = tid; e < nblk + (long)n * half; e += nt) {
        if (e < nblk) {
          // unrank (P, Q) with P <= Q
          int P = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) / 2.0);
          while ((long)(P + 1) * (P + 2) / 2 <= e) ++P;
          while ((long)P * (P + 1) / 2 > e) --P;
          int Q = (int)(e - (long)P * (P + 1) / 2);  // Q <= P
          int p1 = rp[P], q1 = rq[P], p2 = rp[Q], q2 = rq[Q];
          bool va = p1 < n && q1 < n, vb = p2 < n && q2 < n;
          if (P == Q) {
            if (!va || rs[P] == 0.0) continue;
            double c = rc[P], sn = rs[P];
            double app = a[(long)p1 * ld + p1].re, aqq = a[(long)q1 * ld + q1].re;
            cplx64 bpq = a[(long)p1 * ld + q1];
            double ab = sqrt(cabs2(bpq));
            double t = sn / c;
            a[(long)p1 * ld + p1] = cmake<cplx64>(app - t * ab, 0.0);
            a[(long)q1 * ld + q1] = cmake<cplx64>(aqq + t * ab, 0.0);
            a[(long)p1 * ld + q1] = cmake<cplx64>(0.0, 0.0);
            a[(long)q1 * ld + p1] = cmake<cplx64>(0.0, 0.0);
            continue;
          }
          // rows {p1,q1} (pair P) x cols {p2,q2} (pair Q); P != Q
          // J = [[c, s], [-s e^{-i ph}, c e^{-i ph}]];  X' = J_P^H X J_Q
          int r0 = p1, r1 = q1, c0 = p2, c1 = q2;
          if (!va && !vb) continue;
          cplx64 x00 = cmake<cplx64>(0, 0), x01 = x00, x10 = x00, x11 = x00;
          bool r0v = r0 < n, r1v = r1 < n, c0v = c0 < n, c1v = c1 < n;
          if (r0v && c0v) x00 = a[(long)r0 * ld + c0];
          if (r0v && c1v) x01 = a[(long)r0 * ld + c1];
          if (r1v && c0v) x10 = a[(long)r1 * ld + c0];
          if (r1v && c1v) x11 = a[(long)r1 * ld + c1];
          // right multiply by J_Q
          double cq = rc[Q], sq = rs[Q];
          cplx64 pq = cconj(rph[Q]);  // e^{-i ph}
          if (vb && sq != 0.0) {
            cplx64 y00 = csub(cscale(x00, cq), cmul(cscale(x01, sq), pq));
            cplx64 y01 = cadd(cscale(x00, sq), cmul(cscale(x01, cq), pq));
            cplx64 y10 = csub(cscale(x10, cq), cmul(cscale(x11, sq), pq));
            cplx64 y11 = cadd(cscale(x10, sq), cmul(cscale(x11, cq), pq));
            x00 = y00; x01 = y01; x10 = y10; x11 = y11;
          }
          // left multiply by J_P^H = [[c, -s e^{i ph}], [s, c e^{i ph}]]
          double cp = rc[P], sp = rs[P];
          cplx64 pp = rph[P];  // e^{i ph}
          if (va && sp != 0.0) {
            cplx64 y00 = csub(cscale(x00, cp), cmul(cscale(x10, sp), pp));
            cplx64 y01 = csub(cscale(x01, cp), cmul(cscale(x11, sp), pp));
            cplx64 y10 = cadd(cscale(x00, sp), cmul(cscale(x10, cp), pp));
            cplx64 y11 = cadd(cscale(x01, sp), cmul(cscale(x11, cp), pp));
            x00 = y00; x01 = y01; x10 = y10; x11 = y11;
          }
          if (r0v && c0v) { a[(long)r0 * ld + c0] = x00; a[(long)c0 * ld + r0] = cconj(x00); }
          if (r0v && c1v) { a[(long)r0 * ld + c1] = x01; a[(long)c1 * ld + r0] = cconj(x01); }
          if (r1v && c0v) { a[(long)r1 * ld + c0] = x10; a[(long)c0 * ld + r1] = cconj(x10); }
          if (r1v && c1v) { a[(long)r1 * ld + c1] = x11; a[(long)c1 * ld + r1] = cconj(x11); }
        } else {
          long f = e - nblk;
          int k = (int)(f / half), P = (int)(f % half);
          int p1 = rp[P], q1 = rq[P];
          if (p1 >= n || q1 >= n || rs[P] == 0.0) continue;
          double c = rc[P], sn = rs[P];
          cplx64 pq = cconj(rph[P]);
          cplx64 vp = v[(long)k * ld + p1], vq = v[(long)k * ld + q1];
          v[(long)k * ld + p1] = csub(cscale(vp, c), cmul(cscale(vq, sn), pq));
          v[(long)k * ld + q1] = cadd(cscale(vp, sn), cmul(cscale(vq, c), pq));
        }
      }
      __syncthreads();
    }
    converged = (any_rot == 0);
    __syncthreads();
  }
  if (!converged && tid == 0 && err) gbs_set_error(err, GBS_DEVERR_JACOBI_BOND);
  // sort descending: rank of each eigenvalue
  for (int i = tid; i < n; i += nt) {
    double wi = a[(long)i * ld + i].re;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      double wj = a[(long)j * ld + j].re;
      rank += (wj > wi) || (wj == wi && j < i);
    }
    w[(long)b * ld + rank] = wi;
    for (int k = 0; k < n; ++k) Vout[(long)b * sA + (long)k * ld + rank] = v[(long)k * ld + i];
  }
}

// ---------------------------------------------------------------------------
// Batched Hermitian Jacobi, two passes.  The sweep kernel (one workgroup per
// matrix) rotates only the upper triangle of A and logs (s, phi) for every
// rotation (c = sqrt(1 - s^2) since |t| <= 1; the sign of s is kept, as
// (s, phi) and (-s, phi + pi) give different rotations); the replay kernel
// rebuilds the eigenvector matrix from the identity, row blocks in parallel
// across many workgroups; a sort pass orders eigenpairs descending.
namespace {

__device__ inline cplx64 uget(const cplx64* a, long ld, int r, int c) {
  return r <= c ? a[(long)r * ld + c] : cconj(a[(long)c * ld + r]);
}
__device__ inline void uset(cplx64* a, long ld, int r, int c, cplx64 v) {
  if (r <= c) a[(long)r * ld + c] = v;
  else a[(long)c * ld + r] = cconj(v);
}

}  // namespace

__global__ __launch_bounds__(1024) void jacobi_herm_sweep_kernel(cplx64* __restrict__ A, const int* __restrict__ dims,
                                                                 long ld, long sA, int max_sweeps, double tol,
                                                                 int* __restrict__ err, double2* __restrict__ logz,
                                                                 long log_stride, int* __restrict__ nsw,
                                                                 double* __restrict__ w) {
  const int b = blockIdx.x;
  const int n = dims ? dims[b] : (int)ld;
  cplx64* a = A + (long)b * sA;
  double2* lg = logz + (long)b * log_stride;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double rc[GBS_CHI_MAX / 2 + 1], rs[GBS_CHI_MAX / 2 + 1];
  __shared__ cplx64 rz[GBS_CHI_MAX / 2 + 1];  // e^{-i phi}
  __shared__ int rp[GBS_CHI_MAX / 2 + 1], rq[GBS_CHI_MAX / 2 + 1];
  __shared__ int any_rot;
  if (n <= 0) return;
  for (int i = tid; i < n; i += nt) a[(long)i * ld + i].im = 0.0;
  __syncthreads();
  __shared__ double red[16];
  const double floor_abs = fmax(1e-18 * diag_absmax(a, ld, n, red), 1e-300);
  const int npad = n + (n & 1), half = npad / 2;
  const long nblk = (long)half * (half + 1) / 2;
  int sweeps = 0;
  bool converged = (n == 1);
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int s = 0; s < npad - 1; ++s) {
      for (int i = tid; i < half; i += nt) {
        int p, q;
        rr_pair(npad, s, i, p, q);
        double c = 1.0, sn = 0.0, phi = 0.0;
        cplx64 z = cmake<cplx64>(1.0, 0.0);
        if (p < n && q < n) {
          double app = a[(long)p * ld + p].re, aqq = a[(long)q * ld + q].re;
          cplx64 bpq = uget(a, ld, p, q);
          double ab = sqrt(cabs2(bpq));
          if (ab > tol * sqrt(fabs(app * aqq)) && ab > floor_abs) {
            double th = (aqq - app) / (2.0 * ab);
            double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
            z = cmake<cplx64>(bpq.re / ab, -bpq.im / ab);  // e^{-i phi}
            phi = atan2(bpq.im, bpq.re);
            any_rot = 1;
          }
        }
        rp[i] = p;
        rq[i] = q;
        rc[i] = c;
        rs[i] = sn;
        rz[i] = z;
        lg[((long)sweep * (npad - 1) + s) * half + i] = make_double2(sn, phi);
      }
      __syncthreads();
      for (long e = tid; e < nblk; e += nt) {
        int P = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) / 2.0);
        while ((long)(P + 1) * (P + 2) / 2 <= e) ++P;
        while ((long)P * (P + 1) / 2 > e) --P;
        int Q = (int)(e - (long)P * (P + 1) / 2);
        int p1 = rp[P], q1 = rq[P], p2 = rp[Q], q2 = rq[Q];
        if (P == Q) {
          if (p1 >= n || q1 >= n) continue;
          if (rs[P] == 0.0) continue;
          double t = rs[P] / rc[P];
          cplx64 bpq = uget(a, ld, p1, q1);
          double ab = sqrt(cabs2(bpq));
          a[(long)p1 * ld + p1] = cmake<cplx64>(a[(long)p1 * ld + p1].re - t * ab, 0.0);
          a[(long)q1 * ld + q1] = cmake<cplx64>(a[(long)q1 * ld + q1].re + t * ab, 0.0);
          uset(a, ld, p1, q1, cmake<cplx64>(0.0, 0.0));
          continue;
        }
        const bool r0v = p1 < n, r1v = q1 < n, c0v = p2 < n, c1v = q2 < n;
        cplx64 x00 = cmake<cplx64>(0, 0), x01 = x00, x10 = x00, x11 = x00;
        if (r0v && c0v) x00 = uget(a, ld, p1, p2);
        if (r0v && c1v) x01 = uget(a, ld, p1, q2);
        if (r1v && c0v) x10 = uget(a, ld, q1, p2);
        if (r1v && c1v) x11 = uget(a, ld, q1, q2);
        // X J_Q with J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
        if (c0v && c1v && rs[Q] != 0.0) {
          double cq = rc[Q], sq = rs[Q];
          cplx64 eq = rz[Q];  // e^{-i phi}
          cplx64 y00 = csub(cscale(x00, cq), cmul(cscale(x01, sq), eq));
          cplx64 y01 = cadd(cscale(x00, sq), cmul(cscale(x01, cq), eq));
          cplx64 y10 = csub(cscale(x10, cq), cmul(cscale(x11, sq), eq));
          cplx64 y11 = cadd(cscale(x10, sq), cmul(cscale(x11, cq), eq));
          x00 = y00; x01 = y01; x10 = y10; x11 = y11;
        }
        // J_P^H X with J_P^H = [[c, -s e^{i phi}], [s, c e^{i phi}]]
        if (r0v && r1v && rs[P] != 0.0) {
          double cp = rc[P], sp = rs[P];
          cplx64 ep = cconj(rz[P]);  // e^{i phi}
          cplx64 y00 = csub(cscale(x00, cp), cmul(cscale(x10, sp), ep));
          cplx64 y01 = csub(cscale(x01, cp), cmul(cscale(x11, sp), ep));
          cplx64 y10 = cadd(cscale(x00, sp), cmul(cscale(x10, cp), ep));
          cplx64 y11 = cadd(cscale(x01, sp), cmul(cscale(x11, cp), ep));
          x00 = y00; x01 = y01; x10 = y10; x11 = y11;
        }
        if (r0v && c0v) uset(a, ld, p1, p2, x00);
        if (r0v && c1v) uset(a, ld, p1, q2, x01);
        if (r1v && c0v) uset(a, ld, q1, p2, x10);
        if (r1v && c1v) uset(a, ld, q1, q2, x11);
      }
      __syncthreads();
    }
    ++sweeps;
    converged = (any_rot == 0);
    __syncthreads();
  }
  if (!converged && tid == 0 && err) gbs_set_error(err, GBS_DEVERR_JACOBI_BOND);
  if (tid == 0) nsw[b] = sweeps;
  for (int i = tid; i < n; i += nt) w[(long)b * ld + i] = a[(long)i * ld + i].re;
}

// V rows [r0, r0 + rows) of matrix b, from the identity, by replaying the log.
__global__ __launch_bounds__(256) void jacobi_herm_replay_kernel(const int* __restrict__ dims, long ld, long sA,
                                                                  int rows, const double2* __restrict__ logz,
                                                                  long log_stride, const int* __restrict__ nsw,
                                                                  cplx64* __restrict__ V) {
  const int b = blockIdx.y;
  const int n = dims ? dims[b] : (int)ld;
  const int r0 = blockIdx.x * rows;
  if (r0 >= n) return;
  const int nrow = min(rows, n - r0);
  extern __shared__ cplx64 vs[];  // rows x n
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < rows * n; e += nt) {
    int r = e / n, c = e % n;
    vs[e] = cmake<cplx64>((r0 + r == c) ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int npad = n + (n & 1), half = npad / 2;
  const int sweeps = nsw[b];
  const double2* lg = logz + (long)b * log_stride;
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int s = 0; s < npad - 1; ++s) {
      const double2* ls = lg + ((long)sw * (npad - 1) + s) * half;
      for (int e = tid; e < nrow * half; e += nt) {
        int r = e / half, i = e % half;
        const double2 sp = ls[i];
        if (sp.x == 0.0) continue;
        int p, q;
        rr_pair(npad, s, i, p, q);
        if (p >= n || q >= n) continue;
        const double sn = sp.x, c = sqrt(fmax(0.0, 1.0 - sn * sn));
        double sph, cph;
        sincos(sp.y, &sph, &cph);
        const cplx64 e_m = cmake<cplx64>(cph, -sph);  // e^{-i phi}
        cplx64 vp = vs[r * n + p], vq = vs[r * n + q];
        // V' = V J: v_p' = c v_p - s e^{-i phi} v_q ; v_q' = s v_p + c e^{-i phi} v_q
        vs[r * n + p] = csub(cscale(vp, c), cscale(cmul(vq, e_m), sn));
        vs[r * n + q] = cadd(cscale(vp, sn), cscale(cmul(vq, e_m), c));
      }
      __syncthreads();
    }
  }
  cplx64* v = V + (long)b * sA;
  for (int e = tid; e < nrow * n; e += nt) {
    int r = e / n, c = e % n;
    v[(long)(r0 + r) * ld + c] = vs[r * n + c];
  }
}

// Sort eigenpairs of matrix b descending: w (in place) and Vout columns.
__global__ __launch_bounds__(256) void jacobi_herm_sort_kernel(const int* __restrict__ dims, long ld, long sA,
                                                               double* __restrict__ w, const cplx64* __restrict__ V,
                                                               cplx64* __restrict__ Vout) {
  const int b = blockIdx.x;
  const int n = dims ? dims[b] : (int)ld;
  extern __shared__ double ws[];
  int* rk = (int*)(ws + n);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n; i += nt) ws[i] = w[(long)b * ld + i];
  __syncthreads();
  for (int i = tid; i < n; i += nt) {
    double wi = ws[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (ws[j] > wi) || (ws[j] == wi && j < i);
    rk[i] = rank;
    w[(long)b * ld + rank] = wi;
  }
  __syncthreads();
  for (long e = tid; e < (long)n * n; e += nt) {
    int k = (int)(e / n), i = (int)(e % n);
    Vout[(long)b * sA + (long)k * ld + rk[i]] = V[(long)b * sA + (long)k * ld + i];
  }
}

long jacobi_log_entries(int n, int max_sweeps) {
  const long npad = n + (n & 1);
  return (long)max_sweeps * (npad - 1) * (npad / 2);
}

hipError_t jacobi_herm_logged(hipStream_t st, cplx64* A, cplx64* Vtmp, double* w, const int* dims, int nmax, long ld,
                              long sA, int batch, int* err, cplx64* Vout, double2* logz, long log_stride,
                              int* nsw, int max_sweeps) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_herm_sweep_kernel, dim3(batch), dim3(1024), 0, st, A, dims, ld, sA, max_sweeps, 1e-15,
                     err, logz, log_stride, nsw, w);
  int rows = (int)std::max<long>(1, std::min<long>(32, 65536 / ((long)nmax * (long)sizeof(cplx64))));
  dim3 g2((nmax + rows - 1) / rows, batch);
  hipLaunchKernelGGL(jacobi_herm_replay_kernel, g2, dim3(256), (size_t)rows * nmax * sizeof(cplx64), st, dims, ld,
                     sA, rows, logz, log_stride, nsw, Vtmp);
  hipLaunchKernelGGL(jacobi_herm_sort_kernel, dim3(batch), dim3(256),
                     (size_t)nmax * (sizeof(double) + sizeof(int)), st, dims, ld, sA, w, Vtmp, Vout);
  return hipGetLastError();
}

hipError_t jacobi_herm(hipStream_t st, cplx64* A, cplx64* Vtmp, double* w, const int* dims, long ld, long sA,
                       int batch, int* err, cplx64* Vout) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_herm_batched, dim3(batch), dim3(1024), 0, st, A, Vtmp, w, dims, ld, sA, 60, 1e-15, err,
                     Vout);
  return hipGetLastError();
}
