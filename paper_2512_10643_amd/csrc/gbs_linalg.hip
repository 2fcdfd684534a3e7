// Dense building blocks: complex GEMM (FP32/FP64) and batched Hermitian
// Jacobi eigensolver (FP64), both row-major.
#include "gbs_linalg.h"

#include <algorithm>
#include <vector>

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

// Tile (x, y, z) of this workgroup.  The device deals workgroups to its
// eight XCDs (each with its own L2) in turn by launch index, so launch index
// L runs tile (L mod 8) * (count / 8) + L / 8 of the x-fastest order: each
// XCD gets a contiguous eighth of the tiles (whole problems, or whole
// K-slices), whose operands then stay in its L2 instead of every XCD
// streaming all of them.
__device__ inline void xcd_tile(int& tx, int& ty, int& tz) {
  const unsigned nxy = gridDim.x * gridDim.y, ntot = nxy * gridDim.z;
  unsigned L = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  if ((ntot & 7u) == 0) L = (L & 7u) * (ntot >> 3) + (L >> 3);
  tx = (int)(L % gridDim.x);
  ty = (int)((L / gridDim.x) % gridDim.y);
  tz = (int)(L / nxy);
}

namespace {
constexpr int kGT = 32;   // output tile (complex) per workgroup
// LDS row pitch of the staged operand blocks: one element more than the tile,
// so that the lanes writing one row of A (or of B^T) down the K direction
// land in different banks instead of all in the same ones
constexpr int kGP = kGT + 1;
constexpr int kGK = 16;   // K block per stage
}  // namespace

template <typename C>
__global__ __launch_bounds__(256) void zgemm_mfma_kernel(int M, int N, int K, C alpha, const C* __restrict__ A,
                                                         long lda, long sA, int opA, const C* __restrict__ B,
                                                         long ldb, long sB, int opB, C beta, C* __restrict__ Cm,
                                                         long ldc, long sC, int ksplit, C* __restrict__ part_out) {
  typedef mma_traits<C> T;
  typedef typename T::R R;
  typedef typename T::R4 R4;
  typedef typename T::V2 V2;
  // per wave: As[kGK][kGP] and Bs[kGK][kGP]; reused for the 4 partial tiles
  __shared__ V2 lds[4 * 2 * kGK * kGP];
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  // tz = problem * ksplit + slice: a slice of K per workgroup when the
  // output has too few tiles to fill the device (partials summed afterwards)
  const int bz = tz / ksplit, ks = tz % ksplit;
  A += (long)bz * sA;
  B += (long)bz * sB;
  Cm += (long)bz * sC;
  const int i0 = ty * kGT, j0 = tx * kGT;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  V2* As = lds + w * 2 * kGK * kGP;
  V2* Bs = As + kGK * kGP;
  // this wave's K range within the workgroup's slice
  const int ksl = ((K + ksplit * kGK - 1) / (ksplit * kGK)) * kGK;
  const int k_lo = ks * ksl, k_hi = min(K, k_lo + ksl);
  const int kq = ((max(0, k_hi - k_lo) + 4 * kGK - 1) / (4 * kGK)) * kGK;
  const int kb = k_lo + w * kq, ke = min(k_hi, kb + kq);
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
      As[kk * kGP + ii] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = lane + 64 * r;
      int jj, kk;
      if (opB == 0) { kk = e / kGT; jj = e % kGT; } else { jj = e / kGK; kk = e % kGK; }
      Bs[kk * kGP + jj] = rb[r];
    }
  };
  // the wave's K blocks from the last to the first (the partial tiles are
  // summed in the same direction below): the chain products run over kept
  // states in order of decreasing weight, so the small terms are summed
  // before the large ones join them
  const int nbk = ke > kb ? (ke - kb + kGK - 1) / kGK : 0;
  if (nbk > 0) fetch(kb + (nbk - 1) * kGK);
  for (int jb = nbk - 1; jb >= 0; --jb) {
    stage();
    // the wave's own LDS writes complete before its lanes read each other's
    // entries (lgkmcnt(0); the loop trip count differs between waves, so no
    // workgroup barrier here)
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    if (jb > 0) fetch(kb + (jb - 1) * kGK);
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      V2 av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = As[kk * kGP + 16 * t + (lane & 15)];
        bv[t] = Bs[kk * kGP + 16 * t + (lane & 15)];
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
    for (int q = 3; q >= 0; --q) {  // the last K range first
      const V2 z = lds[q * kGT * kGT + e];
      sr += z.x;
      si += z.y;
    }
    if (ksplit > 1) {  // partial of slice ks, dense M x N per (slice, problem)
      const int nbatch = gridDim.z / ksplit;
      part_out[(((long)ks * nbatch + bz) * M + gi) * N + gj] = cmake<C>(sr, si);
      continue;
    }
    C v = cmul(alpha, cmake<C>(sr, si));
    if (beta.re != (R)0 || beta.im != (R)0) v = cadd(v, cmul(beta, Cm[(long)gi * ldc + gj]));
    Cm[(long)gi * ldc + gj] = v;
  }
}

// Sum of the K-slice partials, the last slice first, then alpha / beta.
template <typename C>
__global__ void zgemm_reduce_kernel(int M, int N, int batch, int ksplit, C alpha, C beta, const C* __restrict__ part,
                                    C* __restrict__ Cm, long ldc, long sC) {
  typedef typename real_of<C>::type R;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long per = (long)M * N;
  if (e >= per * batch) return;
  const int bz = (int)(e / per);
  const long r = e % per;
  const int gi = (int)(r / N), gj = (int)(r % N);
  C acc = cmake<C>((R)0, (R)0);
  for (int ks = ksplit - 1; ks >= 0; --ks) acc = cadd(acc, part[((long)ks * batch + bz) * per + r]);  // last slice first
  C v = cmul(alpha, acc);
  C* c = Cm + (long)bz * sC + (long)gi * ldc + gj;
  if (beta.re != (R)0 || beta.im != (R)0) v = cadd(v, cmul(beta, *c));
  *c = v;
}

namespace {
constexpr int kWT = 64;        // output tile (complex) of the wide kernel
constexpr int kWP = kWT + 1;   // its LDS row pitch (see kGP)
}  // namespace

// Wide tiles, for products with enough output to fill the device: a
// workgroup owns a 64 x 64 complex tile over the whole K range, its four
// waves own 32 x 32 quadrants (the same MFMA steps as above) and share the
// 16-deep operand blocks (64 x 16 of op(A), 16 x 64 of op(B)) through LDS,
// double buffered: the block after next is loaded into registers while the
// current one is multiplied, and written to the free buffer before the
// barrier that ends the step.  Each operand element is fetched once per
// workgroup, a quarter of the traffic per flop of the 32 x 32 tiles whose
// waves split K.
template <typename C>
__global__ __launch_bounds__(256) void zgemm_wide_kernel(int M, int N, int K, C alpha, const C* __restrict__ A,
                                                         long lda, long sA, int opA, const C* __restrict__ B,
                                                         long ldb, long sB, int opB, C beta, C* __restrict__ Cm,
                                                         long ldc, long sC) {
  typedef mma_traits<C> T;
  typedef typename T::R R;
  typedef typename T::R4 R4;
  typedef typename T::V2 V2;
  __shared__ V2 lds[2][2][kGK][kWP];  // [buffer][op(A) | op(B)][k][row or column]
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  A += (long)tz * sA;
  B += (long)tz * sB;
  Cm += (long)tz * sC;
  const int i0 = ty * kWT, j0 = tx * kWT;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int qi = w >> 1, qj = w & 1;  // this wave's quadrant
  R4 cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = R4{0, 0, 0, 0};
      cim[a][b] = R4{0, 0, 0, 0};
    }
  // staging: 1024 complex of each operand per block, 4 per thread
  V2 ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int ii, kk;
      if (opA == 0) { ii = e / kGK; kk = e % kGK; } else { kk = e / kWT; ii = e % kWT; }
      const int gi = i0 + ii, gk = k0 + kk;
      V2 v;
      v.x = 0;
      v.y = 0;
      if (gi < M && gk < K) {
        const C z = opA == 0 ? A[(long)gi * lda + gk] : A[(long)gk * lda + gi];
        v.x = z.re;
        v.y = opA == 2 ? -z.im : z.im;
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int jj, kk;
      if (opB == 0) { kk = e / kWT; jj = e % kWT; } else { jj = e / kGK; kk = e % kGK; }
      const int gj = j0 + jj, gk = k0 + kk;
      V2 v;
      v.x = 0;
      v.y = 0;
      if (gj < N && gk < K) {
        const C z = opB == 0 ? B[(long)gk * ldb + gj] : B[(long)gj * ldb + gk];
        v.x = z.re;
        v.y = opB == 2 ? -z.im : z.im;
      }
      rb[r] = v;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int ii, kk;
      if (opA == 0) { ii = e / kGK; kk = e % kGK; } else { kk = e / kWT; ii = e % kWT; }
      lds[buf][0][kk][ii] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int jj, kk;
      if (opB == 0) { kk = e / kWT; jj = e % kWT; } else { jj = e / kGK; kk = e % kGK; }
      lds[buf][1][kk][jj] = rb[r];
    }
  };
  // K blocks from the last to the first: the truncation products run over
  // kept states in order of decreasing weight, so the small terms are summed
  // before the large ones join them (one running sum from the first block
  // cost the FP32 builds two orders of magnitude in 1 - F)
  const int nk = (K + kGK - 1) / kGK;
  auto kofs = [&](int kb) { return (nk - 1 - kb) * kGK; };
  if (nk > 0) {
    fetch(kofs(0));
    stage(0);
  }
  if (nk > 1) fetch(kofs(1));
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = kb & 1;
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      V2 av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = lds[buf][0][kk][32 * qi + 16 * t + (lane & 15)];
        bv[t] = lds[buf][1][kk][32 * qj + 16 * t + (lane & 15)];
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
    // the other buffer was last read in the previous step, before the
    // barrier that ended it
    if (kb + 1 < nk) {
      stage(buf ^ 1);
      if (kb + 2 < nk) fetch(kofs(kb + 2));
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + 32 * qi + 16 * a + T::row(lane, v), gj = j0 + 32 * qj + 16 * b + (lane & 15);
        if (gi >= M || gj >= N) continue;
        C z = cmul(alpha, cmake<C>(cre[a][b][v], cim[a][b][v]));
        if (beta.re != (R)0 || beta.im != (R)0) z = cadd(z, cmul(beta, Cm[(long)gi * ldc + gj]));
        Cm[(long)gi * ldc + gj] = z;
      }
}

// One-row products (M = 1, a vector times a matrix): a 32 x 32 tile would
// leave 31 of its rows idle and stream K through four waves one block at a
// time, so these take a kernel of their own.  A workgroup owns 64 output
// columns and 16 K-slices (one thread each); the slices are summed through
// LDS in slice order, so results are deterministic.
template <typename C>
__global__ __launch_bounds__(1024) void zgemv_kernel(int N, int K, C alpha, const C* __restrict__ A, long lda,
                                                     long sA, int opA, const C* __restrict__ B, long ldb, long sB,
                                                     int opB, C beta, C* __restrict__ Cm, long sC) {
  typedef typename real_of<C>::type R;
  __shared__ C part[16][64];
  const int bz = blockIdx.y;
  A += (long)bz * sA;
  B += (long)bz * sB;
  Cm += (long)bz * sC;
  const int jl = threadIdx.x & 63, ks = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + jl;
  const int kq = (K + 15) / 16;
  const int k0 = ks * kq, k1 = min(K, k0 + kq);
  const long xs = opA == 0 ? 1 : lda;  // op(A) is 1 x K
  R sr = 0, si = 0;
  if (j < N) {
    for (int k = k0; k < k1; ++k) {
      C a = A[(long)k * xs];
      C b = opB == 0 ? B[(long)k * ldb + j] : B[(long)j * ldb + k];
      if (opA == 2) a.im = -a.im;
      if (opB == 2) b.im = -b.im;
      sr += a.re * b.re - a.im * b.im;
      si += a.re * b.im + a.im * b.re;
    }
  }
  part[ks][jl] = cmake<C>(sr, si);
  __syncthreads();
  if (ks != 0 || j >= N) return;
  C acc = part[0][jl];
  for (int q = 1; q < 16; ++q) acc = cadd(acc, part[q][jl]);
  C v = cmul(alpha, acc);
  if (beta.re != (R)0 || beta.im != (R)0) v = cadd(v, cmul(beta, Cm[j]));
  Cm[j] = v;
}

template <typename C>
hipError_t zgemm(hipStream_t st, int M, int N, int K, C alpha, const C* A, long lda, long sA, int opA, const C* B,
                 long ldb, long sB, int opB, C beta, C* Cm, long ldc, long sC, int batch, C* ws, long ws_elems) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (M == 1) {
    if (batch > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zgemv_kernel<C>, dim3((unsigned)((N + 63) / 64), (unsigned)batch), dim3(1024), 0, st, N, K,
                       alpha, A, lda, sA, opA, B, ldb, sB, opB, beta, Cm, sC);
    return hipGetLastError();
  }
  const long wide = (long)((N + kWT - 1) / kWT) * ((M + kWT - 1) / kWT) * batch;
  if (wide >= 512 && K >= 4 * kGK) {
    if (batch > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zgemm_wide_kernel<C>, dim3((N + kWT - 1) / kWT, (M + kWT - 1) / kWT, batch), dim3(256), 0, st,
                       M, N, K, alpha, A, lda, sA, opA, B, ldb, sB, opB, beta, Cm, ldc, sC);
    return hipGetLastError();
  }
  const long tiles = (long)((N + kGT - 1) / kGT) * ((M + kGT - 1) / kGT) * batch;
  int ksplit = 1;
  // a long K over few output tiles: slice K across workgroups (with a
  // workspace), to about two workgroups per CU so that one hides the
  // other's waits
  while (ws && tiles * ksplit < 512 && K / (2 * ksplit) >= 4 * kGK * 4 &&
         (long)(2 * ksplit) * batch * M * N <= ws_elems)
    ksplit *= 2;
  dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT, batch * ksplit);
  hipLaunchKernelGGL(zgemm_mfma_kernel<C>, grid, dim3(256), 0, st, M, N, K, alpha, A, lda, sA, opA, B, ldb, sB, opB,
                     beta, Cm, ldc, sC, ksplit, ws);
  if (ksplit > 1) {
    const long n = (long)batch * M * N;
    hipLaunchKernelGGL(zgemm_reduce_kernel<C>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, N, batch,
                       ksplit, alpha, beta, (const C*)ws, Cm, ldc, sC);
  }
  return hipGetLastError();
}
template hipError_t zgemm<cplx64>(hipStream_t, int, int, int, cplx64, const cplx64*, long, long, int, const cplx64*,
                                  long, long, int, cplx64, cplx64*, long, long, int, cplx64*, long);
template hipError_t zgemm<cplx32>(hipStream_t, int, int, int, cplx32, const cplx32*, long, long, int, const cplx32*,
                                  long, long, int, cplx32, cplx32*, long, long, int, cplx32*, long);

// ---------------------------------------------------------------------------
// Complex GEMM on FP32 data by split-BF16x3 products on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16).  Every FP32 operand x is split as
// x = hi + lo + r with hi = bf16(x), lo = bf16(x - hi); a real product is
// taken as hi_a hi_b + hi_a lo_b + lo_a hi_b, accumulated in FP32, which
// leaves a relative error of order 2^-16 per product (the lo_a lo_b term and
// the residuals r are dropped).  A complex multiply-add is four real products,
// so twelve BF16 MFMAs per complex 16x16x32 step.  Same tiling as
// zgemm_mfma_kernel: a 32x32 complex tile per workgroup, K split over the four
// waves, partial tiles summed in a fixed order.  Operand layout of the BF16
// MFMA: A[i = lane % 16][k = 8 (lane / 16) + e], B[k = 8 (lane / 16) + e][j =
// lane % 16] for e = 0..7; accumulator v holds D[4 (lane / 16) + v][lane % 16].
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kXK = 32;   // K block per stage (one BF16 MFMA deep)

__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}
}  // namespace

__global__ __launch_bounds__(256) void zgemm_bf16x3_kernel(int M, int N, int K, cplx32 alpha,
                                                           const cplx32* __restrict__ A, long lda, long sA, int opA,
                                                           const cplx32* __restrict__ B, long ldb, long sB, int opB,
                                                           cplx32 beta, cplx32* __restrict__ Cm, long ldc, long sC,
                                                           int ksplit, cplx32* __restrict__ part_out) {
  __shared__ float2 lds[4 * 2 * kXK * kGP];
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  const int bz = tz / ksplit, ks = tz % ksplit;
  A += (long)bz * sA;
  B += (long)bz * sB;
  Cm += (long)bz * sC;
  const int i0 = ty * kGT, j0 = tx * kGT;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  float2* As = lds + w * 2 * kXK * kGP;
  float2* Bs = As + kXK * kGP;
  const int ksl = ((K + ksplit * kXK - 1) / (ksplit * kXK)) * kXK;
  const int k_lo = ks * ksl, k_hi = min(K, k_lo + ksl);
  const int kq = ((max(0, k_hi - k_lo) + 4 * kXK - 1) / (4 * kXK)) * kXK;
  const int kb = k_lo + w * kq, ke = min(k_hi, kb + kq);
  f32x4 cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      cim[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  // staging: 1024 complex of each operand per block, 16 per lane
  float2 ra[16], rb[16];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = lane + 64 * r;
      int ii, kk;
      if (opA == 0) { ii = e / kXK; kk = e % kXK; } else { kk = e / kGT; ii = e % kGT; }
      const int gi = i0 + ii, gk = k0 + kk;
      float2 v = make_float2(0.f, 0.f);
      if (gi < M && gk < ke) {
        const cplx32 z = opA == 0 ? A[(long)gi * lda + gk] : A[(long)gk * lda + gi];
        v = make_float2(z.re, opA == 2 ? -z.im : z.im);
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = lane + 64 * r;
      int jj, kk;
      if (opB == 0) { kk = e / kGT; jj = e % kGT; } else { jj = e / kXK; kk = e % kXK; }
      const int gj = j0 + jj, gk = k0 + kk;
      float2 v = make_float2(0.f, 0.f);
      if (gj < N && gk < ke) {
        const cplx32 z = opB == 0 ? B[(long)gk * ldb + gj] : B[(long)gj * ldb + gk];
        v = make_float2(z.re, opB == 2 ? -z.im : z.im);
      }
      rb[r] = v;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = lane + 64 * r;
      int ii, kk;
      if (opA == 0) { ii = e / kXK; kk = e % kXK; } else { kk = e / kGT; ii = e % kGT; }
      As[kk * kGP + ii] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = lane + 64 * r;
      int jj, kk;
      if (opB == 0) { kk = e / kGT; jj = e % kGT; } else { jj = e / kXK; kk = e % kXK; }
      Bs[kk * kGP + jj] = rb[r];
    }
  };
  // K blocks from the last to the first, as in zgemm_mfma_kernel
  const int nbk = ke > kb ? (ke - kb + kXK - 1) / kXK : 0;
  if (nbk > 0) fetch(kb + (nbk - 1) * kXK);
  for (int jb = nbk - 1; jb >= 0; --jb) {
    stage();
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    if (jb > 0) fetch(kb + (jb - 1) * kXK);
    // split operands: for quadrant t, A rows 16 t + lane % 16, B columns 16 t + lane % 16
    bf16x8 arh[2], arl[2], aih[2], ail[2], naih[2], nail[2], brh[2], brl[2], bih[2], bil[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int kk = 8 * (lane >> 4) + e;
        const float2 av = As[kk * kGP + 16 * t + (lane & 15)];
        const float2 bv = Bs[kk * kGP + 16 * t + (lane & 15)];
        __bf16 h, l;
        split_bf16(av.x, h, l); arh[t][e] = h; arl[t][e] = l;
        split_bf16(av.y, h, l); aih[t][e] = h; ail[t][e] = l; naih[t][e] = -h; nail[t][e] = -l;
        split_bf16(bv.x, h, l); brh[t][e] = h; brl[t][e] = l;
        split_bf16(bv.y, h, l); bih[t][e] = h; bil[t][e] = l;
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        f32x4 r = cre[a][b], q = cim[a][b];
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[a], brh[b], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[a], brl[b], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl[a], brh[b], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(naih[a], bih[b], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(naih[a], bil[b], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nail[a], bih[b], r, 0, 0, 0);
        q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[a], bih[b], q, 0, 0, 0);
        q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[a], bil[b], q, 0, 0, 0);
        q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl[a], bih[b], q, 0, 0, 0);
        q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih[a], brh[b], q, 0, 0, 0);
        q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih[a], brl[b], q, 0, 0, 0);
        q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail[a], brh[b], q, 0, 0, 0);
        cre[a][b] = r;
        cim[a][b] = q;
      }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  float2* part = lds + w * kGT * kGT;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = 16 * a + 4 * (lane >> 4) + v, jj = 16 * b + (lane & 15);
        part[ii * kGT + jj] = make_float2(cre[a][b][v], cim[a][b][v]);
      }
  __syncthreads();
  for (int e = tid; e < kGT * kGT; e += 256) {
    const int ii = e / kGT, jj = e % kGT;
    const int gi = i0 + ii, gj = j0 + jj;
    if (gi >= M || gj >= N) continue;
    float sr = 0.f, si = 0.f;
#pragma unroll
    for (int q = 3; q >= 0; --q) {  // the last K range first
      const float2 z = lds[q * kGT * kGT + e];
      sr += z.x;
      si += z.y;
    }
    if (ksplit > 1) {
      const int nbatch = gridDim.z / ksplit;
      part_out[(((long)ks * nbatch + bz) * M + gi) * N + gj] = cmake<cplx32>(sr, si);
      continue;
    }
    cplx32 v = cmul(alpha, cmake<cplx32>(sr, si));
    if (beta.re != 0.f || beta.im != 0.f) v = cadd(v, cmul(beta, Cm[(long)gi * ldc + gj]));
    Cm[(long)gi * ldc + gj] = v;
  }
}

hipError_t zgemm_bf16x3(hipStream_t st, int M, int N, int K, cplx32 alpha, const cplx32* A, long lda, long sA,
                        int opA, const cplx32* B, long ldb, long sB, int opB, cplx32 beta, cplx32* Cm, long ldc,
                        long sC, int batch, cplx32* ws, long ws_elems) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  const long tiles = (long)((N + kGT - 1) / kGT) * ((M + kGT - 1) / kGT) * batch;
  int ksplit = 1;
  while (ws && tiles * ksplit < 256 && K / (2 * ksplit) >= 4 * kXK * 2 &&
         (long)(2 * ksplit) * batch * M * N <= ws_elems)
    ksplit *= 2;
  dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT, batch * ksplit);
  hipLaunchKernelGGL(zgemm_bf16x3_kernel, grid, dim3(256), 0, st, M, N, K, alpha, A, lda, sA, opA, B, ldb, sB, opB,
                     beta, Cm, ldc, sC, ksplit, ws);
  if (ksplit > 1) {
    const long n = (long)batch * M * N;
    hipLaunchKernelGGL(zgemm_reduce_kernel<cplx32>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, N, batch,
                       ksplit, alpha, beta, (const cplx32*)ws, Cm, ldc, sC);
  }
  return hipGetLastError();
}

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

// ---------------------------------------------------------------------------
// Blocked two-sided Jacobi for batches of Hermitian matrices (FP64).
//
// Indices are grouped in blocks of 16; a round pairs the blocks round robin
// (as the scalar method pairs indices) and for every pair applies one cyclic
// sweep of rotations to the 32 x 32 Hermitian subproblem on its rows and
// columns (one workgroup per subproblem, in LDS), giving a unitary V_P; the
// outer sweeps continue until no subproblem needs a rotation.  The round then applies
// A <- V^H A V and W <- W V with V block diagonal over the pairs, as 32 x 32
// tile products spread over many workgroups.  A sweep visits every block pair
// once, so the matrix is read and written once per round instead of once per
// scalar rotation round (16x fewer passes over memory than the scalar
// method).  The sweep loop stops when no subproblem of a whole sweep needed a
// rotation on its first inner sweep.
namespace {
constexpr int kBJ = 16;        // block size
constexpr int kBP = 2 * kBJ;   // subproblem size

__device__ inline void bj_pair_idx(int npb, int round, int pr, int n, int* idx) {
  int pb, qb;
  rr_pair(npb, round, pr, pb, qb);
  for (int k = 0; k < kBP; ++k) {
    const int g = k < kBJ ? pb * kBJ + k : qb * kBJ + (k - kBJ);
    idx[k] = g < n ? g : -1;
  }
}
}  // namespace

__global__ __launch_bounds__(256) void bj_init_kernel(const cplx64* __restrict__ A, const int* __restrict__ dims,
                                                      long ld, long sA, cplx64* __restrict__ Vt,
                                                      double* __restrict__ dm) {
  const int b = blockIdx.y;
  const int n = dims ? dims[b] : (int)ld;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < (long)n * n) {
    const int i = (int)(e / n), j = (int)(e % n);
    Vt[(long)b * sA + (long)i * ld + j] = cmake<cplx64>(i == j ? 1.0 : 0.0, 0.0);
  }
  if (blockIdx.x == 0) {
    __shared__ double red[16];
    const double m = diag_absmax(A + (long)b * sA, ld, n, red);
    if (threadIdx.x == 0) dm[b] = m;
  }
}

__global__ __launch_bounds__(512) void bj_solve_kernel(const cplx64* __restrict__ A, const int* __restrict__ dims,
                                                      long ld, long sA, int npb, int round,
                                                      const double* __restrict__ dm, double tol, int inner_sweeps,
                                                      cplx64* __restrict__ Vs, int* __restrict__ active,
                                                      int* __restrict__ vid) {
  const int pr = blockIdx.x, b = blockIdx.y, lane = threadIdx.x, nth = blockDim.x;
  const int n = dims ? dims[b] : (int)ld;
  const int npairs = npb / 2;
  __shared__ cplx64 S[kBP][kBP + 1], V[kBP][kBP + 1];
  __shared__ int idx[kBP];
  __shared__ int rp[kBP / 2], rq[kBP / 2];
  __shared__ double rc[kBP / 2], rs[kBP / 2];
  __shared__ cplx64 rz[kBP / 2];
  __shared__ int anyrot, needs;
  if (lane == 0) bj_pair_idx(npb, round, pr, n, idx);
  __syncthreads();
  const cplx64* a = A + (long)b * sA;
  for (int e = lane; e < kBP * kBP; e += nth) {
    const int i = e / kBP, j = e % kBP, gi = idx[i], gj = idx[j];
    S[i][j] = (gi >= 0 && gj >= 0) ? a[(long)gi * ld + gj] : cmake<cplx64>(0.0, 0.0);
    V[i][j] = cmake<cplx64>(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (lane < kBP) S[lane][lane].im = 0.0;
  __syncthreads();
  // entries below ~8 ulp of the largest diagonal entry are at the rounding
  // level of the tile products that update A between rounds
  const double floor_abs = fmax(1.8e-15 * dm[b], 1e-300);
  // a subproblem that needs no rotation leaves V = I: flag it, so the update
  // passes skip this pair
  {
    bool need = false;
    for (int e = lane; e < kBP * kBP; e += nth) {
      const int i = e / kBP, j = e % kBP;
      if (j <= i || idx[i] < 0 || idx[j] < 0) continue;
      const double ab = sqrt(cabs2(S[i][j]));
      need = need || (ab > tol * sqrt(fabs(S[i][i].re * S[j][j].re)) && ab > floor_abs);
    }
    if (lane == 0) needs = 0;
    __syncthreads();
    if (need) needs = 1;
    __syncthreads();
    if (!needs) {
      if (lane == 0) vid[(long)b * npairs + pr] = 1;
      return;
    }
    if (lane == 0) vid[(long)b * npairs + pr] = 0;
  }
  bool converged = false;
  for (int sweep = 0; sweep < inner_sweeps && !converged; ++sweep) {
    if (lane == 0) anyrot = 0;
    __syncthreads();
    for (int r = 0; r < kBP - 1; ++r) {
      if (lane < kBP / 2) {
        int p, q;
        rr_pair(kBP, r, lane, p, q);
        double c = 1.0, sn = 0.0;
        cplx64 z = cmake<cplx64>(1.0, 0.0);
        if (idx[p] >= 0 && idx[q] >= 0) {
          const double app = S[p][p].re, aqq = S[q][q].re;
          const cplx64 bpq = S[p][q];
          const double ab = sqrt(cabs2(bpq));
          if (ab > tol * sqrt(fabs(app * aqq)) && ab > floor_abs) {
            const double th = (aqq - app) / (2.0 * ab);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
            z = cmake<cplx64>(bpq.re / ab, -bpq.im / ab);  // e^{-i phi}
            anyrot = 1;
          }
        }
        rp[lane] = p;
        rq[lane] = q;
        rc[lane] = c;
        rs[lane] = sn;
        rz[lane] = z;
      }
      __syncthreads();
      // The round's 16 rotations act on disjoint index pairs, so S <- J^H S J
      // splits into independent 2 x 2 blocks (rows of pair P, columns of pair
      // Q): each is updated in one step, rows first, then columns, as the
      // two-sided product takes them, and V <- V J by pairs of columns.
      //   rows:    y_p = c x_p - s e^{i phi} x_q,  y_q = s x_p + c e^{i phi} x_q
      //   columns: y_p = c x_p - s e^{-i phi} x_q, y_q = s x_p + c e^{-i phi} x_q
      if (lane < (kBP / 2) * (kBP / 2)) {
        const int P = lane / (kBP / 2), Q = lane % (kBP / 2);
        const double sP = rs[P], sQ = rs[Q];
        if (sP != 0.0 || sQ != 0.0) {
          const int p = rp[P], q = rq[P], u = rp[Q], v = rq[Q];
          cplx64 x00 = S[p][u], x01 = S[p][v], x10 = S[q][u], x11 = S[q][v];
          if (sP != 0.0) {
            const double c = rc[P];
            const cplx64 ep = cconj(rz[P]);
            const cplx64 y00 = csub(cscale(x00, c), cmul(cscale(x10, sP), ep));
            const cplx64 y10 = cadd(cscale(x00, sP), cmul(cscale(x10, c), ep));
            const cplx64 y01 = csub(cscale(x01, c), cmul(cscale(x11, sP), ep));
            const cplx64 y11 = cadd(cscale(x01, sP), cmul(cscale(x11, c), ep));
            x00 = y00; x10 = y10; x01 = y01; x11 = y11;
          }
          if (sQ != 0.0) {
            const double c = rc[Q];
            const cplx64 em = rz[Q];
            const cplx64 y00 = csub(cscale(x00, c), cmul(cscale(x01, sQ), em));
            const cplx64 y01 = cadd(cscale(x00, sQ), cmul(cscale(x01, c), em));
            const cplx64 y10 = csub(cscale(x10, c), cmul(cscale(x11, sQ), em));
            const cplx64 y11 = cadd(cscale(x10, sQ), cmul(cscale(x11, c), em));
            x00 = y00; x10 = y10; x01 = y01; x11 = y11;
          }
          if (P == Q) {  // the rotated pair: its off-diagonal entries vanish
            x01 = cmake<cplx64>(0.0, 0.0);
            x10 = cmake<cplx64>(0.0, 0.0);
            x00.im = 0.0;
            x11.im = 0.0;
          }
          S[p][u] = x00;
          S[p][v] = x01;
          S[q][u] = x10;
          S[q][v] = x11;
        }
      }
      for (int e = lane; e < (kBP / 2) * kBP; e += nth) {
        const int pi = e / kBP, i = e % kBP;
        const double sn = rs[pi];
        if (sn == 0.0) continue;
        const double c = rc[pi];
        const cplx64 em = rz[pi];
        const int p = rp[pi], q = rq[pi];
        const cplx64 xp = V[i][p], xq = V[i][q];
        V[i][p] = csub(cscale(xp, c), cmul(cscale(xq, sn), em));
        V[i][q] = cadd(cscale(xp, sn), cmul(cscale(xq, c), em));
      }
      __syncthreads();
    }
    converged = (anyrot == 0);
    if (sweep == 0 && !converged && lane == 0) active[b] = 1;
    __syncthreads();
  }
  // an unconverged subproblem is fine: later rounds keep rotating its indices
  cplx64* vo = Vs + ((long)b * npairs + pr) * kBP * kBP;
  for (int e = lane; e < kBP * kBP; e += nth) vo[e] = V[e / kBP][e % kBP];
}

// The eigenvector side of a round, on FP64 matrix cores: the columns of
// pair P of W, 32 rows at a time, W[c, P] <- W[c, P] V_P.  Each wave forms
// one 16 x 16 quadrant of the 32 x 32 complex tile (4 real MFMAs per complex
// k-step), its fragments of V_P loaded straight into registers.
__global__ __launch_bounds__(256) void bj_w_kernel(cplx64* __restrict__ Wv, const int* __restrict__ dims, long ld,
                                                   long sA, int npb, int round, const cplx64* __restrict__ Vs,
                                                   const int* __restrict__ vid) {
  typedef mma_traits<cplx64> T;
  const int P = blockIdx.x, b = blockIdx.z;
  const int n = dims ? dims[b] : (int)ld;
  const int npairs = npb / 2;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  __shared__ cplx64 X[kBP][kBP + 1];
  __shared__ int ip[kBP];
  const int c0 = kBP * blockIdx.y;
  if (c0 >= n) return;
  if (vid[(long)b * npairs + P]) return;  // V_P = I
  if (tid == 0) bj_pair_idx(npb, round, P, n, ip);
  __syncthreads();
  if (ip[0] < 0 && ip[kBJ] < 0) return;  // pair entirely beyond n (uniform)
  cplx64* m = Wv + (long)b * sA;
  const cplx64* vp = Vs + ((long)b * npairs + P) * kBP * kBP;
  for (int e = tid; e < kBP * kBP; e += 256) {
    const int i = e / kBP, j = e % kBP;
    const int gi = c0 + i, gj = ip[j];
    X[i][j] = (gi < n && gj >= 0) ? m[(long)gi * ld + gj] : cmake<cplx64>(0.0, 0.0);
  }
  const int qi = w >> 1, qj = w & 1;
  cplx64 fv[kBP / 4];
#pragma unroll
  for (int s = 0; s < kBP / 4; ++s) fv[s] = vp[(4 * s + (lane >> 4)) * kBP + 16 * qj + (lane & 15)];
  __syncthreads();
  T::R4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
#pragma unroll
  for (int k0 = 0; k0 < kBP; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const cplx64 av = X[16 * qi + (lane & 15)][k];
    const cplx64 bv = fv[k0 / 4];
    re = T::mma(av.re, bv.re, re);
    re = T::mma(-av.im, bv.im, re);
    im = T::mma(av.re, bv.im, im);
    im = T::mma(av.im, bv.re, im);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gi = c0 + 16 * qi + T::row(lane, v), gj = ip[16 * qj + (lane & 15)];
    if (gi < n && gj >= 0) m[(long)gi * ld + gj] = cmake<cplx64>(re[v], im[v]);
  }
}

// The round's whole two-sided update A <- V^H A V of a Hermitian matrix, by
// pair blocks: workgroup (P, Q), P <= Q, forms R = V_P^H A[P, Q] V_Q (rows
// of pair P, columns of pair Q) and writes R and, for P < Q, its conjugate
// transpose as block (Q, P); block (P, P) is written exactly Hermitian.  Each
// entry of A is then read about half a time and written once per round
// (the row and column passes read and write it twice each).  A pair whose
// subproblem needed no rotation has V = I (its Vs slot is not written).
__global__ __launch_bounds__(256) void bj_sym_kernel(cplx64* __restrict__ A, const int* __restrict__ dims, long ld,
                                                     long sA, int npb, int round, const cplx64* __restrict__ Vs,
                                                     const int* __restrict__ vid) {
  typedef mma_traits<cplx64> T;
  const int b = blockIdx.y;
  const int n = dims ? dims[b] : (int)ld;
  const int npairs = npb / 2;
  int P = 0, r = blockIdx.x;
  while (r >= npairs - P) {
    r -= npairs - P;
    ++P;
  }
  const int Q = P + r;
  const int idP = vid[(long)b * npairs + P], idQ = vid[(long)b * npairs + Q];
  if (idP && idQ) return;  // both identity: the block keeps its values
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  __shared__ cplx64 X[kBP][kBP + 1];
  __shared__ int ipP[kBP], ipQ[kBP];
  if (tid == 0) bj_pair_idx(npb, round, P, n, ipP);
  if (tid == 1) bj_pair_idx(npb, round, Q, n, ipQ);
  __syncthreads();
  if ((ipP[0] < 0 && ipP[kBJ] < 0) || (ipQ[0] < 0 && ipQ[kBJ] < 0)) return;  // uniform
  cplx64* m = A + (long)b * sA;
  const cplx64* vp = Vs + ((long)b * npairs + P) * kBP * kBP;
  const cplx64* vq = Vs + ((long)b * npairs + Q) * kBP * kBP;
  for (int e = tid; e < kBP * kBP; e += 256) {
    const int i = e / kBP, j = e % kBP;
    const int gi = ipP[i], gj = ipQ[j];
    X[i][j] = (gi >= 0 && gj >= 0) ? m[(long)gi * ld + gj] : cmake<cplx64>(0.0, 0.0);
  }
  const int qi = w >> 1, qj = w & 1;
  // this lane's MFMA fragments of V_Q (column 16 qj + lane % 16) and V_P
  // (column 16 qi + lane % 16), rows k = 4 s + lane / 16, straight from
  // memory into registers
  cplx64 fq[kBP / 4], fp[kBP / 4];
#pragma unroll
  for (int s = 0; s < kBP / 4; ++s) {
    const int k = 4 * s + (lane >> 4), jq = 16 * qj + (lane & 15), jp = 16 * qi + (lane & 15);
    fq[s] = idQ ? cmake<cplx64>(k == jq ? 1.0 : 0.0, 0.0) : vq[k * kBP + jq];
    fp[s] = idP ? cmake<cplx64>(k == jp ? 1.0 : 0.0, 0.0) : vp[k * kBP + jp];
  }
  __syncthreads();
  // Y = X V_Q, this wave's 16 x 16 quadrant
  T::R4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
#pragma unroll
  for (int k0 = 0; k0 < kBP; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const cplx64 av = X[16 * qi + (lane & 15)][k];
    const cplx64 bv = fq[k0 / 4];
    re = T::mma(av.re, bv.re, re);
    re = T::mma(-av.im, bv.im, re);
    im = T::mma(av.re, bv.im, im);
    im = T::mma(av.im, bv.re, im);
  }
  __syncthreads();  // every wave is done reading X
#pragma unroll
  for (int v = 0; v < 4; ++v) X[16 * qi + T::row(lane, v)][16 * qj + (lane & 15)] = cmake<cplx64>(re[v], im[v]);
  __syncthreads();
  // R = V_P^H Y
  re = T::R4{0, 0, 0, 0};
  im = T::R4{0, 0, 0, 0};
#pragma unroll
  for (int k0 = 0; k0 < kBP; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const cplx64 av = cconj(fp[k0 / 4]);
    const cplx64 bv = X[k][16 * qj + (lane & 15)];
    re = T::mma(av.re, bv.re, re);
    re = T::mma(-av.im, bv.im, re);
    im = T::mma(av.re, bv.im, im);
    im = T::mma(av.im, bv.re, im);
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) X[16 * qi + T::row(lane, v)][16 * qj + (lane & 15)] = cmake<cplx64>(re[v], im[v]);
  __syncthreads();
  for (int e = tid; e < kBP * kBP; e += 256) {
    const int i = e / kBP, j = e % kBP;
    const int gi = ipP[i], gj = ipQ[j];
    if (gi < 0 || gj < 0) continue;
    // block (P, P): entry (i, j) below the diagonal from (j, i), so the
    // stored matrix stays exactly Hermitian
    m[(long)gi * ld + gj] = (P == Q && i > j) ? cconj(X[j][i]) : X[i][j];
  }
  if (P != Q) {
    for (int e = tid; e < kBP * kBP; e += 256) {
      const int j = e / kBP, i = e % kBP;  // row j of block (Q, P), columns i
      const int gi = ipP[i], gj = ipQ[j];
      if (gi < 0 || gj < 0) continue;
      m[(long)gj * ld + gi] = cconj(X[i][j]);
    }
  }
}

__global__ void bj_diag_kernel(const cplx64* __restrict__ A, const int* __restrict__ dims, long ld, long sA,
                               double* __restrict__ w) {
  const int b = blockIdx.x;
  const int n = dims ? dims[b] : (int)ld;
  for (int i = threadIdx.x; i < n; i += blockDim.x) w[(long)b * ld + i] = A[(long)b * sA + (long)i * ld + i].re;
}

long jacobi_blocked_ws_elems(int nmax, int batch) {
  const int nb = (nmax + kBJ - 1) / kBJ;
  const int npb = nb + (nb & 1);
  return (long)batch * (npb / 2) * kBP * kBP;
}

hipError_t jacobi_herm_blocked(hipStream_t st, cplx64* A, cplx64* Vtmp, double* w, const int* dims, int nmax,
                               long ld, long sA, int batch, int* err, cplx64* Vout, cplx64* Vs, int* active,
                               int* vid, double* dm, int max_sweeps, int* sweeps_done) {
  if (batch <= 0 || nmax <= 0) return hipSuccess;
  const int nb = (nmax + kBJ - 1) / kBJ;
  const int npb = std::max(2, nb + (nb & 1));
  const int npairs = npb / 2;
  const long nn = (long)nmax * nmax;
  hipLaunchKernelGGL(bj_init_kernel, dim3((unsigned)((nn + 255) / 256), batch), dim3(256), 0, st, A, dims, ld, sA,
                     Vtmp, dm);
  std::vector<int> act(batch);
  int sw = 0;
  for (; sw < max_sweeps; ++sw) {
    hipError_t e = hipMemsetAsync(active, 0, batch * sizeof(int), st);
    if (e != hipSuccess) return e;
    for (int r = 0; r < npb - 1; ++r) {
      hipLaunchKernelGGL(bj_solve_kernel, dim3(npairs, batch), dim3(512), 0, st, A, dims, ld, sA, npb, r, dm, 1e-15,
                         1, Vs, active, vid);
      const int nch = (nmax + kBP - 1) / kBP;
      // A <- V^H A V by pair blocks, then the eigenvector matrix W <- W V
      hipLaunchKernelGGL(bj_sym_kernel, dim3(npairs * (npairs + 1) / 2, batch), dim3(256), 0, st, A, dims, ld, sA,
                         npb, r, Vs, vid);
      hipLaunchKernelGGL(bj_w_kernel, dim3(npairs, nch, batch), dim3(256), 0, st, Vtmp, dims, ld, sA, npb, r, Vs,
                         vid);
    }
    e = hipMemcpyAsync(act.data(), active, batch * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    bool any = false;
    for (int v : act) any = any || v;
    if (!any) {
      ++sw;
      break;
    }
  }
  if (sweeps_done) *sweeps_done = sw;
  if (sw == max_sweeps) {  // the last sweep still rotated
    (void)err;
    if (sweeps_done) *sweeps_done = -1;
  }
  hipLaunchKernelGGL(bj_diag_kernel, dim3(batch), dim3(256), 0, st, A, dims, ld, sA, w);
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
