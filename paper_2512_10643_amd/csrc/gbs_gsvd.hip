// Input validation and the iterative Gaussian SVD (Sec. II.A-B, App. A), FP64.
//
// Cuts run in order on the stream because each consumes the residual the
// previous one produced.  Williamson form of the left block L = (r_{m-1}, a_m):
//   2 Gamma_LL = L L^T (Cholesky), A = L^T Omega L (antisymmetric),
//   B = A^T A (symmetric, eigenvalues D_q^2 twice) by Jacobi rotations,
//   symplectic pairs (u, v = -A u / D) from the sorted eigenvectors (within
//   a cluster of equal eigenvalues by Gram-Schmidt), and
//   S = L [u.., v..] diag(D, D)^(-1/2).
// Bogoliubov matrices follow from Eq. MUV, the paired form of the local
// state from the regularised Q_L of App. A, and the next residual from the
// b-mode quadrature map T = -S^T Omega restricted to the active modes.
#include "gbs_gsvd.h"

namespace {

__device__ inline void wg_sync() { __syncthreads(); }

// Round-robin pair for parallel Jacobi.
__device__ inline void rr_pair_s(int npad, int s, int i, int& p, int& q) {
  int m = npad - 1;
  if (i == 0) {
    p = 0;
    q = 1 + (s % m);
  } else {
    p = 1 + ((s + i) % m);
    q = 1 + (((s - i) % m + m) % m);
  }
}

// Parallel reduction of one value per thread into red[0] (block of 1024).
__device__ double wg_sum(double x, double* red) {
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = x;
  wg_sync();
  double r = 0.0;
  if (tid == 0) {
    for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) r += red[i];
    red[32] = r;
  }
  wg_sync();
  r = red[32];
  wg_sync();
  return r;
}

}  // namespace

// ---------------------------------------------------------------------------
// Validation: symmetry and purity residual (2 Gamma Omega)^2 = -1, then PD of
// the xx block (for a symmetric symplectic 2 Gamma, positive definiteness is
// equivalent to that of its xx block: the Schur complement equals its inverse).
__global__ void validate_sym_kernel(const double* g, int n2, double* out_max_asym, double* out_max_abs) {
  double asym = 0.0, mx = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n2 * n2; e += (long)gridDim.x * blockDim.x) {
    long i = e / n2, j = e % n2;
    asym = fmax(asym, fabs(g[i * n2 + j] - g[j * n2 + i]));
    mx = fmax(mx, fabs(g[i * n2 + j]));
  }
  // max-reduce via atomics on the bit pattern (values are >= 0)
  atomicMax((unsigned long long*)out_max_asym, (unsigned long long)__double_as_longlong(asym));
  atomicMax((unsigned long long*)out_max_abs, (unsigned long long)__double_as_longlong(mx));
}

// P = (2 Gamma Omega), R = P*P + I; max |R| written atomically.  Tiled FP64.
__global__ __launch_bounds__(256) void purity_kernel(const double* g, int M, double* out_max_res) {
  const int n2 = 2 * M;
  __shared__ double As[16][17], Bs[16][17];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  // P_ij = 2 sum_k g_ik Omega_kj; Omega_kj = +1 if j = k + M (k < M), -1 if j = k - M (k >= M)
  // => P_ij = 2 * (j >= M ? g_{i, j-M} : -g_{i, j+M})
  double acc = 0.0;
  for (int k0 = 0; k0 < n2; k0 += 16) {
    int ka = k0 + tx, kb = k0 + ty;
    double pa = 0.0, pb = 0.0;
    if (row < n2 && ka < n2) pa = 2.0 * (ka >= M ? g[(long)row * n2 + ka - M] : -g[(long)row * n2 + ka + M]);
    if (kb < n2 && col < n2) pb = 2.0 * (col >= M ? g[(long)kb * n2 + col - M] : -g[(long)kb * n2 + col + M]);
    As[ty][tx] = pa;
    Bs[ty][tx] = pb;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += As[ty][k] * Bs[k][tx];
    __syncthreads();
  }
  double r = 0.0;
  if (row < n2 && col < n2) r = fabs(acc + (row == col ? 1.0 : 0.0));
  atomicMax((unsigned long long*)out_max_res, (unsigned long long)__double_as_longlong(r));
}

// Cholesky of the xx block (M x M) in one workgroup; sets NOT_PD on failure.
__global__ __launch_bounds__(1024) void chol_xx_kernel(const double* g, int M, double* w, int* err) {
  const int n2 = 2 * M, tid = threadIdx.x, nt = blockDim.x;
  for (long e = tid; e < (long)M * M; e += nt) w[e] = g[(e / M) * n2 + (e % M)];
  __shared__ double piv;
  __syncthreads();
  for (int j = 0; j < M; ++j) {
    if (tid == 0) {
      double d = w[(long)j * M + j];
      piv = d > 0.0 ? sqrt(d) : -1.0;
      if (piv > 0.0) w[(long)j * M + j] = piv;
    }
    __syncthreads();
    if (piv <= 0.0) {
      if (tid == 0) gbs_set_error(err, GBS_DEVERR_NOT_PD);
      return;
    }
    for (int i = j + 1 + tid; i < M; i += nt) w[(long)i * M + j] /= piv;
    __syncthreads();
    const long rem = M - j - 1;
    for (long e = tid; e < rem * rem; e += nt) {
      long i = j + 1 + e / rem, k = j + 1 + e % rem;
      if (k <= i) w[i * M + k] -= w[i * M + j] * w[k * M + j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Gaussian SVD chain, three launches per cut (all sizes read from device
// state so the host enqueues every cut without synchronising):
//   stage 1 (one workgroup): Gamma_LL, Cholesky, A = L^T Omega L, B = A^T A,
//            Jacobi on B packed in LDS; every rotation (c, s) is logged;
//   V-apply (several workgroups): eigenvectors of B by replaying the log on
//            row blocks of the identity (rows are independent);
//   stage 2 (one workgroup): symplectic pairs, S, U, V, (U^dag)^-1, Q^m and
//            the next residual.
namespace {

constexpr int TILE = 32;

// C (M x N, ldc) = alpha op(A) op(B) + beta C by one workgroup on the FP64
// matrix cores: each wave owns 16 x 16 output tiles (v_mfma_f64_16x16x4f64,
// operands read straight from the L2-resident workspaces).  op(X) = X^T when
// the flag is set.  C must not alias A or B.  Callers synchronise afterwards.
__device__ void wg_dgemm(int M, int N, int K, double alpha, const double* A, long lda, bool tA, const double* B,
                         long ldb, bool tB, double beta, double* C, long ldc, double* /*smem*/) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int ti = (M + 15) / 16, tj = (N + 15) / 16;
  const int r = lane & 15, kk = lane >> 4;
  for (int t = wv; t < ti * tj; t += nw) {
    const int i0 = (t / tj) * 16, j0 = (t % tj) * 16;
    const int i = i0 + r, j = j0 + r;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + kk;
      double av = 0.0, bv = 0.0;
      if (i < M && k < K) av = tA ? A[(long)k * lda + i] : A[(long)i * lda + k];
      if (j < N && k < K) bv = tB ? B[(long)j * ldb + k] : B[(long)k * ldb + j];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = i0 + 4 * v + kk, col = j0 + r;  // FP64 accumulator layout
      if (row < M && col < N) {
        double x = alpha * acc[v];
        if (beta != 0.0) x += beta * C[(long)row * ldc + col];
        C[(long)row * ldc + col] = x;
      }
    }
  }
}

__device__ inline long pk(int i, int j) {  // packed lower triangle, any order
  return i >= j ? (long)i * (i + 1) / 2 + j : (long)j * (j + 1) / 2 + i;
}

}  // namespace

// Stage 1.
__global__ __launch_bounds__(1024) void gsvd_stage1_kernel(GsvdArgs a, int m) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int M = a.M;
  if (*a.err) return;
  const int n_prev = a.ne[m - 1];
  const int nL = n_prev + 1, N2 = 2 * nL;
  if (N2 > GBS_GSVD_N2_MAX) {
    if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_KMAX);
    return;
  }
  extern __shared__ double lds[];
  __shared__ double rc[GBS_GSVD_N2_MAX / 2 + 1], rs[GBS_GSVD_N2_MAX / 2 + 1];
  __shared__ int rp[GBS_GSVD_N2_MAX / 2 + 1], rq[GBS_GSVD_N2_MAX / 2 + 1];
  __shared__ int flag, bad;
  const long ld = a.ld_ws;
  const long npk = (long)N2 * (N2 + 1) / 2;
  const bool in_lds = N2 <= GBS_GSVD_LDS_N2;
  double* P = in_lds ? lds : a.ws_pack;        // packed symmetric working matrix
  double* tiles = lds + (long)GBS_GSVD_LDS_N2 * (GBS_GSVD_LDS_N2 + 1) / 2;
  double* G = a.ws_G;
  double* Lm = a.ws_L;
  double* W = a.ws_W;
  double* Am = a.ws_A;
  const double* g = a.gamma;
  const int n2g = 2 * M;
  const double* Drr = a.drr_in;
  const double* CR = a.cr_in;
  const long ldd = a.ld_drr, ldc = a.ld_cr;
  const int gxa = m - 1, gpa = M + m - 1;

  // Gamma_LL in the xxpp order of (r_1..r_nprev, a_m); 2 Gamma_LL packed.
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    int i = (int)(e / N2), j = (int)(e % N2);
    int ii = i % nL, jj = j % nL;
    bool ip = i >= nL, jp = j >= nL;
    double val;
    if (ii < n_prev && jj < n_prev) val = Drr[(long)(ip ? n_prev + ii : ii) * ldd + (jp ? n_prev + jj : jj)];
    else if (ii < n_prev) val = CR[(long)(ip ? n_prev + ii : ii) * ldc + (jp ? gpa : gxa)];
    else if (jj < n_prev) val = CR[(long)(jp ? n_prev + jj : jj) * ldc + (ip ? gpa : gxa)];
    else val = g[(long)(ip ? gpa : gxa) * n2g + (jp ? gpa : gxa)];
    G[(long)i * ld + j] = val;
    if (j <= i) P[pk(i, j)] = 2.0 * val;
  }
  wg_sync();
  // Cholesky (right looking, packed lower triangle).
  for (int j = 0; j < N2; ++j) {
    if (tid == 0) {
      double dj = P[pk(j, j)];
      bad = !(dj > 0.0);
      P[pk(j, j)] = dj > 0.0 ? sqrt(dj) : 1.0;
    }
    wg_sync();
    if (bad) {
      if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_NOT_PD);
      return;
    }
    const double piv = P[pk(j, j)];
    for (int i = j + 1 + tid; i < N2; i += nt) P[pk(i, j)] /= piv;
    wg_sync();
    const int rem = N2 - j - 1;
    const long ntri = (long)rem * (rem + 1) / 2;
    for (long e = tid; e < ntri; e += nt) {
      int ii = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) / 2.0);
      while ((long)(ii + 1) * (ii + 2) / 2 <= e) ++ii;
      while ((long)ii * (ii + 1) / 2 > e) --ii;
      int kk = (int)(e - (long)ii * (ii + 1) / 2);
      int i = j + 1 + ii, k = j + 1 + kk;
      P[pk(i, k)] -= P[pk(i, j)] * P[pk(k, j)];
    }
    wg_sync();
  }
  // L (full, row-major) and W = Omega L: W_k = L_{k+nL} (k < nL), -L_{k-nL} (k >= nL).
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    int i = (int)(e / N2), j = (int)(e % N2);
    Lm[(long)i * ld + j] = j <= i ? P[pk(i, j)] : 0.0;
  }
  wg_sync();
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    int k = (int)(e / N2), j = (int)(e % N2);
    W[(long)k * ld + j] = k < nL ? Lm[(long)(k + nL) * ld + j] : -Lm[(long)(k - nL) * ld + j];
  }
  wg_sync();
  // A = L^T W;  B = A^T A (packed into P).
  wg_dgemm(N2, N2, N2, 1.0, Lm, ld, true, W, ld, false, 0.0, Am, ld, tiles);
  wg_sync();
  wg_dgemm(N2, N2, N2, 1.0, Am, ld, true, Am, ld, false, 0.0, a.ws_B, ld, tiles);
  wg_sync();
  for (long e = tid; e < npk; e += nt) {
    int i = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) / 2.0);
    while ((long)(i + 1) * (i + 2) / 2 <= e) ++i;
    while ((long)i * (i + 1) / 2 > e) --i;
    int j = (int)(e - (long)i * (i + 1) / 2);
    P[e] = 0.5 * (a.ws_B[(long)i * ld + j] + a.ws_B[(long)j * ld + i]);
  }
  wg_sync();
  // Jacobi on the packed matrix; rotations logged for the eigenvector pass.
  const int npad = N2 + (N2 & 1), half = npad / 2;
  const long nblk = (long)half * (half + 1) / 2;
  double2* log = a.rot_log;
  int sweeps = 0;
  bool converged = false;
  for (int sweep = 0; sweep < GBS_GSVD_MAX_SWEEPS && !converged; ++sweep) {
    if (tid == 0) flag = 0;
    wg_sync();
    for (int s = 0; s < npad - 1; ++s) {
      for (int i = tid; i < half; i += nt) {
        int p, q;
        rr_pair_s(npad, s, i, p, q);
        double c = 1.0, sn = 0.0;
        if (p < N2 && q < N2) {
          double app = P[pk(p, p)], aqq = P[pk(q, q)], apq = P[pk(p, q)];
          if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-300) {
            double th = (aqq - app) / (2.0 * apq);
            double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
            flag = 1;
          }
        }
        rp[i] = p;
        rq[i] = q;
        rc[i] = c;
        rs[i] = sn;
        log[((long)sweep * (npad - 1) + s) * half + i] = make_double2(c, sn);
      }
      wg_sync();
      for (long e = tid; e < nblk; e += nt) {
        int PP = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) / 2.0);
        while ((long)(PP + 1) * (PP + 2) / 2 <= e) ++PP;
        while ((long)PP * (PP + 1) / 2 > e) --PP;
        int QQ = (int)(e - (long)PP * (PP + 1) / 2);
        int p1 = rp[PP], q1 = rq[PP], p2 = rp[QQ], q2 = rq[QQ];
        if (PP == QQ) {
          if (p1 >= N2 || q1 >= N2 || rs[PP] == 0.0) continue;
          double t = rs[PP] / rc[PP];
          double apq = P[pk(p1, q1)];
          P[pk(p1, p1)] -= t * apq;
          P[pk(q1, q1)] += t * apq;
          P[pk(p1, q1)] = 0.0;
          continue;
        }
        bool r0v = p1 < N2, r1v = q1 < N2, c0v = p2 < N2, c1v = q2 < N2;
        double x00 = (r0v && c0v) ? P[pk(p1, p2)] : 0.0;
        double x01 = (r0v && c1v) ? P[pk(p1, q2)] : 0.0;
        double x10 = (r1v && c0v) ? P[pk(q1, p2)] : 0.0;
        double x11 = (r1v && c1v) ? P[pk(q1, q2)] : 0.0;
        double cq = rc[QQ], sq = rs[QQ];
        if (sq != 0.0) {
          double y00 = cq * x00 - sq * x01, y01 = sq * x00 + cq * x01;
          double y10 = cq * x10 - sq * x11, y11 = sq * x10 + cq * x11;
          x00 = y00; x01 = y01; x10 = y10; x11 = y11;
        }
        double cp = rc[PP], sp = rs[PP];
        if (sp != 0.0) {
          double y00 = cp * x00 - sp * x10, y01 = cp * x01 - sp * x11;
          double y10 = sp * x00 + cp * x10, y11 = sp * x01 + cp * x11;
          x00 = y00; x01 = y01; x10 = y10; x11 = y11;
        }
        if (r0v && c0v) P[pk(p1, p2)] = x00;
        if (r0v && c1v) P[pk(p1, q2)] = x01;
        if (r1v && c0v) P[pk(q1, p2)] = x10;
        if (r1v && c1v) P[pk(q1, q2)] = x11;
      }
      wg_sync();
    }
    ++sweeps;
    converged = (flag == 0);
    wg_sync();
  }
  if (!converged) {
    if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_JACOBI);
    return;
  }
  // eigenvalues and their descending order
  for (int i = tid; i < N2; i += nt) a.ws_w[i] = P[pk(i, i)];
  wg_sync();
  for (int i = tid; i < N2; i += nt) {
    double wi = a.ws_w[i];
    int rank = 0;
    for (int j = 0; j < N2; ++j) {
      double wj = a.ws_w[j];
      rank += (wj > wi) || (wj == wi && j < i);
    }
    a.ws_ord[rank] = i;
  }
  if (tid == 0) *a.nsweep = sweeps;
}

// Eigenvectors: rows [r0, r0 + ROWS) of V = J_1 J_2 ... (product of the logged
// rotations); V starts as the identity.
__global__ __launch_bounds__(256) void gsvd_vapply_kernel(GsvdArgs a, int m) {
  constexpr int ROWS = GBS_GSVD_VROWS;
  if (*a.err) return;
  const int n_prev = a.ne[m - 1];
  const int N2 = 2 * (n_prev + 1);
  const int r0 = blockIdx.x * ROWS;
  if (r0 >= N2) return;
  const int nrow = min(ROWS, N2 - r0);
  extern __shared__ double vs[];  // ROWS x N2
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < ROWS * N2; e += nt) {
    int r = e / N2, c = e % N2;
    vs[e] = (r0 + r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int npad = N2 + (N2 & 1), half = npad / 2;
  const int sweeps = *a.nsweep;
  const double2* log = a.rot_log;
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int s = 0; s < npad - 1; ++s) {
      const double2* lg = log + ((long)sw * (npad - 1) + s) * half;
      for (int e = tid; e < nrow * half; e += nt) {
        int r = e / half, i = e % half;
        double2 cs = lg[i];
        if (cs.y == 0.0) continue;
        int p, q;
        rr_pair_s(npad, s, i, p, q);
        if (p >= N2 || q >= N2) continue;
        double vp = vs[r * N2 + p], vq = vs[r * N2 + q];
        vs[r * N2 + p] = cs.x * vp - cs.y * vq;
        vs[r * N2 + q] = cs.y * vp + cs.x * vq;
      }
      __syncthreads();
    }
  }
  const long ld = a.ld_ws;
  for (int e = tid; e < nrow * N2; e += nt) {
    int r = e / N2, c = e % N2;
    a.ws_E[(long)(r0 + r) * ld + c] = vs[r * N2 + c];
  }
}

// Stage 2.
__global__ __launch_bounds__(1024) void gsvd_stage2_kernel(GsvdArgs a, int m) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
  const int M = a.M;
  if (*a.err) return;
  const int n_prev = a.ne[m - 1];
  const int nL = n_prev + 1, N2 = 2 * nL, nR = M - m;
  const long ld = a.ld_ws;
  extern __shared__ double lds[];
  double* tiles = lds;
  __shared__ double red[40];
  __shared__ double dsel[GBS_GSVD_N2_MAX / 2 + 1];
  __shared__ int cl_start[GBS_GSVD_N2_MAX + 1], pair_src[GBS_GSVD_N2_MAX + 1];
  __shared__ int ncl, npairs, bad, flag;
  double* G = a.ws_G;
  double* Lm = a.ws_L;
  double* Am = a.ws_A;
  double* Ev = a.ws_E;
  double* AE = a.ws_B;   // A E
  double* Om = a.ws_O;   // pairs [u.., v..] (unscaled, unsorted)
  double* Op = a.ws_W;   // sorted, scaled pairs
  double* Sm = a.ws_S;
  const double* w = a.ws_w;
  const int* ord = a.ws_ord;
  const double* g = a.gamma;
  const int n2g = 2 * M;
  const double* CR = a.cr_in;
  const long ldd = a.ld_drr, ldc = a.ld_cr;
  const int gxa = m - 1, gpa = M + m - 1;

  // A E (all eigenvectors; columns in original order)
  wg_dgemm(N2, N2, N2, 1.0, Am, ld, false, Ev, ld, false, 0.0, AE, ld, tiles);
  // eigenvalue clusters in descending order (relative gap 1e-6)
  if (tid == 0) {
    int nc = 0;
    cl_start[nc++] = 0;
    for (int j = 1; j < N2; ++j) {
      double hi = w[ord[j - 1]], lo = w[ord[j]];
      if (hi - lo > 1e-6 * fabs(hi)) cl_start[nc++] = j;
    }
    cl_start[nc] = N2;
    ncl = nc;
    npairs = 0;
  }
  wg_sync();
  // clusters of exactly two eigenvectors: u = e, v = -A u / |A u| (one wave each)
  // larger clusters: Gram-Schmidt within the cluster (whole workgroup)
  // pass 1: count pairs per cluster to assign slots
  if (tid == 0) {
    int k = 0;
    for (int c = 0; c < ncl; ++c) {
      int sz = cl_start[c + 1] - cl_start[c];
      pair_src[c] = k;  // first pair slot of this cluster
      k += sz / 2;
    }
    npairs = k;
    bad = (k != nL);
  }
  wg_sync();
  if (bad) {
    if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_WILLIAMSON);
    return;
  }
  for (int c = wv; c < ncl; c += nwv) {
    const int j0 = cl_start[c], sz = cl_start[c + 1] - j0;
    if (sz != 2) continue;
    const int col = ord[j0], slot = pair_src[c];
    double s = 0.0;
    for (int k = lane; k < N2; k += 64) s += AE[(long)k * ld + col] * AE[(long)k * ld + col];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const double dl = sqrt(s);
    for (int k = lane; k < N2; k += 64) {
      Om[(long)k * ld + slot] = Ev[(long)k * ld + col];
      Om[(long)k * ld + nL + slot] = -AE[(long)k * ld + col] / dl;
    }
    if (lane == 0) dsel[slot] = dl;
  }
  wg_sync();
  double* e_v = a.ws_vec;
  double* au = a.ws_vec + ld;
  double* dots = lds + 2 * TILE * (TILE + 1);  // up to N2 dot products
  for (int c = 0; c < ncl; ++c) {
    const int j0 = cl_start[c], sz = cl_start[c + 1] - j0;
    if (sz == 2) continue;
    const int slot0 = pair_src[c], want = sz / 2;
    int found = 0;
    for (int jj = 0; jj < sz && found < want; ++jj) {
      const int col = ord[j0 + jj];
      for (int k = tid; k < N2; k += nt) e_v[k] = Ev[(long)k * ld + col];
      wg_sync();
      for (int pass = 0; pass < 2; ++pass) {
        const int nch = 2 * found;  // chosen columns of this cluster
        for (int q = wv; q < nch; q += nwv) {
          const int cc = q < found ? slot0 + q : nL + slot0 + (q - found);
          double s = 0.0;
          for (int k = lane; k < N2; k += 64) s += Om[(long)k * ld + cc] * e_v[k];
          for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
          if (lane == 0) dots[q] = s;
        }
        wg_sync();
        for (int k = tid; k < N2; k += nt) {
          double v = e_v[k];
          for (int q = 0; q < nch; ++q) {
            const int cc = q < found ? slot0 + q : nL + slot0 + (q - found);
            v -= dots[q] * Om[(long)k * ld + cc];
          }
          e_v[k] = v;
        }
        wg_sync();
      }
      double part = 0.0;
      for (int k = tid; k < N2; k += nt) part += e_v[k] * e_v[k];
      const double nrm = sqrt(wg_sum(part, red));
      if (nrm < 0.5) continue;
      for (int k = tid; k < N2; k += nt) e_v[k] /= nrm;
      wg_sync();
      for (int i = tid; i < N2; i += nt) {
        double s = 0.0;
        for (int k = 0; k < N2; ++k) s += Am[(long)i * ld + k] * e_v[k];
        au[i] = s;
      }
      wg_sync();
      part = 0.0;
      for (int k = tid; k < N2; k += nt) part += au[k] * au[k];
      const double dl = sqrt(wg_sum(part, red));
      const int slot = slot0 + found;
      for (int k = tid; k < N2; k += nt) {
        Om[(long)k * ld + slot] = e_v[k];
        Om[(long)k * ld + nL + slot] = -au[k] / dl;
      }
      if (tid == 0) dsel[slot] = dl;
      ++found;
      wg_sync();
    }
    if (found < want) {
      if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_WILLIAMSON);
      return;
    }
  }
  wg_sync();
  // pairs by D descending (stable): pair_src[rank] = slot
  for (int i = tid; i < nL; i += nt) {
    int rank = 0;
    for (int j = 0; j < nL; ++j) rank += (dsel[j] > dsel[i]) || (dsel[j] == dsel[i] && j < i);
    cl_start[rank] = i;
  }
  wg_sync();
  // O' = sorted pairs scaled by D^(-1/2); S = L O'
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    int k = (int)(e / N2), j = (int)(e % N2);
    int src = cl_start[j % nL];
    Op[(long)k * ld + j] = Om[(long)k * ld + src + (j >= nL ? nL : 0)] / sqrt(dsel[src]);
  }
  wg_sync();
  wg_dgemm(N2, N2, N2, 1.0, Lm, ld, false, Op, ld, false, 0.0, Sm, ld, tiles);
  if (tid == 0) {
    int ne = 0;
    for (int k = 0; k < nL; ++k) {
      double dv = dsel[cl_start[k]];
      a.dsym[(long)m * a.ld_dsym + k] = dv;
      a.lam[(long)m * a.ld_dsym + k] = dv > 1.0 ? sqrt((dv - 1.0) / (dv + 1.0)) : 0.0;
      if (dv >= a.dstar) ++ne;
    }
    if (ne > nR) ne = nR;
    a.ne[m] = (m == M) ? 0 : ne;
    flag = (m == M) ? 0 : ne;
  }
  wg_sync();
  const int ne = flag;
  // U, V from S (Eq. MUV)
  cplx64* U = a.ws_U;
  cplx64* V = a.ws_V;
  cplx64* Aug = a.ws_aug;
  const long ldu = a.ld_u;
  for (long e = tid; e < (long)nL * nL; e += nt) {
    int i = (int)(e / nL), j = (int)(e % nL);
    double s11 = Sm[(long)i * ld + j], s12 = Sm[(long)i * ld + nL + j];
    double s21 = Sm[(long)(nL + i) * ld + j], s22 = Sm[(long)(nL + i) * ld + nL + j];
    U[i * ldu + j] = cmake<cplx64>(0.5 * (s21 - s12), -0.5 * (s11 + s22));
    V[i * ldu + j] = cmake<cplx64>(0.5 * (-s12 - s21), -0.5 * (s11 - s22));
  }
  wg_sync();
  // (U^dag)^-1 by Gauss-Jordan with partial pivoting on [U^dag | I]
  for (long e = tid; e < (long)nL * 2 * nL; e += nt) {
    int i = (int)(e / (2 * nL)), j = (int)(e % (2 * nL));
    Aug[i * 2 * ldu + j] = j < nL ? cconj(U[(long)j * ldu + i]) : cmake<cplx64>(j - nL == i ? 1.0 : 0.0, 0.0);
  }
  wg_sync();
  __shared__ int piv_row;
  for (int col = 0; col < nL; ++col) {
    // pivot search by wave 0
    if (wv == 0) {
      double bv = -1.0;
      int best = col;
      for (int r = col + lane; r < nL; r += 64) {
        double v = cabs2(Aug[(long)r * 2 * ldu + col]);
        if (v > bv) { bv = v; best = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(bv, off, 64);
        int ob = __shfl_xor(best, off, 64);
        if (ov > bv || (ov == bv && ob < best)) { bv = ov; best = ob; }
      }
      if (lane == 0) {
        piv_row = best;
        bad = !(bv > 1e-280);
      }
    }
    wg_sync();
    if (bad) {
      if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_SINGULAR);
      return;
    }
    const int pr = piv_row;
    if (pr != col) {
      for (int j = tid; j < 2 * nL; j += nt) {
        cplx64 t = Aug[(long)col * 2 * ldu + j];
        Aug[(long)col * 2 * ldu + j] = Aug[(long)pr * 2 * ldu + j];
        Aug[(long)pr * 2 * ldu + j] = t;
      }
    }
    wg_sync();
    cplx64 pv = Aug[(long)col * 2 * ldu + col];
    double pn = cabs2(pv);
    cplx64 pinv = cmake<cplx64>(pv.re / pn, -pv.im / pn);
    wg_sync();
    for (int j = tid; j < 2 * nL; j += nt) Aug[(long)col * 2 * ldu + j] = cmul(Aug[(long)col * 2 * ldu + j], pinv);
    wg_sync();
    for (long e = tid; e < (long)nL * 2 * nL; e += nt) {
      int r = (int)(e / (2 * nL)), j = (int)(e % (2 * nL));
      if (r == col || j == col) continue;
      cplx64 f = Aug[(long)r * 2 * ldu + col];
      Aug[(long)r * 2 * ldu + j] = csub(Aug[(long)r * 2 * ldu + j], cmul(f, Aug[(long)col * 2 * ldu + j]));
    }
    wg_sync();
    for (int r = tid; r < nL; r += nt)
      if (r != col) Aug[(long)r * 2 * ldu + col] = cmake<cplx64>(0.0, 0.0);
    wg_sync();
  }
  // Q^m on (r_{m-1}, a_m, l_m): [[Uih V^dag, Uih[:, :ne]], [.^T, -V^T Uih]]
  const int nmod = nL + ne;
  cplx64* Q = a.Q + (long)(m - 1) * a.q_stride;
  const long ldq = a.ld_q;
  for (long e = tid; e < (long)nmod * nmod; e += nt) {
    int i = (int)(e / nmod), j = (int)(e % nmod);
    cplx64 s = cmake<cplx64>(0.0, 0.0);
    if (i < nL && j < nL) {
      for (int k = 0; k < nL; ++k) cfma(s, Aug[(long)i * 2 * ldu + nL + k], cconj(V[(long)j * ldu + k]));
    } else if (i < nL) {
      s = Aug[(long)i * 2 * ldu + nL + (j - nL)];
    } else if (j < nL) {
      s = Aug[(long)j * 2 * ldu + nL + (i - nL)];
    } else {
      int q1 = i - nL, q2 = j - nL;
      for (int k = 0; k < nL; ++k) cfma(s, V[(long)k * ldu + q1], Aug[(long)k * 2 * ldu + nL + q2]);
      s = cmake<cplx64>(-s.re, -s.im);
    }
    Q[(long)i * ldq + j] = s;
  }
  if (m == M) return;
  wg_sync();
  // Next residual.  T = -S^T Omega; T_act rows: x_b,q -> q, p_b,q -> nL + q.
  double* Ta = a.ws_A;   // reuse: T_act (2ne x N2)
  double* TG = a.ws_B;   // T_act Gamma_LL
  double* GLR = a.ws_glr;  // Gamma_{L,R} (N2 x 2 nR)
  for (long e = tid; e < (long)2 * ne * N2; e += nt) {
    int r = (int)(e / N2), c = (int)(e % N2);
    int rr = r < ne ? r : nL + (r - ne);
    Ta[(long)r * ld + c] = c < nL ? Sm[(long)(c + nL) * ld + rr] : -Sm[(long)(c - nL) * ld + rr];
  }
  for (long e = tid; e < (long)N2 * 2 * nR; e += nt) {
    int c = (int)(e / (2 * nR)), cc = (int)(e % (2 * nR));
    int gcol = cc < nR ? m + cc : M + m + (cc - nR);
    int ci = c % nL;
    bool cp = c >= nL;
    GLR[(long)c * a.ld_glr + cc] = ci < n_prev ? CR[(long)(cp ? n_prev + ci : ci) * ldc + gcol]
                                              : g[(long)(cp ? gpa : gxa) * n2g + gcol];
  }
  wg_sync();
  wg_dgemm(2 * ne, N2, N2, 1.0, Ta, ld, false, G, ld, false, 0.0, TG, ld, tiles);
  wg_sync();
  wg_dgemm(2 * ne, 2 * ne, N2, 1.0, TG, ld, false, Ta, ld, true, 0.0, a.drr_out, ldd, tiles);
  // CR' columns m..M-1 (x of a_{m+1..M}) and M+m..2M-1 (p)
  wg_dgemm(2 * ne, nR, N2, 1.0, Ta, ld, false, GLR, a.ld_glr, false, 0.0, a.cr_out + m, ldc, tiles);
  wg_dgemm(2 * ne, nR, N2, 1.0, Ta, ld, false, GLR + nR, a.ld_glr, false, 0.0, a.cr_out + M + m, ldc, tiles);
}

hipError_t launch_gsvd_cut(hipStream_t st, const GsvdArgs& a, int m, int n2max) {
  const size_t lds1 = sizeof(double) * ((size_t)GBS_GSVD_LDS_N2 * (GBS_GSVD_LDS_N2 + 1) / 2 + 2 * 32 * 33);
  hipLaunchKernelGGL(gsvd_stage1_kernel, dim3(1), dim3(1024), lds1, st, a, m);
  const int nblk = (n2max + GBS_GSVD_VROWS - 1) / GBS_GSVD_VROWS;
  const size_t lds2 = sizeof(double) * (size_t)GBS_GSVD_VROWS * n2max;
  hipLaunchKernelGGL(gsvd_vapply_kernel, dim3(nblk), dim3(256), lds2, st, a, m);
  const size_t lds3 = sizeof(double) * ((size_t)2 * 32 * 33 + GBS_GSVD_N2_MAX + 8);
  hipLaunchKernelGGL(gsvd_stage2_kernel, dim3(1), dim3(1024), lds3, st, a, m);
  return hipGetLastError();
}

hipError_t launch_validate(hipStream_t st, const double* gamma, int M, double* scal, double* wsM, int* err) {
  const int n2 = 2 * M;
  hipError_t e = hipMemsetAsync(scal, 0, 3 * sizeof(double), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(validate_sym_kernel, dim3(64), dim3(256), 0, st, gamma, n2, scal + 0, scal + 1);
  hipLaunchKernelGGL(purity_kernel, dim3((n2 + 15) / 16, (n2 + 15) / 16), dim3(256), 0, st, gamma, M, scal + 2);
  hipLaunchKernelGGL(chol_xx_kernel, dim3(1), dim3(1024), 0, st, gamma, M, wsM, err);
  return hipGetLastError();
}
