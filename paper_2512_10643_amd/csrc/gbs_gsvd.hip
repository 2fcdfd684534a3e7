// Input validation and the iterative Gaussian SVD (Sec. II.A-B, App. A), FP64.
//
// Cuts run in order on the stream because each consumes the residual the
// previous one produced.  Williamson form of the left block L = (r_{m-1}, a_m)
// (stage 1, one workgroup):
//   2 Gamma_LL = L L^T in closed form (the r modes are already in normal
//   form: sqrt(D) on their pairs, a 2x2 Cholesky for the new mode),
//   A = L^T Omega L formed entry by entry (pair entries +-D_k plus the new
//   mode's rank-2 term), reduced to skew-tridiagonal form by Householder
//   reflections; its singular values D are the positive eigenvalues of the
//   zero-diagonal symmetric tridiagonal matrix with the same off-diagonal,
//   found by Sturm-count bisection on each unreduced block; eigenvectors by
//   inverse iteration, orthonormalised within clusters of close eigenvalues;
//   their even and odd entries are the real Schur pairs (u, v), back-
//   transformed by the reflectors, and S = L [u.., v..] diag(D, D)^(-1/2).
// Stage 2 (a second workgroup, beside the next cut's stage 1): Bogoliubov
// matrices from Eq. MUV, the paired form of the local state from the
// regularised Q_L of App. A, and the next residual from the b-mode
// quadrature map T = -S^T Omega restricted to the active modes.
#include "gbs_gsvd.h"

#include <algorithm>


namespace {

__device__ inline void wg_sync() { __syncthreads(); }

// A count or flag that steers the whole workgroup, read as wave-uniform.  The
// batched kernels read their argument blocks from device memory, so a load
// through a pointer held there is a generic (flat) load, which the compiler
// must take as per-lane; the loops it bounds then become exec-masked loops.
// At the exit of one of them the register allocator placed copies of live
// values ahead of the exec restore, where they write no lane; that broke the
// Williamson step of the batched cut (a later orthogonality test compared
// i == j against a stale -n in every lane but the first).  Reading these
// values with readfirstlane keeps such loops scalar, as in the kernels that
// take their arguments by value.
__device__ inline int uniform_load(const int* p) { return __builtin_amdgcn_readfirstlane(*p); }

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

// Maximum of one value per thread, same protocol as wg_sum.
__device__ double wg_max(double x, double* red) {
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = x;
  wg_sync();
  double r = 0.0;
  if (tid == 0) {
    for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) r = fmax(r, red[i]);
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
// Gaussian SVD chain, two launches per cut (all sizes read from device state
// so the host enqueues every cut without synchronising):
//   stage 1 (one workgroup): Gamma_LL, Cholesky 2 Gamma_LL = L L^T, the
//            antisymmetric A = L^T Omega L, and the real Schur pairs of A:
//            Householder reduction A = Q T Q^T to skew-tridiagonal T; the
//            singular values D of A are the positive eigenvalues of the
//            symmetric tridiagonal G with T's off-diagonal and zero diagonal
//            (Golub-Kahan form), found by Sturm bisection; inverse iteration on
//            G gives z, and its even / odd entries (signs + + - - ...) give the
//            pair x_e, x_o with T x_e = D x_o, T x_o = -D x_e; back-transformed
//            by Q they are orthonormal eigenvectors of A^T A for D^2;
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

// packed strict lower triangle of an antisymmetric matrix: a(i, j) for i > j
__device__ inline long pk2(int i, int j) { return (long)i * (i - 1) / 2 + j; }


// Number of eigenvalues below x of the symmetric tridiagonal matrix with zero
// diagonal and squared off-diagonal t2[0..n-2] (Sturm sequence of the LDL^T
// pivots).  The division is a full IEEE division: a hardware reciprocal
// refined by Newton steps is not accurate enough here (near-degenerate
// Williamson values of a 1024-mode chain move by up to 1e-10 with it).
__device__ int sturm_below(const double* t2, int n, double x) {
  int cnt = 0;
  double d = -x;
  if (d < 0.0) ++cnt;
  for (int i = 1; i < n; ++i) {
    if (d == 0.0) d = 1e-300;
    d = -x - t2[i - 1] / d;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// Solve (G - s I) y = b in place (y holds b), G as in sturm_below, by
// Gaussian elimination with partial pivoting.  Interleaved storage: y[i] at
// y[i * ys], element i of scratch array a (0..3) at w[(a * n + i) * wsd].  Zero
// pivots are replaced by `tiny` (inverse iteration only needs a direction).
__device__ void tri_shift_solve_il(const double* t, int n, double s, double* y, long ys, double* w, long wsd,
                                   double tiny) {
  // forward elimination with the current row carried in registers; the final
  // pivot rows (diag, super, second super) go to the scratch arrays
  double* D = w;
  double* DU = w + (long)n * wsd;
  double* DU2 = w + 2L * n * wsd;
  double cd = -s, cdu = n > 1 ? t[0] : 0.0, cy = y[0];
  for (int i = 0; i + 1 < n; ++i) {
    const double tn = t[i], nd = -s, ndu = i + 2 < n ? t[i + 1] : 0.0, ny = y[(long)(i + 1) * ys];
    if (fabs(cd) >= fabs(tn)) {
      if (cd == 0.0) cd = tiny;
      const double f = tn / cd;
      D[(long)i * wsd] = cd;
      DU[(long)i * wsd] = cdu;
      DU2[(long)i * wsd] = 0.0;
      y[(long)i * ys] = cy;
      cd = nd - f * cdu;
      cdu = ndu;
      cy = ny - f * cy;
    } else {  // the next row becomes the pivot row
      const double f = cd / tn;
      D[(long)i * wsd] = tn;
      DU[(long)i * wsd] = nd;
      DU2[(long)i * wsd] = ndu;
      y[(long)i * ys] = ny;
      const double ed = cdu - f * nd, edu = -f * ndu, ey = cy - f * ny;
      cd = ed;
      cdu = edu;
      cy = ey;
    }
  }
  if (cd == 0.0) cd = tiny;
  // back substitution, the two later unknowns carried in registers
  double x2 = 0.0, x1 = cy / cd;
  y[(long)(n - 1) * ys] = x1;
  for (int i = n - 2; i >= 0; --i) {
    const double xi = (y[(long)i * ys] - DU[(long)i * wsd] * x1 - DU2[(long)i * wsd] * x2) / D[(long)i * wsd];
    y[(long)i * ys] = xi;
    x2 = x1;
    x1 = xi;
  }
}

}  // namespace

// Bogoliubov U, V of cut m from its S (Eq. MUV), (U^dag)^-1 and the pair
// matrix Q^m.  Nothing later in the chain reads these, so the workgroup that
// computes them for cut m runs beside the Williamson step of cut m + 1.
__device__ void q_from_s(const GsvdArgs& a, int m) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6;
  if (uniform_load(a.err)) return;
  const int nL = uniform_load(a.ne + (m - 1)) + 1;
  const int ne = uniform_load(a.ne + m);
  const long ld = a.ld_ws;
  const double* Sm = a.ws_S;
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
  __shared__ int piv_row, sing;
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
        sing = !(bv > 1e-280);
      }
    }
    wg_sync();
    if (sing) {
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
  cplx64* Q = a.Q + (long)(m - 1 - a.q_slot0) * a.q_stride;
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
}

// Stage 1.
__device__ void stage1_body(const GsvdArgs& a, int m) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int M = a.M;
  if (uniform_load(a.err)) return;
  const int n_prev = uniform_load(a.ne + (m - 1));
  const int nL = n_prev + 1, N2 = 2 * nL;
  if (N2 > GBS_GSVD_N2_MAX) {
    if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_KMAX);
    return;
  }
  extern __shared__ double lds[];
  __shared__ double vL[GBS_GSVD_N2_MAX], pL[GBS_GSVD_N2_MAX], part[1024], red[40];
  __shared__ double tL[GBS_GSVD_N2_MAX], tauL[GBS_GSVD_N2_MAX];
  __shared__ double sig0[GBS_GSVD_N2_MAX / 2], sigR[GBS_GSVD_N2_MAX / 2];
  __shared__ int first[GBS_GSVD_N2_MAX / 2];
  __shared__ int vblk[GBS_GSVD_N2_MAX / 2];  // block of the split tridiagonal form holding each sorted vector
  __shared__ int bad;
  const long ld = a.ld_ws;
  const bool in_lds = N2 <= GBS_GSVD_LDS_N2;
  double* P = in_lds ? lds : a.ws_pack;        // packed working matrix (Cholesky, then A)
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
  // A factor L with L L^T = 2 Gamma_LL.  The r block is the Williamson normal
  // form left by the previous cut (diagonal), so in the order (x_r, p_r, x_a,
  // p_a) the factor is [[sqrt(Dd), 0], [c^T Dd^-1/2, chol(h)]] with
  // h = g - c^T Dd^-1 c (2 x 2); its rows are stored back in the xxpp order
  // (any factor serves: the Williamson form only needs L L^T = 2 Gamma_LL).
  // A general Cholesky is used when the r block is not diagonal to 1e-13.
  const int nr = n_prev;
  auto orow = [&](int i) { return i < nr ? i : (i < 2 * nr ? nL + (i - nr) : (i == 2 * nr ? nL - 1 : 2 * nL - 1)); };
  double dmx = 0.0;
  for (int i = tid; i < 2 * nr; i += nt) dmx = fmax(dmx, fabs(G[(long)orow(i) * ld + orow(i)]));
  dmx = wg_max(dmx, red);
  if (tid == 0) bad = 0;
  wg_sync();
  for (long e = tid; e < 4L * nr * nr; e += nt) {
    const int i = (int)(e / (2 * nr)), j = (int)(e % (2 * nr));
    if (i != j && fabs(G[(long)orow(i) * ld + orow(j)]) > 1e-13 * dmx) bad = 1;
  }
  wg_sync();
  const bool structured = (bad == 0);
  wg_sync();
  if (structured) {
    for (long e = tid; e < (long)N2 * N2; e += nt) Lm[(long)(e / N2) * ld + (e % N2)] = 0.0;
    wg_sync();
    const int xa = nL - 1, pa = 2 * nL - 1;
    double h00 = 0.0, h01 = 0.0, h11 = 0.0;
    for (int i = tid; i < 2 * nr; i += nt) {
      const int o = orow(i);
      const double dd = 2.0 * G[(long)o * ld + o];
      const double c0 = 2.0 * G[(long)o * ld + xa], c1 = 2.0 * G[(long)o * ld + pa];
      if (dd > 0.0) {
        const double sd = sqrt(dd);
        Lm[(long)o * ld + i] = sd;
        Lm[(long)xa * ld + i] = c0 / sd;
        Lm[(long)pa * ld + i] = c1 / sd;
        h00 += c0 * c0 / dd;
        h01 += c0 * c1 / dd;
        h11 += c1 * c1 / dd;
      } else {
        bad = 2;
      }
    }
    h00 = 2.0 * G[(long)xa * ld + xa] - wg_sum(h00, red);
    h01 = 2.0 * G[(long)xa * ld + pa] - wg_sum(h01, red);
    h11 = 2.0 * G[(long)pa * ld + pa] - wg_sum(h11, red);
    if (tid == 0) {
      const double s00 = h00 > 0.0 ? sqrt(h00) : 0.0;
      const double s10 = s00 > 0.0 ? h01 / s00 : 0.0;
      const double r11 = h11 - s10 * s10;
      if (!(s00 > 0.0) || !(r11 > 0.0)) bad = 2;
      Lm[(long)xa * ld + 2 * nr] = s00;
      Lm[(long)pa * ld + 2 * nr] = s10;
      Lm[(long)pa * ld + 2 * nr + 1] = r11 > 0.0 ? sqrt(r11) : 0.0;
    }
    wg_sync();
    if (bad == 2) {
      if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_NOT_PD);
      return;
    }
  } else if (!in_lds) {
    // Cholesky by block columns of kCholB (right looking) when the packed
    // triangle lives in device memory: each block column is factored in LDS
    // (the dynamic LDS is free on this path), written back once, and the
    // trailing triangle takes its rank-kCholB update in one read and write,
    // instead of one per column.
    constexpr int kCholB = 16, kCP = kCholB + 1;  // block width, LDS row pitch
    double* pan = lds;  // rows J..N2-1 of block column J, row-major
    for (int J = 0; J < N2; J += kCholB) {
      const int jb = min(kCholB, N2 - J), nr = N2 - J;
      for (int e = tid; e < nr * jb; e += nt) {
        const int i = e / jb, c = e % jb;
        pan[i * kCP + c] = (i >= jb || c <= i) ? P[pk(J + i, J + c)] : 0.0;
      }
      wg_sync();
      for (int c = 0; c < jb; ++c) {
        if (tid == 0) {
          const double dj = pan[c * kCP + c];
          bad = !(dj > 0.0);
          pan[c * kCP + c] = dj > 0.0 ? sqrt(dj) : 1.0;
        }
        wg_sync();
        if (bad) {
          if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_NOT_PD);
          return;
        }
        const double piv = pan[c * kCP + c];
        for (int i = c + 1 + tid; i < nr; i += nt) pan[i * kCP + c] /= piv;
        wg_sync();
        // the block column's later columns t (rows i >= t)
        const int w2 = jb - c - 1;
        if (w2 > 0)
          for (int e = tid; e < (nr - c - 1) * w2; e += nt) {
            const int i = c + 1 + e / w2, t = c + 1 + e % w2;
            if (t <= i) pan[i * kCP + t] -= pan[i * kCP + c] * pan[t * kCP + c];
          }
        wg_sync();
      }
      for (int e = tid; e < nr * jb; e += nt) {
        const int i = e / jb, c = e % jb;
        if (i >= jb || c <= i) P[pk(J + i, J + c)] = pan[i * kCP + c];
      }
      // trailing triangle, a packed row per group of 32 lanes (contiguous in k)
      for (int i = jb + (tid >> 5); i < nr; i += nt >> 5) {
        double li[kCholB];
#pragma unroll
        for (int c = 0; c < kCholB; ++c) li[c] = c < jb ? pan[i * kCP + c] : 0.0;
        double* Pi = P + (long)(J + i) * (J + i + 1) / 2 + J;
        for (int k = jb + (tid & 31); k <= i; k += 32) {
          double acc = 0.0;
#pragma unroll
          for (int c = 0; c < kCholB; ++c)
            if (c < jb) acc = fma(li[c], pan[k * kCP + c], acc);
          Pi[k] -= acc;
        }
      }
      wg_sync();
    }
    for (long e = tid; e < (long)N2 * N2; e += nt) {
      int i = (int)(e / N2), j = (int)(e % N2);
      Lm[(long)i * ld + j] = j <= i ? P[pk(i, j)] : 0.0;
    }
  } else {
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
      // trailing update, a row of the packed triangle per group of 32 lanes
      // (row i is contiguous in k)
      for (int i = j + 1 + (tid >> 5); i < N2; i += nt >> 5) {
        const double lij = P[pk(i, j)];
        double* Pi = P + (long)i * (i + 1) / 2;
        for (int k = j + 1 + (tid & 31); k <= i; k += 32) Pi[k] -= lij * P[pk(k, j)];
      }
      wg_sync();
    }
    // L (full, row-major)
    for (long e = tid; e < (long)N2 * N2; e += nt) {
      int i = (int)(e / N2), j = (int)(e % N2);
      Lm[(long)i * ld + j] = j <= i ? P[pk(i, j)] : 0.0;
    }
  }
  // A = L^T Omega L = sum_k (x_k p_k^T - p_k x_k^T) over the rows x_k, p_k of
  // L (mode k).  With the structured factor, row x_k of an r mode has one
  // entry (column k, sx_k) and row p_k one (column nr + k, sp_k), so A is the
  // pair entries +-sx_k sp_k plus the rank-2 term of the new mode's rows; a
  // general factor goes through a product with W = Omega L.
  wg_sync();
  if (structured) {
    const double* Xa = Lm + (long)(nL - 1) * ld;
    const double* Pa = Lm + (long)(2 * nL - 1) * ld;
    for (long e = tid; e < (long)N2 * N2; e += nt) {
      const int i = (int)(e / N2), j = (int)(e % N2);
      double v = Xa[i] * Pa[j] - Pa[i] * Xa[j];
      if (i < nr && j == nr + i) v += Lm[(long)i * ld + i] * Lm[(long)(nL + i) * ld + j];
      if (j < nr && i == nr + j) v -= Lm[(long)j * ld + j] * Lm[(long)(nL + j) * ld + i];
      Am[(long)i * ld + j] = v;
    }
  } else {
    // W = Omega L: W_k = L_{k+nL} (k < nL), -L_{k-nL} (k >= nL).
    for (long e = tid; e < (long)N2 * N2; e += nt) {
      int k = (int)(e / N2), j = (int)(e % N2);
      W[(long)k * ld + j] = k < nL ? Lm[(long)(k + nL) * ld + j] : -Lm[(long)(k - nL) * ld + j];
    }
    wg_sync();
    wg_dgemm(N2, N2, N2, 1.0, Lm, ld, true, W, ld, false, 0.0, Am, ld, nullptr);
  }
  wg_sync();
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    const int i = (int)(e / N2), j = (int)(e % N2);
    if (i > j) P[pk2(i, j)] = 0.5 * (Am[(long)i * ld + j] - Am[(long)j * ld + i]);
  }
  wg_sync();
  double* Vh = a.ws_B;            // reflector k in row k (length N2 - k - 1)
  // Householder: column k of the trailing block -> beta e_1; A <- H A H keeps
  // A antisymmetric: A_sub += v p^T - p v^T with p = tau A_sub v.
  for (int k = 0; k + 2 < N2; ++k) {
    const int r = N2 - k - 1;
    // the reflector of column k by the first wave alone (its r entries are
    // reduced by shuffles), published with one barrier
    if (tid < 64) {
      double ss = 0.0, xf = 0.0;
      for (int i = tid; i < r; i += 64) {
        const double x = P[pk2(k + 1 + i, k)];
        if (i == 0) xf = x;
        vL[i] = x;
        ss += x * x;
      }
      for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
      const double x0 = __shfl(xf, 0, 64);
      const double alpha = sqrt(ss);
      const double beta = x0 > 0.0 ? -alpha : alpha;
      const double vtv = 2.0 * (ss - x0 * beta);
      const double tau = vtv > 0.0 ? 2.0 / vtv : 0.0;
      if (tid == 0) {
        vL[0] = x0 - beta;
        tauL[k] = tau;
        tL[k] = alpha > 0.0 ? beta : x0;
      }
    }
    wg_sync();
    const double tau = tauL[k];
    for (int i = tid; i < r; i += nt) Vh[(long)k * ld + i] = vL[i];
    // p = tau A_sub v: 32 threads per row, rows strided by nt / 32; the row's
    // part left of the diagonal is contiguous in the packed triangle, the part
    // right of it is read down its column with a sign change
    const int K1 = k + 1;
    for (int row = tid >> 5; row < r; row += nt >> 5) {
      const int gi = K1 + row;
      const double* Prow = P + (long)gi * (gi - 1) / 2 + K1;
      double acc = 0.0;
      for (int j = tid & 31; j < row; j += 32) acc += Prow[j] * vL[j];
      for (int j = row + 1 + (tid & 31); j < r; j += 32) {
        const int gj = K1 + j;
        acc -= P[(long)gj * (gj - 1) / 2 + gi] * vL[j];
      }
      for (int off = 16; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 32);
      if ((tid & 31) == 0) pL[row] = tau * acc;
    }
    wg_sync();
    for (int i = tid >> 5; i < r; i += nt >> 5) {
      const double vi = vL[i], pi = pL[i];
      double* Pi = P + pk2(k + 1 + i, k + 1);
      for (int j = tid & 31; j < i; j += 32) Pi[j] += vi * pL[j] - pi * vL[j];
    }
    wg_sync();
  }
  if (tid == 0) tL[N2 - 2] = P[pk2(N2 - 1, N2 - 2)];
  wg_sync();
  // positive eigenvalues of G by Sturm bisection (one thread each)
  double tm = 0.0;
  for (int i = tid; i < N2 - 1; i += nt) tm = fmax(tm, fabs(tL[i]));
  tm = wg_max(tm, red);
  // off-diagonal entries at the rounding level of the reduction split G into
  // independent blocks: set them to zero, or a tiny coupling mixes the null
  // vectors of blocks that share an eigenvalue (degenerate D) in the solves
  for (int i = tid; i < N2 - 1; i += nt)
    if (fabs(tL[i]) <= 2.2e-16 * N2 * tm) tL[i] = 0.0;
  wg_sync();
  const double bound = 2.0 * tm + 1e-300;
  const double tiny = 2.2e-16 * bound + 1e-300;
  const int n = nL;
  double* t2L = pL;  // squared off-diagonal for the Sturm counts (pL is free now)
  for (int i = tid; i < N2 - 1; i += nt) t2L[i] = tL[i] * tL[i];
  // Unreduced blocks of the split G.  Each even block of G (zero diagonal)
  // holds half of its eigenvalues above zero; eigenvalue q of the whole is
  // taken as eigenvalue k of its own block, and its vector is solved on that
  // block alone.  Equal eigenvalues of different blocks (modes in vacuum,
  // D = 1) then get vectors of disjoint support, which no solve over the
  // whole matrix can separate.  If a block is odd (a zero eigenvalue, which
  // a definite Gamma excludes) the whole matrix is taken as one block.
  int* bst = reinterpret_cast<int*>(part);  // block starts (part is free until the checks below)
  int* bpre = bst + 1024;                   // eigenvalues above zero before each block
  __shared__ int nblk;
  if (tid == 0) {
    int nb = 0, cnt = 0;
    bool even = true;
    bst[0] = 0;
    for (int i = 0; i < N2 - 1; ++i)
      if (tL[i] == 0.0) bst[++nb] = i + 1;
    bst[++nb] = N2;
    for (int b = 0; b < nb; ++b) {
      const int sz = bst[b + 1] - bst[b];
      bpre[b] = cnt;
      even = even && !(sz & 1);
      cnt += sz / 2;
    }
    bpre[nb] = cnt;
    if (!even || cnt != n) {
      nb = 1;
      bst[1] = N2;
      bpre[0] = 0;
      bpre[1] = n;
    }
    nblk = nb;
  }
  wg_sync();
  auto block_of = [&](int q) {  // the block holding eigenvalue q (bpre[b] <= q < bpre[b + 1])
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (bpre[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  // 8-section: the 8 lanes of a group test 8 interior points of the interval
  // at once (the Sturm count is monotone in x), so each round shrinks it 9x
  {
    const int grpi = tid >> 3, gl = tid & 7, ngrp = nt >> 3;
    const int sh = (threadIdx.x & 63) & ~7;  // first lane of this group in the wave
    for (int q0 = 0; q0 < n; q0 += ngrp) {
      const int q = q0 + grpi;
      const bool live = q < n;
      const int b = live ? block_of(q) : 0;
      const int b0 = bst[b], nbk = bst[b + 1] - b0, k = live ? q - bpre[b] : 0;
      double lo = 0.0, hi = bound;
      for (int it = 0; it < 17; ++it) {
        const double x = lo + (hi - lo) * (double)(gl + 1) / 9.0;
        const bool below = live && sturm_below(t2L + b0, nbk, x) <= nbk - 1 - k;
        const unsigned long long bal = __ballot(below);
        const int j = __popcll((bal >> sh) & 0xFFull);   // points at or below the target
        const double xl = __shfl(x, sh + (j > 0 ? j - 1 : 0), 64);
        const double xh = __shfl(x, sh + (j < 8 ? j : 7), 64);
        const double nlo = j > 0 ? xl : lo, nhi = j < 8 ? xh : hi;
        lo = nlo;
        hi = nhi;
      }
      if (live && gl == 0) sig0[q] = 0.5 * (lo + hi);
    }
  }
  wg_sync();
  // z_q as column q of Z (entry i at Z[i n + q]) and per-thread scratch with
  // the same interleaving, so a wave's threads touch consecutive addresses.
  // Two inverse-iteration solves per vector on its own block, all vectors at
  // once (one thread each); rows outside the block are zero.
  double* Z = a.ws_O;
  double* scr = a.ws_tri;
  for (int u = tid; u < n; u += nt) {
    const int b = block_of(u), b0 = bst[b], nbk = bst[b + 1] - b0;
    for (int i = 0; i < N2; ++i) Z[(long)i * n + u] = (i >= b0 && i < b0 + nbk) ? cos(0.7 * (u + 1) * i + 0.3) : 0.0;
    for (int it = 0; it < 2; ++it) {
      tri_shift_solve_il(tL + b0, nbk, sig0[u], Z + (long)b0 * n + u, n, scr + u, n, tiny);
      double nn = 0.0;
      for (int i = b0; i < b0 + nbk; ++i) nn += Z[(long)i * n + u] * Z[(long)i * n + u];
      const double inv = 1.0 / sqrt(nn);
      for (int i = b0; i < b0 + nbk; ++i) Z[(long)i * n + u] *= inv;
    }
  }
  wg_sync();
  // all eigenvalues in descending order (stable), vectors with them
  {
    double* Zs = a.ws_W;  // free here
    for (int u = tid; u < n; u += nt) {
      int r = 0;
      for (int v = 0; v < n; ++v) r += (sig0[v] > sig0[u]) || (sig0[v] == sig0[u] && v < u);
      first[u] = r;
    }
    wg_sync();
    for (long e = tid; e < (long)N2 * n; e += nt) {
      const int i = (int)(e / n), u = (int)(e % n);
      Zs[(long)i * n + first[u]] = Z[e];
    }
    for (int u = tid; u < n; u += nt) {
      sigR[first[u]] = sig0[u];
      vblk[first[u]] = block_of(u);
    }
    wg_sync();
    for (long e = tid; e < (long)N2 * n; e += nt) Z[e] = Zs[e];
    for (int u = tid; u < n; u += nt) sig0[u] = sigR[u];
    wg_sync();
  }
  // clusters of shifts closer than 1e-5 bound
  if (tid == 0) {
    first[0] = 0;
    for (int q = 1; q < n; ++q) first[q] = (sig0[q - 1] - sig0[q] < 1e-5 * bound) ? first[q - 1] : q;
  }
  wg_sync();
  // The members of a cluster are orthonormalised in order by one wave
  // (modified Gram-Schmidt): their solves resolve directions whose
  // eigenvalues are further apart than the shifts' error, and within a
  // degenerate set any orthonormal basis is an eigenbasis.  Members from
  // different blocks of the split form have disjoint support, so their
  // products are exact zeros and are skipped (the vacuum modes of a start
  // from Gamma form one large cluster spread over many blocks).
  {
    const int lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
    auto wave_sum = [&](double x) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      return x;
    };
    for (int q = wv; q < n; q += nwv) {
      if (first[q] != q || q + 1 >= n || first[q + 1] != q) continue;  // singletons need nothing
      int qe = q + 1;
      while (qe < n && first[qe] == q) ++qe;
      for (int u = q; u < qe; ++u) {
        for (int v2 = q; v2 < u; ++v2) {
          if (vblk[v2] != vblk[u]) continue;
          double c = 0.0;
          for (int i = lane; i < N2; i += 64) c += Z[(long)i * n + v2] * Z[(long)i * n + u];
          c = wave_sum(c);
          for (int i = lane; i < N2; i += 64) Z[(long)i * n + u] -= c * Z[(long)i * n + v2];
        }
        double nn = 0.0;
        for (int i = lane; i < N2; i += 64) nn += Z[(long)i * n + u] * Z[(long)i * n + u];
        const double inv = 1.0 / sqrt(wave_sum(nn));
        for (int i = lane; i < N2; i += 64) Z[(long)i * n + u] *= inv;
      }
    }
  }
  wg_sync();
  for (int u = tid; u < n; u += nt) {
    double rq = 0.0;  // Rayleigh quotient z^T G z
    for (int i = 0; i + 1 < N2; ++i) rq += 2.0 * tL[i] * Z[(long)i * n + u] * Z[(long)i * n + u + n];
    sigR[u] = fabs(rq);
  }
  wg_sync();
  // Check Z^T Z = 1; if the solves left a vector mixed (close eigenvalues in
  // different blocks), re-orthogonalise all of them in order (modified
  // Gram-Schmidt against the accurate earlier vectors restores it).
  {
    double* Gz = a.ws_W;  // n x n (W is free here; S of the previous cut is still read)
    wg_dgemm(n, n, N2, 1.0, Z, n, true, Z, n, false, 0.0, Gz, ld, nullptr);
    wg_sync();
    double dev = 0.0;
    for (long e = tid; e < (long)n * n; e += nt) {
      const int i = (int)(e / n), j = (int)(e % n);
      dev = fmax(dev, fabs(Gz[(long)i * ld + j] - (i == j ? 1.0 : 0.0)));
    }
    dev = wg_max(dev, red);
    if (dev > 1e-10) {
      for (int q = 0; q < n; ++q) {
        for (int rr = tid; rr < q; rr += nt) {
          double c = 0.0;
          for (int i = 0; i < N2; ++i) c += Z[(long)i * n + rr] * Z[(long)i * n + q];
          part[rr] = c;
        }
        wg_sync();
        double nn = 0.0;
        for (int i = tid; i < N2; i += nt) {
          double z = Z[(long)i * n + q];
          for (int rr = 0; rr < q; ++rr) z -= part[rr] * Z[(long)i * n + rr];
          Z[(long)i * n + q] = z;
          nn += z * z;
        }
        nn = wg_sum(nn, red);
        const double inv = 1.0 / sqrt(nn);
        for (int i = tid; i < N2; i += nt) Z[(long)i * n + q] *= inv;
        wg_sync();
        if (tid == 0) {
          double rq = 0.0;
          for (int i = 0; i + 1 < N2; ++i) rq += 2.0 * tL[i] * Z[(long)i * n + q] * Z[(long)(i + 1) * n + q];
          sigR[q] = fabs(rq);
        }
        wg_sync();
      }
    }
  }
  // U = Q X_e with X_e column q = sqrt2 (even entries of z_q, signs + + - - ..),
  // kept in LDS (the packed A is no longer needed): column q at XU[q N2 + i].
  // Reflectors are applied last to first, each by all threads: G threads per
  // column form the dot product v^T x, then update their share of rows.
  double* XU = in_lds && (long)n * N2 <= (long)GBS_GSVD_LDS_N2 * (GBS_GSVD_LDS_N2 + 1) / 2 ? lds : a.ws_W;
  for (long e = tid; e < (long)n * N2; e += nt) {
    const int q = (int)(e / N2), i = (int)(e % N2);
    const double sg = ((i >> 1) & 1) ? -1.41421356237309515 : 1.41421356237309515;
    XU[e] = (i & 1) ? 0.0 : sg * Z[(long)i * n + q];
  }
  // With the columns in LDS and room beside them, a column belongs to an
  // aligned group of Gp lanes of one wave and each lane to a fixed set of
  // rows (i = g mod Gp), so a reflector needs no barrier: the dot product is
  // reduced by shuffles within the group and every lane updates only its own
  // rows.  The reflectors are staged into LDS a few at a time (two barriers
  // per group).  When U lives in device memory (wide blocks), the columns go
  // through LDS in chunks that leave room for 8 staged reflectors, each chunk
  // taking every reflector (the columns are independent).
  const long lds_cap = (long)GBS_GSVD_LDS_N2 * (GBS_GSVD_LDS_N2 + 1) / 2;
  int nst = XU == lds ? (int)min(8L, (lds_cap - (long)n * N2) / N2) : 0;
  int nc = n;
  if (XU != lds) {
    const int room = (int)(lds_cap / N2) - 8;  // columns per chunk
    if (room >= 1) {
      const int np = (n + room - 1) / room;
      nc = (n + np - 1) / np;
      nst = 8;
    }
  }
  if (nst >= 2 && nc <= nt) {
    for (int q0 = 0; q0 < n; q0 += nc) {
      const int ncc = min(nc, n - q0);
      if (XU != lds) {
        wg_sync();
        for (long e = tid; e < (long)ncc * N2; e += nt) lds[e] = XU[(long)q0 * N2 + e];
      }
      int Gp = 64;
      while (Gp > 1 && Gp * ncc > nt) Gp >>= 1;
      const int cq = tid / Gp, gq = tid % Gp;
      double* VS = lds + (long)ncc * N2;  // staged reflectors, slot s at VS[s N2 + j]
      double* xc = lds + (long)cq * N2;
      for (int kb = N2 - 3; kb >= 0; kb -= nst) {
        const int kl = max(0, kb - nst + 1);
        wg_sync();
        for (int e = tid; e < (kb - kl + 1) * N2; e += nt) {
          const int sl = e / N2, j = e % N2, k = kb - sl;
          VS[e] = j < N2 - k - 1 ? Vh[(long)k * ld + j] : 0.0;
        }
        wg_sync();
        if (cq < ncc) {
          for (int k = kb; k >= kl; --k) {
            const double* v = VS + (long)(kb - k) * N2 - (k + 1);  // v[i]: entry of row i
            const int i0 = k + 1 <= gq ? gq : gq + (k + 1 - gq + Gp - 1) / Gp * Gp;
            double acc = 0.0;
            for (int i = i0; i < N2; i += Gp) acc += v[i] * xc[i];
            for (int off = Gp >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            const double w = acc * tauL[k];
            for (int i = i0; i < N2; i += Gp) xc[i] -= w * v[i];
          }
        }
      }
      if (XU != lds) {
        wg_sync();
        for (long e = tid; e < (long)ncc * N2; e += nt) XU[(long)q0 * N2 + e] = lds[e];
      }
    }
  } else {
    const int Gp = max(1, nt / n);
    const int cq = tid / Gp, gq = tid % Gp;
    for (int k = N2 - 3; k >= 0; --k) {
      const int r = N2 - k - 1;
      wg_sync();
      for (int i = tid; i < r; i += nt) vL[i] = Vh[(long)k * ld + i];
      wg_sync();
      double acc = 0.0;
      if (cq < n)
        for (int i = gq; i < r; i += Gp) acc += vL[i] * XU[(long)cq * N2 + k + 1 + i];
      part[tid] = acc;
      wg_sync();
      if (cq < n) {
        double w = 0.0;
        for (int g2 = 0; g2 < Gp; ++g2) w += part[cq * Gp + g2];
        w *= tauL[k];
        for (int i = gq; i < r; i += Gp) XU[(long)cq * N2 + k + 1 + i] -= w * vL[i];
      }
    }
  }
  wg_sync();
  // E: column 2q = u_q, column 2q + 1 = A u_q / D_q (the partner in the plane)
  double* Uc = a.ws_O;   // U (N2 x n); z is no longer needed
  double* AU = a.ws_B;   // A U; the reflectors are no longer needed
  for (long e = tid; e < (long)n * N2; e += nt) {
    const int q = (int)(e / N2), i = (int)(e % N2);
    a.ws_E[(long)i * ld + 2 * q] = XU[e];
    Uc[(long)i * ld + q] = XU[e];
  }
  wg_sync();
  wg_dgemm(N2, n, N2, 1.0, Am, ld, false, Uc, ld, false, 0.0, AU, ld, nullptr);
  wg_sync();
  for (long e = tid; e < (long)n * N2; e += nt) {
    const int i = (int)(e / n), q = (int)(e % n);
    a.ws_E[(long)i * ld + 2 * q + 1] = AU[(long)i * ld + q] / sigR[q];
  }
  // eigenvalues of A^T A (D^2, each twice), already in descending order
  for (int c = tid; c < N2; c += nt) {
    const double sgm = sigR[c >> 1];
    a.ws_w[c] = sgm * sgm;
    a.ws_ord[c] = c;
  }
}

__global__ __launch_bounds__(1024) void gsvd_stage1_kernel(GsvdArgs a, int m) {
  if (blockIdx.x == 1) {  // Q^{m-1} beside the Williamson step of cut m
    if (m - 1 >= a.q_first) q_from_s(a, m - 1);
    return;
  }
  stage1_body(a, m);
}

// Stage 2.
__device__ void stage2_body(const GsvdArgs& a, int m) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
  const int M = a.M;
  if (uniform_load(a.err)) return;
  const int n_prev = uniform_load(a.ne + (m - 1));
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
  const double* AU = a.ws_B;   // A u_q from stage 1, column q
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
  // (stage 1 gives the eigenvectors in pairs: column 2q = u_q, and a pair's
  // two equal eigenvalues are never split between clusters, so a two-vector
  // cluster starts at an even column and A u_q is column q of AU)
  for (int c = wv; c < ncl; c += nwv) {
    const int j0 = cl_start[c], sz = cl_start[c + 1] - j0;
    if (sz != 2) continue;
    const int col = ord[j0], slot = pair_src[c];
    if (col & 1) {
      if (lane == 0) bad = 1;
      continue;
    }
    const double* au_q = AU + (col >> 1);
    double s = 0.0;
    for (int k = lane; k < N2; k += 64) s += au_q[(long)k * ld] * au_q[(long)k * ld];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const double dl = sqrt(s);
    for (int k = lane; k < N2; k += 64) {
      Om[(long)k * ld + slot] = Ev[(long)k * ld + col];
      Om[(long)k * ld + nL + slot] = -au_q[(long)k * ld] / dl;
    }
    if (lane == 0) dsel[slot] = dl;
  }
  wg_sync();
  if (bad) {
    if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_WILLIAMSON);
    return;
  }
  double* e_v = a.ws_vec;
  double* au = a.ws_vec + ld;
  double* dots = lds + 2 * TILE * (TILE + 1);  // up to N2 dot products
  // A cut whose pair matrix is not formed (the first cut of a single-site
  // build) needs only its active pairs: the next residual takes the active
  // columns of S alone, so a cluster of vacuum modes (D below D*) keeps zero
  // columns there instead of a Gram-Schmidt pairing of the whole cluster.
  const bool pair_vacuum = m >= a.q_first;
  for (int c = 0; c < ncl; ++c) {
    const int j0 = cl_start[c], sz = cl_start[c + 1] - j0;
    if (sz == 2) continue;
    const int slot0 = pair_src[c], want = sz / 2;
    if (!pair_vacuum && w[ord[j0]] < a.dstar * a.dstar) {
      for (long e = tid; e < (long)N2 * want; e += nt) {
        const int k = (int)(e / want), q = (int)(e % want);
        Om[(long)k * ld + slot0 + q] = 0.0;
        Om[(long)k * ld + nL + slot0 + q] = 0.0;
      }
      for (int q = tid; q < want; q += nt) dsel[slot0 + q] = 1.0;
      wg_sync();
      continue;
    }
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
  if (m == M) return;  // the last site's Q^M is computed from S by q_from_s
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

__global__ __launch_bounds__(1024) void gsvd_stage2_kernel(GsvdArgs a, int m) { stage2_body(a, m); }

__global__ __launch_bounds__(1024) void gsvd_q_kernel(GsvdArgs a, int m) { q_from_s(a, m); }

// ---- every site on its own: element y of a batch runs its own cut cuts[y]
// (0: nothing) with its own arguments and workspaces.
__global__ __launch_bounds__(1024) void gsvd_stage1_batch_kernel(const GsvdArgs* __restrict__ args,
                                                                 const int* __restrict__ cuts) {
  const int m = cuts[blockIdx.y];
  if (m <= 0) return;
  const GsvdArgs a = args[blockIdx.y];
  stage1_body(a, m);
}

__global__ __launch_bounds__(1024) void gsvd_stage2_batch_kernel(const GsvdArgs* __restrict__ args,
                                                                 const int* __restrict__ cuts) {
  const int m = cuts[blockIdx.y];
  if (m <= 0) return;
  const GsvdArgs a = args[blockIdx.y];
  stage2_body(a, m);
}

__global__ __launch_bounds__(1024) void gsvd_q_batch_kernel(const GsvdArgs* __restrict__ args,
                                                            const int* __restrict__ cuts) {
  const int m = cuts[blockIdx.y];
  if (m <= 0) return;
  const GsvdArgs a = args[blockIdx.y];
  q_from_s(a, m);
}

// Start from Gamma at cut k = cuts[y] (>= 2): Gamma's rows of a_1..a_{k-1}
// into the element's drr_in / cr_in (as gsvd_restart_kernel).
__global__ void gsvd_restart_batch_kernel(const GsvdArgs* __restrict__ args, const int* __restrict__ cuts) {
  const int k = cuts[blockIdx.y];
  if (k < 2) return;
  const GsvdArgs& a = args[blockIdx.y];
  const int M = a.M, nr = k - 1, n2r = 2 * nr, n2g = 2 * M;
  double* drr = const_cast<double*>(a.drr_in);
  double* cr = const_cast<double*>(a.cr_in);
  const double* g = a.gamma;
  const long tot_c = (long)n2r * n2g, tot = tot_c + (long)n2r * n2r;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    if (e < tot_c) {
      const int i = (int)(e / n2g), c = (int)(e % n2g);
      const int gi = i < nr ? i : M + (i - nr);
      cr[(long)i * a.ld_cr + c] = g[(long)gi * n2g + c];
    } else {
      const long f = e - tot_c;
      const int i = (int)(f / n2r), j = (int)(f % n2r);
      const int gi = i < nr ? i : M + (i - nr), gj = j < nr ? j : M + (j - nr);
      drr[(long)i * a.ld_drr + j] = g[(long)gi * n2g + gj];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ne[k - 1] = nr;
}

// Keep the b-mode map rows of the element's first cut (active rows, left in
// ws_A by stage 2) before the second cut overwrites the workspace.
__global__ void gsvd_keep_map_batch_kernel(const GsvdArgs* __restrict__ args, const int* __restrict__ cuts,
                                           double* const* __restrict__ dst, const long* __restrict__ ld_dst) {
  const int k = cuts[blockIdx.y];
  if (k <= 0) return;
  const GsvdArgs& a = args[blockIdx.y];
  if (uniform_load(a.err)) return;
  const int ne = uniform_load(a.ne + k), n2 = 2 * (uniform_load(a.ne + (k - 1)) + 1);
  double* out = dst[blockIdx.y];
  const long ldo = ld_dst[blockIdx.y];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < 2L * ne * n2; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e / n2), c = (int)(e % n2);
    out[(long)r * ldo + c] = a.ws_A[(long)r * a.ld_ws + c];
  }
}

// Align the bond modes of cut m between site m (its chain step) and site
// m+1 (its start from Gamma), and put the phases into Q^m: for each active
// mode q, the rows of the step's b-mode map written on the quadratures of
// a_1..a_m (through the start map of cut m-1, which defines r_{m-1}) times
// the inverse of the start map of cut m is a rotation of the mode's (x, p)
// pair by theta_q; l_q's row and column of Q^m take e^{i theta_q}.
__global__ __launch_bounds__(256) void gsvd_align_kernel(const GsvdAlign* __restrict__ al, int* err) {
  const GsvdAlign A = al[blockIdx.x];
  const int m = A.m, k = m - 1;
  const int n0 = uniform_load(A.ne_e + (m - 1)), n = uniform_load(A.ne_e + m), nl = n0 + 1;
  // (no early exit on *err: another block may set it while this one runs,
  // and every wave of the block must reach the barrier below)
  if (uniform_load(A.ne_r + m) != n) {
    if (threadIdx.x == 0) gbs_set_error(err, GBS_DEVERR_ALIGN);
    return;
  }
  if (n > GBS_GSVD_N2_MAX / 2) {
    if (threadIdx.x == 0) gbs_set_error(err, GBS_DEVERR_KMAX);
    return;
  }
  __shared__ double th_s[GBS_GSVD_N2_MAX / 2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  cplx64* Q = A.Q;
  // F row i (quadratures of r_{m-1} and a_m) on a_1..a_m, column j in [0, 2m)
  auto frow = [&](int i, int j) -> double {
    const int jx = j < m ? j : j - m;   // mode of column j
    const bool jp = j >= m;
    if (i == n0) return (!jp && jx == m - 1) ? 1.0 : 0.0;           // x of a_m
    if (i == 2 * nl - 1) return (jp && jx == m - 1) ? 1.0 : 0.0;    // p of a_m
    if (jx == m - 1) return 0.0;
    const int r = i < n0 ? i : n0 + (i - nl);                       // row of the start map
    return A.t0[(long)r * A.ldt0 + (jp ? k + jx : jx)];
  };
  for (int q = wv; q < n; q += nwv) {
    // omega(v_x, tr_p), omega(v_x, tr_x), omega(v_p, tr_p), omega(v_p, tr_x)
    double o[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = lane; j < m; j += 64) {
      // v[j] and v[m + j] for v = step rows x_q and p_q times F
      double vx0 = 0.0, vx1 = 0.0, vp0 = 0.0, vp1 = 0.0;
      for (int i = 0; i < 2 * nl; ++i) {
        const double f0 = frow(i, j), f1 = frow(i, m + j);
        const double tx = A.t1[(long)q * A.ldt1 + i], tp = A.t1[(long)(n + q) * A.ldt1 + i];
        vx0 += tx * f0;
        vx1 += tx * f1;
        vp0 += tp * f0;
        vp1 += tp * f1;
      }
      const double rx0 = A.tr[(long)q * A.ldtr + j], rx1 = A.tr[(long)q * A.ldtr + m + j];
      const double rp0 = A.tr[(long)(n + q) * A.ldtr + j], rp1 = A.tr[(long)(n + q) * A.ldtr + m + j];
      o[0] += vx0 * rp1 - vx1 * rp0;
      o[1] += vx0 * rx1 - vx1 * rx0;
      o[2] += vp0 * rp1 - vp1 * rp0;
      o[3] += vp0 * rx1 - vp1 * rx0;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      for (int off = 32; off > 0; off >>= 1) o[t] += __shfl_xor(o[t], off, 64);
    // R = [[o0, -o1], [o2, -o3]]
    if (lane == 0) th_s[q] = atan2(o[2] + o[1], o[0] - o[3]);
  }
  __syncthreads();
  // Q_ij *= e^{i (theta_i + theta_j)}, theta = 0 off the l modes: every entry
  // is scaled once, by one thread (row and column l_q in place would have two
  // waves update the entry of two l modes at the same time)
  const int nmod = nl + n;
  for (long e = threadIdx.x; e < (long)nmod * nmod; e += blockDim.x) {
    const int i = (int)(e / nmod), j = (int)(e % nmod);
    const double th = (i >= nl ? th_s[i - nl] : 0.0) + (j >= nl ? th_s[j - nl] : 0.0);
    if (th != 0.0) Q[(long)i * A.ld_q + j] = cmul(Q[(long)i * A.ld_q + j], cmake<cplx64>(cos(th), sin(th)));
  }
}

hipError_t launch_gsvd_cut(hipStream_t st, const GsvdArgs& a, int m, int n2max) {
  (void)n2max;
  const size_t lds1 = sizeof(double) * ((size_t)GBS_GSVD_LDS_N2 * (GBS_GSVD_LDS_N2 + 1) / 2);
  hipLaunchKernelGGL(gsvd_stage1_kernel, dim3(m >= 2 ? 2 : 1), dim3(1024), lds1, st, a, m);
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

hipError_t launch_gsvd_last_q(hipStream_t st, const GsvdArgs& a) {
  hipLaunchKernelGGL(gsvd_q_kernel, dim3(1), dim3(1024), 0, st, a, a.M);
  return hipGetLastError();
}

hipError_t launch_gsvd_q(hipStream_t st, const GsvdArgs& a, int m) {
  hipLaunchKernelGGL(gsvd_q_kernel, dim3(1), dim3(1024), 0, st, a, m);
  return hipGetLastError();
}

// Rows of Gamma for the quadratures (x_1..x_{k-1}, p_1..p_{k-1}): the r-r
// block (columns in the same order) into drr_in and whole rows into cr_in.
__global__ void gsvd_restart_kernel(const double* g, int M, int k, double* drr, long ldd, double* cr, long ldc,
                                    int* ne) {
  const int nr = k - 1, n2r = 2 * nr, n2g = 2 * M;
  const long tot_c = (long)n2r * n2g, tot = tot_c + (long)n2r * n2r;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    if (e < tot_c) {
      const int i = (int)(e / n2g), c = (int)(e % n2g);
      const int gi = i < nr ? i : M + (i - nr);
      cr[(long)i * ldc + c] = g[(long)gi * n2g + c];
    } else {
      const long f = e - tot_c;
      const int i = (int)(f / n2r), j = (int)(f % n2r);
      const int gi = i < nr ? i : M + (i - nr), gj = j < nr ? j : M + (j - nr);
      drr[(long)i * ldd + j] = g[(long)gi * n2g + gj];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ne[k - 1] = nr;
}

hipError_t launch_gsvd_restart(hipStream_t st, const GsvdArgs& a, int k) {
  if (k < 1 || k > a.M || 2L * k > a.ld_drr) return hipErrorInvalidValue;
  const long tot = (long)(2 * (k - 1)) * (2 * a.M + 2 * (k - 1));
  const int blocks = (int)std::max<long>(1, std::min<long>(1024, (tot + 255) / 256));
  // drr_in / cr_in are read-only inputs of the cut kernels; the restart
  // writes the buffers that the next cut will read through them
  hipLaunchKernelGGL(gsvd_restart_kernel, dim3(blocks), dim3(256), 0, st, a.gamma, a.M, k,
                     const_cast<double*>(a.drr_in), a.ld_drr, const_cast<double*>(a.cr_in), a.ld_cr, a.ne);
  return hipGetLastError();
}

__global__ void reverse_modes_kernel(const double* g, int M, double* out) {
  const long n2 = 2L * M;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n2 * n2; e += (long)gridDim.x * blockDim.x) {
    const long i = e / n2, j = e % n2;
    const long si = i < M ? M - 1 - i : 3L * M - 1 - i, sj = j < M ? M - 1 - j : 3L * M - 1 - j;
    out[e] = g[si * n2 + sj];
  }
}

hipError_t launch_reverse_modes(hipStream_t st, const double* gamma, int M, double* out) {
  const long tot = 4L * M * M;
  const int blocks = (int)std::max<long>(1, std::min<long>(4096, (tot + 255) / 256));
  hipLaunchKernelGGL(reverse_modes_kernel, dim3(blocks), dim3(256), 0, st, gamma, M, out);
  return hipGetLastError();
}

// 32 x 32 tiles of one physical index p through LDS, so that both the reads
// (along b) and the writes (along a) are contiguous.
__global__ __launch_bounds__(256) void transpose_bonds_kernel(const cplx64* in, long A, int d, long B, cplx64* out) {
  __shared__ cplx64 tile[32][33];
  const int p = blockIdx.z;
  const long a0 = (long)blockIdx.y * 32, b0 = (long)blockIdx.x * 32;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const long a = a0 + r, b = b0 + threadIdx.x;
    if (a < A && b < B) tile[r][threadIdx.x] = in[(a * d + p) * B + b];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) {
    const long b = b0 + r, a = a0 + threadIdx.x;
    if (a < A && b < B) out[(b * d + p) * A + a] = tile[threadIdx.x][r];
  }
}

hipError_t launch_transpose_bonds(hipStream_t st, const cplx64* in, long A, int d, long B, cplx64* out) {
  if (A < 1 || B < 1 || d < 1 || (B + 31) / 32 > 0x7fffffffL || (A + 31) / 32 > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_bonds_kernel, dim3((unsigned)((B + 31) / 32), (unsigned)((A + 31) / 32), d), dim3(32, 8),
                     0, st, in, A, d, B, out);
  return hipGetLastError();
}

hipError_t launch_gsvd_independent(hipStream_t st, const GsvdArgs* args0, const GsvdArgs* args1, const int* cut0,
                                   const int* cut1, int nel, double* const* keep_dst, const long* keep_ld,
                                   const GsvdAlign* al, int nalign, int* err) {
  if (nel <= 0) return hipSuccess;
  const size_t lds1 = sizeof(double) * ((size_t)GBS_GSVD_LDS_N2 * (GBS_GSVD_LDS_N2 + 1) / 2);
  const size_t lds3 = sizeof(double) * ((size_t)2 * 32 * 33 + GBS_GSVD_N2_MAX + 8);
  const dim3 one(1, (unsigned)nel), many(64, (unsigned)nel);
  // first cut of every element: from Gamma at cut m - 1 (or the first cut)
  hipLaunchKernelGGL(gsvd_restart_batch_kernel, many, dim3(256), 0, st, args0, cut0);
  hipLaunchKernelGGL(gsvd_stage1_batch_kernel, one, dim3(1024), lds1, st, args0, cut0);
  hipLaunchKernelGGL(gsvd_stage2_batch_kernel, one, dim3(1024), lds3, st, args0, cut0);
  hipLaunchKernelGGL(gsvd_keep_map_batch_kernel, many, dim3(256), 0, st, args0, cut0, keep_dst, keep_ld);
  // second cut: the step that gives each site's right bond and Q^m
  hipLaunchKernelGGL(gsvd_stage1_batch_kernel, one, dim3(1024), lds1, st, args1, cut1);
  hipLaunchKernelGGL(gsvd_stage2_batch_kernel, one, dim3(1024), lds3, st, args1, cut1);
  hipLaunchKernelGGL(gsvd_q_batch_kernel, one, dim3(1024), 0, st, args1, cut1);
  if (nalign > 0) hipLaunchKernelGGL(gsvd_align_kernel, dim3((unsigned)nalign), dim3(256), 0, st, al, err);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void q_compact_kernel(const cplx64* __restrict__ src, long q_stride, long ld_q,
                                                        int slot0, const int* __restrict__ site,
                                                        const int* __restrict__ nn, const long* __restrict__ dst_off,
                                                        cplx64* __restrict__ dst) {
  const int m = site[blockIdx.x], n = nn[blockIdx.x];
  const cplx64* q = src + (long)(m - 1 - slot0) * q_stride;
  cplx64* o = dst + dst_off[blockIdx.x];
  for (long e = threadIdx.x; e < (long)n * n; e += blockDim.x) o[e] = q[(e / n) * ld_q + e % n];
}

hipError_t launch_q_compact(hipStream_t st, const cplx64* src, long q_stride, long ld_q, int slot0, const int* site,
                            const int* n, const long* dst_off, int nsites, cplx64* dst) {
  if (nsites <= 0) return hipSuccess;
  hipLaunchKernelGGL(q_compact_kernel, dim3((unsigned)nsites), dim3(256), 0, st, src, q_stride, ld_q, slot0, site, n,
                     dst_off, dst);
  return hipGetLastError();
}

__global__ void gsvd_gather_cuts_kernel(const GsvdArgs* __restrict__ args, int M, int* __restrict__ ne_out,
                                        double* __restrict__ lam_out, long ld_out) {
  const int m = blockIdx.x + 1;  // cut m, from site m's second cut
  if (m >= M) return;
  const GsvdArgs& a = args[m - 1];
  const int ne = uniform_load(a.ne + m);
  if (threadIdx.x == 0) ne_out[m] = ne;
  for (int q = threadIdx.x; q < ne && q < ld_out; q += blockDim.x) lam_out[(long)m * ld_out + q] = a.lam[(long)m * a.ld_dsym + q];
}

hipError_t launch_gsvd_gather_cuts(hipStream_t st, const GsvdArgs* args, int M, int* ne_out, double* lam_out,
                                   long ld_out) {
  if (M < 2) return hipSuccess;
  hipLaunchKernelGGL(gsvd_gather_cuts_kernel, dim3((unsigned)(M - 1)), dim3(64), 0, st, args, M, ne_out, lam_out,
                     ld_out);
  return hipGetLastError();
}
