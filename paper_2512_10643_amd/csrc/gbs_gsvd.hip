// Input validation and the iterative Gaussian SVD (Sec. II.A-B, App. A), FP64.
//
// One 1024-thread workgroup handles one cut; cuts run in order on the
// stream because each consumes the residual the previous one produced.
// Williamson form of the left block L = (r_{m-1}, a_m):
//   2 Gamma_LL = L L^T (Cholesky), A = L^T Omega L (antisymmetric),
//   B = A^T A (symmetric, eigenvalues D_q^2 twice) by Jacobi rotations,
//   symplectic pairs (u, v = -A u / D) by Gram-Schmidt over the sorted
//   eigenvectors, S = L [u.., v..] diag(D, D)^(-1/2).
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

// Real symmetric Jacobi by one workgroup.  a (n x n, ld) is diagonalised in
// place, v receives the eigenvectors as columns.  Returns false if it did not
// converge within max_sweeps.
__device__ bool jacobi_sym_wg(double* a, double* v, int n, long ld, int max_sweeps, double* rc, double* rs, int* rp,
                              int* rq, int* flag) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (long e = tid; e < (long)n * n; e += nt) {
    long i = e / n, j = e % n;
    v[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  wg_sync();
  if (n == 1) return true;
  const int npad = n + (n & 1), half = npad / 2;
  const long nblk = (long)half * (half + 1) / 2;
  bool converged = false;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    if (tid == 0) *flag = 0;
    wg_sync();
    for (int s = 0; s < npad - 1; ++s) {
      for (int i = tid; i < half; i += nt) {
        int p, q;
        rr_pair_s(npad, s, i, p, q);
        double c = 1.0, sn = 0.0;
        if (p < n && q < n) {
          double app = a[(long)p * ld + p], aqq = a[(long)q * ld + q], apq = a[(long)p * ld + q];
          if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-300) {
            double th = (aqq - app) / (2.0 * apq);
            double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
            *flag = 1;
          }
        }
        rp[i] = p;
        rq[i] = q;
        rc[i] = c;
        rs[i] = sn;
      }
      wg_sync();
      for (long e = tid; e < nblk + (long)n * half; e += nt) {
        if (e < nblk) {
          int P = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) / 2.0);
          while ((long)(P + 1) * (P + 2) / 2 <= e) ++P;
          while ((long)P * (P + 1) / 2 > e) --P;
          int Q = (int)(e - (long)P * (P + 1) / 2);
          int p1 = rp[P], q1 = rq[P], p2 = rp[Q], q2 = rq[Q];
          if (P == Q) {
            if (p1 >= n || q1 >= n || rs[P] == 0.0) continue;
            double t = rs[P] / rc[P];
            double apq = a[(long)p1 * ld + q1];
            a[(long)p1 * ld + p1] -= t * apq;
            a[(long)q1 * ld + q1] += t * apq;
            a[(long)p1 * ld + q1] = 0.0;
            a[(long)q1 * ld + p1] = 0.0;
            continue;
          }
          bool r0v = p1 < n, r1v = q1 < n, c0v = p2 < n, c1v = q2 < n;
          double x00 = (r0v && c0v) ? a[(long)p1 * ld + p2] : 0.0;
          double x01 = (r0v && c1v) ? a[(long)p1 * ld + q2] : 0.0;
          double x10 = (r1v && c0v) ? a[(long)q1 * ld + p2] : 0.0;
          double x11 = (r1v && c1v) ? a[(long)q1 * ld + q2] : 0.0;
          double cq = rc[Q], sq = rs[Q];
          if (sq != 0.0) {  // X J_Q, J = [[c, s], [-s, c]]
            double y00 = cq * x00 - sq * x01, y01 = sq * x00 + cq * x01;
            double y10 = cq * x10 - sq * x11, y11 = sq * x10 + cq * x11;
            x00 = y00; x01 = y01; x10 = y10; x11 = y11;
          }
          double cp = rc[P], sp = rs[P];
          if (sp != 0.0) {  // J_P^T X
            double y00 = cp * x00 - sp * x10, y01 = cp * x01 - sp * x11;
            double y10 = sp * x00 + cp * x10, y11 = sp * x01 + cp * x11;
            x00 = y00; x01 = y01; x10 = y10; x11 = y11;
          }
          if (r0v && c0v) { a[(long)p1 * ld + p2] = x00; a[(long)p2 * ld + p1] = x00; }
          if (r0v && c1v) { a[(long)p1 * ld + q2] = x01; a[(long)q2 * ld + p1] = x01; }
          if (r1v && c0v) { a[(long)q1 * ld + p2] = x10; a[(long)p2 * ld + q1] = x10; }
          if (r1v && c1v) { a[(long)q1 * ld + q2] = x11; a[(long)q2 * ld + q1] = x11; }
        } else {
          long f = e - nblk;
          int k = (int)(f / half), P = (int)(f % half);
          int p1 = rp[P], q1 = rq[P];
          if (p1 >= n || q1 >= n || rs[P] == 0.0) continue;
          double c = rc[P], sn = rs[P];
          double vp = v[(long)k * ld + p1], vq = v[(long)k * ld + q1];
          v[(long)k * ld + p1] = c * vp - sn * vq;
          v[(long)k * ld + q1] = sn * vp + c * vq;
        }
      }
      wg_sync();
    }
    converged = (*flag == 0);
    wg_sync();
  }
  return converged;
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
// One GSVD step.  Dimensions read from device state so the host can enqueue
// every cut without synchronising.
__global__ __launch_bounds__(1024) void gsvd_cut_kernel(GsvdArgs a, int m) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int M = a.M;
  if (*a.err) return;
  const int n_prev = a.ne[m - 1];
  const int nL = n_prev + 1, N2 = 2 * nL, nR = M - m;
  if (N2 > GBS_GSVD_N2_MAX) {
    if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_KMAX);
    return;
  }
  const long ld = a.ld_ws;
  double* G = a.ws_G;     // Gamma_LL (kept)
  double* Lm = a.ws_L;    // Cholesky factor of 2 Gamma_LL
  double* Am = a.ws_A;    // L^T Omega L
  double* Bm = a.ws_B;    // A^T A -> diagonalised
  double* Ev = a.ws_E;    // eigenvectors of B
  double* Om = a.ws_O;    // symplectic pairs [u.., v..]
  double* Sm = a.ws_S;    // symplectic M of the Williamson form
  double* vec = a.ws_vec; // scratch vectors (3 * ld)
  const double* g = a.gamma;
  const int n2g = 2 * M;
  const double* Drr = a.drr_in;
  const double* CR = a.cr_in;
  const long ldd = a.ld_drr, ldc = a.ld_cr;
  __shared__ double rc[600], rs[600], red[40];
  __shared__ int rp[600], rq[600], flag, npairs, bad;
  __shared__ double dsel[600];

  // 1. Gamma_LL in the xxpp order of (r_1..r_nprev, a_m).
  const int gxa = m - 1, gpa = M + m - 1;  // rows of a_m in Gamma
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    int i = (int)(e / N2), j = (int)(e % N2);
    int ii = i % nL, jj = j % nL;
    bool ip = i >= nL, jp = j >= nL;
    double val;
    if (ii < n_prev && jj < n_prev) {
      val = Drr[(long)(ip ? n_prev + ii : ii) * ldd + (jp ? n_prev + jj : jj)];
    } else if (ii < n_prev) {  // r row, a_m column
      val = CR[(long)(ip ? n_prev + ii : ii) * ldc + (jp ? gpa : gxa)];
    } else if (jj < n_prev) {
      val = CR[(long)(jp ? n_prev + jj : jj) * ldc + (ip ? gpa : gxa)];
    } else {
      val = g[(long)(ip ? gpa : gxa) * n2g + (jp ? gpa : gxa)];
    }
    G[(long)i * ld + j] = val;
    Lm[(long)i * ld + j] = 2.0 * val;
  }
  wg_sync();
  // 2. Cholesky 2 Gamma_LL = L L^T (lower, in place in Lm).
  for (int j = 0; j < N2; ++j) {
    if (tid == 0) {
      double d = Lm[(long)j * ld + j];
      bad = !(d > 0.0);
      Lm[(long)j * ld + j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    wg_sync();
    if (bad) {
      if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_NOT_PD);
      return;
    }
    double piv = Lm[(long)j * ld + j];
    for (int i = j + 1 + tid; i < N2; i += nt) Lm[(long)i * ld + j] /= piv;
    wg_sync();
    const long rem = N2 - j - 1;
    for (long e = tid; e < rem * rem; e += nt) {
      long i = j + 1 + e / rem, k = j + 1 + e % rem;
      if (k <= i) Lm[i * ld + k] -= Lm[i * ld + j] * Lm[k * ld + j];
    }
    wg_sync();
  }
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    long i = e / N2, j = e % N2;
    if (j > i) Lm[i * ld + j] = 0.0;
  }
  wg_sync();
  // 3. A = L^T (Omega L); (Omega L)_k = L_{k+nL} for k < nL, -L_{k-nL} otherwise.
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    int i = (int)(e / N2), j = (int)(e % N2);
    double s = 0.0;
    for (int k = 0; k < N2; ++k) {
      double ol = k < nL ? Lm[(long)(k + nL) * ld + j] : -Lm[(long)(k - nL) * ld + j];
      s += Lm[(long)k * ld + i] * ol;
    }
    Am[(long)i * ld + j] = s;
  }
  wg_sync();
  // 4. B = A^T A.
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    int i = (int)(e / N2), j = (int)(e % N2);
    double s = 0.0;
    for (int k = 0; k < N2; ++k) s += Am[(long)k * ld + i] * Am[(long)k * ld + j];
    Bm[(long)i * ld + j] = s;
  }
  wg_sync();
  for (long e = tid; e < (long)N2 * N2; e += nt) {  // exact symmetry
    long i = e / N2, j = e % N2;
    if (j > i) Bm[j * ld + i] = Bm[i * ld + j];
  }
  wg_sync();
  // 5. Jacobi.
  bool conv = jacobi_sym_wg(Bm, Ev, N2, ld, 60, rc, rs, rp, rq, &flag);
  if (!conv) {
    if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_JACOBI);
    return;
  }
  // order of eigenvalues (descending): rank sort into rp[] (index by rank)
  for (int i = tid; i < N2; i += nt) {
    double wi = Bm[(long)i * ld + i];
    int rank = 0;
    for (int j = 0; j < N2; ++j) {
      double wj = Bm[(long)j * ld + j];
      rank += (wj > wi) || (wj == wi && j < i);
    }
    rq[rank] = i;
  }
  if (tid == 0) npairs = 0;
  wg_sync();
  // 6. Symplectic pairing by Gram-Schmidt over eigenvectors in order.
  double* e_v = vec;
  double* au = vec + ld;
  for (int jr = 0; jr < N2; ++jr) {
    if (npairs >= nL) break;
    int col = rq[jr];
    for (int k = tid; k < N2; k += nt) e_v[k] = Ev[(long)k * ld + col];
    wg_sync();
    for (int pass = 0; pass < 2; ++pass) {
      const int nc = npairs;
      // project out chosen columns u_c = Om[:, c], v_c = Om[:, nL + c]
      for (int c = 0; c < 2 * nc; ++c) {
        int cc = c < nc ? c : nL + (c - nc);
        double part = 0.0;
        for (int k = tid; k < N2; k += nt) part += Om[(long)k * ld + cc] * e_v[k];
        double dot = wg_sum(part, red);
        for (int k = tid; k < N2; k += nt) e_v[k] -= dot * Om[(long)k * ld + cc];
        wg_sync();
      }
    }
    double part = 0.0;
    for (int k = tid; k < N2; k += nt) part += e_v[k] * e_v[k];
    double nrm = sqrt(wg_sum(part, red));
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
    double dlt = sqrt(wg_sum(part, red));
    const int c = npairs;
    for (int k = tid; k < N2; k += nt) {
      Om[(long)k * ld + c] = e_v[k];
      Om[(long)k * ld + nL + c] = -au[k] / dlt;
    }
    if (tid == 0) {
      dsel[c] = dlt;
      npairs = c + 1;
    }
    wg_sync();
  }
  if (npairs < nL) {
    if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_WILLIAMSON);
    return;
  }
  // Order pairs by D descending (stable); rp[k] = source pair of slot k.
  for (int i = tid; i < nL; i += nt) {
    int rank = 0;
    for (int j = 0; j < nL; ++j) rank += (dsel[j] > dsel[i]) || (dsel[j] == dsel[i] && j < i);
    rp[rank] = i;
  }
  wg_sync();
  // 7. S = L O diag(D, D)^(-1/2) with permuted pairs.
  for (long e = tid; e < (long)N2 * N2; e += nt) {
    int i = (int)(e / N2), j = (int)(e % N2);
    int jj = j % nL;
    int src = rp[jj] + (j >= nL ? nL : 0);
    double s = 0.0;
    for (int k = 0; k <= i; ++k) s += Lm[(long)i * ld + k] * Om[(long)k * ld + src];
    Sm[(long)i * ld + j] = s / sqrt(dsel[rp[jj]]);
  }
  wg_sync();
  // D values (descending) and active count.
  if (tid == 0) {
    int ne = 0;
    for (int k = 0; k < nL; ++k) {
      double d = dsel[rp[k]];
      a.dsym[(long)m * a.ld_dsym + k] = d;
      if (d >= a.dstar) ++ne;
    }
    if (ne > nR) ne = nR;
    a.ne[m] = (m == M) ? 0 : ne;
    flag = (m == M) ? 0 : ne;
    for (int k = 0; k < nL; ++k) {
      double d = dsel[rp[k]];
      a.lam[(long)m * a.ld_dsym + k] = d > 1.0 ? sqrt((d - 1.0) / (d + 1.0)) : 0.0;
    }
  }
  wg_sync();
  const int ne = flag;
  // 8. U, V from S (Eq. MUV): U = ((S21 - S12) - i (S11 + S22)) / 2, V = ((-S12 - S21) - i (S11 - S22)) / 2.
  cplx64* U = a.ws_U;
  cplx64* V = a.ws_V;
  cplx64* Aug = a.ws_aug;  // nL x 2nL
  const long ldu = a.ld_u;
  for (long e = tid; e < (long)nL * nL; e += nt) {
    int i = (int)(e / nL), j = (int)(e % nL);
    double s11 = Sm[(long)i * ld + j], s12 = Sm[(long)i * ld + nL + j];
    double s21 = Sm[(long)(nL + i) * ld + j], s22 = Sm[(long)(nL + i) * ld + nL + j];
    U[i * ldu + j] = cmake<cplx64>(0.5 * (s21 - s12), -0.5 * (s11 + s22));
    V[i * ldu + j] = cmake<cplx64>(0.5 * (-s12 - s21), -0.5 * (s11 - s22));
  }
  wg_sync();
  // 9. (U^dag)^-1 by Gauss-Jordan with partial pivoting on [U^dag | I].
  for (long e = tid; e < (long)nL * 2 * nL; e += nt) {
    int i = (int)(e / (2 * nL)), j = (int)(e % (2 * nL));
    Aug[i * 2 * ldu + j] = j < nL ? cconj(U[(long)j * ldu + i]) : cmake<cplx64>(j - nL == i ? 1.0 : 0.0, 0.0);
  }
  wg_sync();
  for (int col = 0; col < nL; ++col) {
    if (tid == 0) {
      int best = col;
      double bv = cabs2(Aug[(long)col * 2 * ldu + col]);
      for (int r = col + 1; r < nL; ++r) {
        double v = cabs2(Aug[(long)r * 2 * ldu + col]);
        if (v > bv) { bv = v; best = r; }
      }
      rp[0] = best;
      bad = !(bv > 1e-280);
    }
    wg_sync();
    if (bad) {
      if (tid == 0) gbs_set_error(a.err, GBS_DEVERR_SINGULAR);
      return;
    }
    const int pr = rp[0];
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
  // Uih(i, j) = Aug[i][nL + j]
  // 10. Q^m on (r_{m-1}, a_m, l_m): [[Uih V^dag, Uih[:, :ne]], [.^T, -V^T Uih restricted]].
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
  // 11. Next residual: T = -S^T Omega; T[r][c] = c < nL ? S[c+nL][r] : -S[c-nL][r].
  // Active rows: x_b,q -> r = q, p_b,q -> r = nL + q (q < ne).
  // Drr' = T_act Gamma_LL T_act^T (2ne x 2ne); CR' = T_act Gamma_{L, R}.
  double* Dn = a.drr_out;
  double* CRn = a.cr_out;
  double* TG = a.ws_B;  // reuse: T_act Gamma_LL (2ne x N2)
  for (long e = tid; e < (long)2 * ne * N2; e += nt) {
    int r = (int)(e / N2), j = (int)(e % N2);
    int rr = r < ne ? r : nL + (r - ne);
    double s = 0.0;
    for (int c = 0; c < N2; ++c) {
      double t = c < nL ? Sm[(long)(c + nL) * ld + rr] : -Sm[(long)(c - nL) * ld + rr];
      s += t * G[(long)c * ld + j];
    }
    TG[(long)r * ld + j] = s;
  }
  wg_sync();
  for (long e = tid; e < (long)2 * ne * 2 * ne; e += nt) {
    int r = (int)(e / (2 * ne)), r2 = (int)(e % (2 * ne));
    int rr2 = r2 < ne ? r2 : nL + (r2 - ne);
    double s = 0.0;
    for (int c = 0; c < N2; ++c) {
      double t = c < nL ? Sm[(long)(c + nL) * ld + rr2] : -Sm[(long)(c - nL) * ld + rr2];
      s += TG[(long)r * ld + c] * t;
    }
    Dn[(long)r * ldd + r2] = s;
  }
  // CR' columns: x of a_{m+1..M} at Gamma column j (j >= m), p at M + j.
  for (long e = tid; e < (long)2 * ne * 2 * nR; e += nt) {
    int r = (int)(e / (2 * nR)), cc = (int)(e % (2 * nR));
    int gcol = cc < nR ? m + cc : M + m + (cc - nR);
    int rr = r < ne ? r : nL + (r - ne);
    double s = 0.0;
    for (int c = 0; c < N2; ++c) {
      double t = c < nL ? Sm[(long)(c + nL) * ld + rr] : -Sm[(long)(c - nL) * ld + rr];
      int ci = c % nL;
      bool cp = c >= nL;
      double gv = ci < n_prev ? CR[(long)(cp ? n_prev + ci : ci) * ldc + gcol]
                              : g[(long)(cp ? gpa : gxa) * n2g + gcol];
      s += t * gv;
    }
    CRn[(long)r * ldc + gcol] = s;
  }
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

hipError_t launch_gsvd_cut(hipStream_t st, const GsvdArgs& a, int m) {
  hipLaunchKernelGGL(gsvd_cut_kernel, dim3(1), dim3(1024), 0, st, a, m);
  return hipGetLastError();
}
