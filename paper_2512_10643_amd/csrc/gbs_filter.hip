// Mixed -> pure filtration of a Gaussian covariance (Sec. III, Eq. decompose;
// App. C, Eq. loss and the Riemannian descent on Sp(2N)), FP64.
//
// The descent is sequential: every step needs the lowest eigenpair of
// W = Gamma_th - S S^T / 2 at the current S.  One workgroup runs a batch of
// steps per launch with W, a working copy of it and S resident in L2:
//   1. Householder reduction of the copy to tridiagonal form T (reflectors
//      kept in the copy's lower part);
//   2. lambda_min of T by Sturm-count multisection (every thread one shift);
//   3. its eigenvector by inverse iteration on T, back-transformed by the
//      reflectors (one wave, no barriers);
//   4. w = S^T v0, u = Omega w, loss L = -lambda_min; stop when L <= eps;
//   5. step alpha = min(alpha_max, L / dL) with dL = |w|^2 / sqrt(2), the
//      derivative of L along the unit gradient G = (w w^T - u u^T) / (sqrt(2) |w|^2);
//   6. retraction S <- S exp(-alpha G) in closed form: G has eigenvalues
//      +-1/sqrt(2) on w/|w| and u/|w| (w and u are orthogonal and of equal
//      norm) and 0 elsewhere, so with a = alpha/sqrt(2), x = S w^, y = S u^:
//        S <- S + (e^{-a} - 1) x w^T + (e^{a} - 1) y u^T,
//        S S^T <- S S^T + (e^{-2a} - 1) x x^T + (e^{2a} - 1) y y^T,
//      a rank-2 update of W.
// The host repeats launches until the loss is below eps or the step budget
// is spent.  Then Gamma_p = S S^T / 2 by a separate product over many
// workgroups.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <string>

#include "gbs_common.h"
#include "gbs_internal.h"

namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr int kNMax = 2 * GBS_FILTER_MODES_MAX;  // largest 2N
constexpr int kStepsPerLaunch = 32;

struct FilterState {
  int iterations;  // retraction steps taken
  int done;        // 1 once L <= eps at the current S
  double loss;     // L at the current S
  double n_eff;    // filled by the final kernel
};

__device__ inline double wave_sum(double x) {
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Sum over the workgroup; every thread gets the result.
__device__ double wg_sum(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = x;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < kWaves; ++i) r += red[i];
  return r;
}

// Number of eigenvalues of the tridiagonal (d, e) below s (Sturm count of the
// LDL^T pivots; a zero pivot is moved off zero by a tiny amount).
__device__ int sturm_count(const double* d, const double* e, int n, double s, double tiny) {
  int c = 0;
  double q = d[0] - s;
  if (q == 0.0) q = -tiny;
  c += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - s - e[i - 1] * e[i - 1] / q;
    if (q == 0.0) q = -tiny;
    c += q < 0.0;
  }
  return c;
}

__global__ __launch_bounds__(kThreads) void filter_steps_kernel(double* __restrict__ Wm, double* __restrict__ A,
                                                                double* __restrict__ S, int n, double eps,
                                                                double alpha_max, int steps, int max_iter,
                                                                FilterState* __restrict__ st) {
  __shared__ double dd[kNMax], ee[kNMax], tau[kNMax];
  __shared__ double va[kNMax], vb[kNMax], vc[kNMax], vd[kNMax];
  __shared__ double red[kWaves];
  __shared__ double sh_lo, sh_hi, sh_lambda;
  __shared__ int sh_idx;
  __shared__ int sh_iter, sh_done;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int N = n / 2;
  if (tid == 0) {
    sh_iter = st->iterations;
    sh_done = st->done;
  }
  __syncthreads();
  for (int it = 0; it < steps; ++it) {
    if (sh_done || sh_iter >= max_iter) break;  // uniform: LDS, updated before a barrier
    // ---- 1. A (a copy of W) to tridiagonal form
    for (int k = 0; k + 2 < n; ++k) {
      const int m = n - k - 1;
      for (int j = tid; j < m; j += kThreads) va[j] = A[(long)(k + 1 + j) * n + k];
      __syncthreads();
      double part = 0.0;
      for (int j = 1 + tid; j < m; j += kThreads) part += va[j] * va[j];
      const double tail = wg_sum(part, red);
      const double x0 = va[0];
      double t = 0.0, beta = x0;
      if (tail > 0.0) {
        beta = -copysign(sqrt(x0 * x0 + tail), x0);
        t = (beta - x0) / beta;
        const double sc = 1.0 / (x0 - beta);
        __syncthreads();
        for (int j = 1 + tid; j < m; j += kThreads) va[j] *= sc;
      }
      __syncthreads();
      if (tid == 0) {
        va[0] = 1.0;
        dd[k] = A[(long)k * n + k];
        ee[k] = beta;
        tau[k] = t;
      }
      __syncthreads();
      for (int j = tid; j < m; j += kThreads) A[(long)(k + 1 + j) * n + k] = va[j];  // reflector, for step 3
      __syncthreads();
      if (t == 0.0) continue;  // uniform
      // p = t * A_sub v, one wave per row
      for (int i = wv; i < m; i += kWaves) {
        const double* row = A + (long)(k + 1 + i) * n + (k + 1);
        double s = 0.0;
        for (int j = lane; j < m; j += 64) s += row[j] * va[j];
        s = wave_sum(s);
        if (lane == 0) vb[i] = t * s;
      }
      __syncthreads();
      double pv = 0.0;
      for (int j = tid; j < m; j += kThreads) pv += vb[j] * va[j];
      const double K = 0.5 * t * wg_sum(pv, red);
      for (int j = tid; j < m; j += kThreads) vb[j] -= K * va[j];
      __syncthreads();
      // A_sub -= v w^T + w v^T
      for (int i = wv; i < m; i += kWaves) {
        double* row = A + (long)(k + 1 + i) * n + (k + 1);
        const double vi = va[i], wi = vb[i];
        for (int j = lane; j < m; j += 64) row[j] -= vi * vb[j] + wi * va[j];
      }
      __syncthreads();
    }
    if (tid == 0) {
      if (n >= 2) {
        dd[n - 2] = A[(long)(n - 2) * n + (n - 2)];
        ee[n - 2] = A[(long)(n - 1) * n + (n - 2)];
      }
      dd[n - 1] = A[(long)(n - 1) * n + (n - 1)];
      double lo = 0.0, hi = 0.0;
      for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
        lo = i == 0 ? dd[i] - r : fmin(lo, dd[i] - r);
        hi = i == 0 ? dd[i] + r : fmax(hi, dd[i] + r);
      }
      const double w = fmax(fabs(lo), fabs(hi));
      sh_lo = lo - 1e-12 * w - 1e-300;
      sh_hi = hi + 1e-12 * w + 1e-300;
    }
    __syncthreads();
    // ---- 2. lambda_min by multisection: count(lo) = 0, count(hi) >= 1
    const double scale = fmax(fabs(sh_lo), fabs(sh_hi));
    const double tiny = 1e-300 + 1e-30 * scale;
    for (int round = 0; round < 12; ++round) {
      const double lo = sh_lo, hi = sh_hi;
      if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + 1e-300) break;
      if (tid == 0) sh_idx = kThreads;
      __syncthreads();
      const double s = lo + (hi - lo) * (double)(tid + 1) / (double)(kThreads + 1);
      if (s > lo && s < hi && sturm_count(dd, ee, n, s, tiny) >= 1) atomicMin(&sh_idx, tid);
      __syncthreads();
      if (tid == 0) {
        const int f = sh_idx;
        if (f < kThreads) sh_hi = lo + (hi - lo) * (double)(f + 1) / (double)(kThreads + 1);
        if (f > 0) sh_lo = lo + (hi - lo) * (double)f / (double)(kThreads + 1);
      }
      __syncthreads();
    }
    // ---- 3. eigenvector: inverse iteration on T - lambda, then Q x
    if (tid == 0) {
      const double lam = 0.5 * (sh_lo + sh_hi);
      sh_lambda = lam;
      // LU with partial pivoting of T - lam (rows: diag a, super b, second super c)
      const double pert = 2.220446049250313e-16 * scale + 1e-300;
      double* a = vb;  // diagonal of U
      double* b = vc;  // first superdiagonal of U
      double* c = vd;  // second superdiagonal of U (fill from row interchanges)
      // start vector: fixed, with no special structure
      for (int i = 0; i < n; ++i) va[i] = 1.0 + 0.1 * (double)((i * 2654435761u) % 97u) / 97.0;
      for (int iter = 0; iter < 3; ++iter) {
        // forward elimination with partial pivoting, applied to the right-hand side on the fly
        double di = dd[0] - lam, ui = n > 1 ? ee[0] : 0.0, wi = 0.0;  // current row (diag, super1, super2)
        for (int i = 0; i + 1 < n; ++i) {
          // row i: (di, ui, wi) at columns (i, i+1, i+2); row i+1: (ee[i], dd[i+1]-lam, ee[i+1])
          const double sub = ee[i];
          const double d1 = dd[i + 1] - lam, u1 = i + 2 < n ? ee[i + 1] : 0.0;
          if (fabs(sub) > fabs(di)) {
            // swap rows i and i+1
            const double f = di / sub;
            a[i] = sub;
            b[i] = d1;
            c[i] = u1;
            const double r = va[i];
            va[i] = va[i + 1];
            va[i + 1] = r - f * va[i];
            di = ui - f * d1;
            ui = wi - f * u1;
            wi = 0.0;
          } else {
            double p = di;
            if (p == 0.0) p = pert;
            const double f = sub / p;
            a[i] = p;
            b[i] = ui;
            c[i] = wi;
            va[i + 1] -= f * va[i];
            di = d1 - f * ui;
            ui = u1 - f * wi;
            wi = 0.0;
          }
        }
        a[n - 1] = di == 0.0 ? pert : di;
        // back substitution
        for (int i = n - 1; i >= 0; --i) {
          double r = va[i];
          if (i + 1 < n) r -= b[i] * va[i + 1];
          if (i + 2 < n) r -= c[i] * va[i + 2];
          va[i] = r / a[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) nrm += va[i] * va[i];
        nrm = 1.0 / sqrt(nrm);
        for (int i = 0; i < n; ++i) va[i] *= nrm;
      }
    }
    __syncthreads();
    if (wv == 0) {  // y <- H_0 ... H_{n-3} y, reflectors from last to first
      for (int k = n - 3; k >= 0; --k) {
        const double t = tau[k];
        if (t == 0.0) continue;
        const int m = n - k - 1;
        double s = 0.0;
        for (int j = lane; j < m; j += 64) s += A[(long)(k + 1 + j) * n + k] * va[k + 1 + j];
        s = t * wave_sum(s);
        for (int j = lane; j < m; j += 64) va[k + 1 + j] -= s * A[(long)(k + 1 + j) * n + k];
      }
    }
    __syncthreads();
    // ---- 4. w = S^T v0 (thread j: column j), u = Omega w, |w|^2, loss
    for (int j = tid; j < n; j += kThreads) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += S[(long)i * n + j] * va[i];
      vb[j] = s;
    }
    __syncthreads();
    double part = 0.0;
    for (int j = tid; j < n; j += kThreads) part += vb[j] * vb[j];
    const double w2 = wg_sum(part, red);
    const double L = -sh_lambda;
    if (tid == 0) st->loss = L;
    if (L <= eps) {
      if (tid == 0) sh_done = 1;
      break;
    }
    // ---- 5, 6. step and retraction
    const double inv = 1.0 / sqrt(w2);
    for (int j = tid; j < n; j += kThreads) {
      const double wj = vb[j] * inv;
      const double uj = (j < N ? vb[j + N] : -vb[j - N]) * inv;
      vc[j] = wj;  // w^
      vd[j] = uj;  // u^
    }
    const double dl = w2 / sqrt(2.0);
    const double alpha = fmin(alpha_max, L / dl);
    const double ah = alpha / sqrt(2.0);
    __syncthreads();
    for (int i = wv; i < n; i += kWaves) {  // x = S w^, y = S u^
      const double* row = S + (long)i * n;
      double sx = 0.0, sy = 0.0;
      for (int j = lane; j < n; j += 64) {
        sx += row[j] * vc[j];
        sy += row[j] * vd[j];
      }
      sx = wave_sum(sx);
      sy = wave_sum(sy);
      if (lane == 0) {
        va[i] = sx;
        vb[i] = sy;
      }
    }
    __syncthreads();
    const double em = expm1(-ah), ep = expm1(ah), em2 = expm1(-2.0 * ah), ep2 = expm1(2.0 * ah);
    for (int i = wv; i < n; i += kWaves) {
      double* srow = S + (long)i * n;
      double* wrow = Wm + (long)i * n;
      double* arow = A + (long)i * n;
      const double xi = va[i], yi = vb[i];
      for (int j = lane; j < n; j += 64) {
        srow[j] += em * xi * vc[j] + ep * yi * vd[j];
        const double wn = wrow[j] - 0.5 * (em2 * xi * va[j] + ep2 * yi * vb[j]);
        wrow[j] = wn;
        arow[j] = wn;
      }
    }
    if (tid == 0) sh_iter += 1;
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) {
    st->iterations = sh_iter;
    st->done = sh_done;
  }
}

__global__ void filter_init_kernel(const double* __restrict__ G, double* __restrict__ Wm, double* __restrict__ A,
                                   double* __restrict__ S, int n, FilterState* st) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e == 0) {
    st->iterations = 0;
    st->done = 0;
    st->loss = 0.0;
    st->n_eff = 0.0;
  }
  if (e >= (long)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  const double g = 0.5 * (G[(long)i * n + j] + G[(long)j * n + i]);  // symmetric part
  const double w = g - (i == j ? 0.5 : 0.0);
  Wm[e] = w;
  A[e] = w;
  S[e] = i == j ? 1.0 : 0.0;
}

// Gamma_p = S S^T / 2 (16 x 16 tiles) and the largest |G - G^T|.
__global__ void filter_gram_kernel(const double* __restrict__ S, int n, double* __restrict__ Gp) {
  __shared__ double ta[16][17], tb[16][17];
  const int ti = threadIdx.y, tj = threadIdx.x;
  const int i = blockIdx.y * 16 + ti, j = blockIdx.x * 16 + tj;
  double acc = 0.0;
  for (int k0 = 0; k0 < n; k0 += 16) {
    ta[ti][tj] = (i < n && k0 + tj < n) ? S[(long)i * n + k0 + tj] : 0.0;
    tb[ti][tj] = (blockIdx.x * 16 + ti < n && k0 + tj < n) ? S[(long)(blockIdx.x * 16 + ti) * n + k0 + tj] : 0.0;
    __syncthreads();
    for (int k = 0; k < 16; ++k) acc += ta[ti][k] * tb[tj][k];
    __syncthreads();
  }
  if (i < n && j < n) Gp[(long)i * n + j] = 0.5 * acc;
}

__global__ void filter_neff_kernel(const double* __restrict__ Gp, int n, FilterState* st) {
  __shared__ double red[kWaves];
  double part = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) part += Gp[(long)i * n + i];
  const double tr = wg_sum(part, red);
  if (threadIdx.x == 0) st->n_eff = 0.5 * tr - 0.25 * (double)n;
}

__global__ void asym_kernel(const double* __restrict__ G, int n, double* __restrict__ out) {
  __shared__ double red[kWaves];
  double mx = 0.0, ma = 0.0;
  for (long e = threadIdx.x; e < (long)n * n; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const double g = G[e];
    mx = fmax(mx, fabs(g - G[(long)j * n + i]));
    ma = fmax(ma, fabs(g));
    if (!(g == g)) ma = INFINITY;  // NaN
  }
  for (int o = 32; o >= 1; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    ma = fmax(ma, __shfl_xor(ma, o, 64));
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < (int)(blockDim.x / 64); ++i) r = fmax(r, red[i]);
    out[0] = r;
  }
  __syncthreads();
  if (lane == 0) red[wv] = ma;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < (int)(blockDim.x / 64); ++i) r = fmax(r, red[i]);
    out[1] = r;
  }
}

double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Stream-ordered device buffers released in order on the same stream.
struct Buf {
  hipStream_t st;
  void* p = nullptr;
  explicit Buf(hipStream_t s) : st(s) {}
  ~Buf() {
    if (p) (void)hipFreeAsync(p, st);
  }
};

int hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return gbs_fail(e == hipErrorOutOfMemory ? GBS_E_NOMEM : GBS_E_DEVICE,
                  std::string("HIP error '") + hipGetErrorString(e) + "' in " + what);
}

#define FCHECK(x)                                \
  do {                                           \
    hipError_t _e = (x);                         \
    if (_e != hipSuccess) return hip_fail(_e, #x); \
  } while (0)

}  // namespace

extern "C" int gbs_filter_pure(const double* gamma_th, int32_t N, const gbs_filter_opts* opt, double* gamma_p,
                               double* S_out, gbs_filter_info_t* info, void* stream) {
  if (!gamma_th || !gamma_p || !opt || !info) return gbs_fail(GBS_E_INVAL, "NULL argument");
  if (N < 1 || N > GBS_FILTER_MODES_MAX) return gbs_fail(GBS_E_INVAL, "N must be in [1, 288]");
  if (!(opt->eps >= 0.0) || !(opt->alpha_max >= 0.0) || opt->max_iter < 0)
    return gbs_fail(GBS_E_INVAL, "eps, alpha_max and max_iter must be >= 0");
  const double eps = opt->eps > 0.0 ? opt->eps : 1e-12;
  const double alpha_max = opt->alpha_max > 0.0 ? opt->alpha_max : 0.5;
  const int max_iter = opt->max_iter > 0 ? opt->max_iter : 100000;
  *info = gbs_filter_info_t{};
  const double t0 = wall_ms();
  hipStream_t st = (hipStream_t)stream;
  const int n = 2 * N;
  const size_t mat = (size_t)n * n * sizeof(double);
  Buf wm(st), a(st), s(st), stb(st), chk(st);
  FCHECK(hipMallocAsync(&wm.p, mat, st));
  FCHECK(hipMallocAsync(&a.p, mat, st));
  FCHECK(hipMallocAsync(&s.p, mat, st));
  FCHECK(hipMallocAsync(&stb.p, sizeof(FilterState), st));
  FCHECK(hipMallocAsync(&chk.p, 2 * sizeof(double), st));
  // symmetric, finite input
  hipLaunchKernelGGL(asym_kernel, dim3(1), dim3(kThreads), 0, st, gamma_th, n, (double*)chk.p);
  FCHECK(hipGetLastError());
  double hc[2];
  FCHECK(hipMemcpyAsync(hc, chk.p, sizeof hc, hipMemcpyDeviceToHost, st));
  FCHECK(hipStreamSynchronize(st));
  if (!(hc[1] < INFINITY)) return gbs_fail(GBS_E_INVAL, "Gamma_th holds a non-finite entry");
  if (!(hc[0] <= 1e-10 * std::max(1.0, hc[1]))) return gbs_fail(GBS_E_NOT_PD, "Gamma_th is not symmetric");
  const long tot = (long)n * n;
  hipLaunchKernelGGL(filter_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, gamma_th,
                     (double*)wm.p, (double*)a.p, (double*)s.p, n, (FilterState*)stb.p);
  FCHECK(hipGetLastError());
  FilterState hs{};
  while (true) {
    hipLaunchKernelGGL(filter_steps_kernel, dim3(1), dim3(kThreads), 0, st, (double*)wm.p, (double*)a.p,
                       (double*)s.p, n, eps, alpha_max, kStepsPerLaunch, max_iter, (FilterState*)stb.p);
    FCHECK(hipGetLastError());
    FCHECK(hipMemcpyAsync(&hs, stb.p, sizeof hs, hipMemcpyDeviceToHost, st));
    FCHECK(hipStreamSynchronize(st));
    if (hs.done || hs.iterations >= max_iter) break;
    if (!(hs.loss == hs.loss)) return gbs_fail(GBS_E_INTERNAL, "the filtration loss became NaN");
  }
  hipLaunchKernelGGL(filter_gram_kernel, dim3((unsigned)((n + 15) / 16), (unsigned)((n + 15) / 16)), dim3(16, 16), 0,
                     st, (const double*)s.p, n, gamma_p);
  FCHECK(hipGetLastError());
  hipLaunchKernelGGL(filter_neff_kernel, dim3(1), dim3(kThreads), 0, st, (const double*)gamma_p, n,
                     (FilterState*)stb.p);
  FCHECK(hipGetLastError());
  if (S_out) FCHECK(hipMemcpyAsync(S_out, s.p, mat, hipMemcpyDeviceToDevice, st));
  FCHECK(hipMemcpyAsync(&hs, stb.p, sizeof hs, hipMemcpyDeviceToHost, st));
  FCHECK(hipStreamSynchronize(st));
  info->iterations = hs.iterations;
  info->converged = hs.done;
  info->loss = hs.loss;
  info->n_eff = hs.n_eff;
  info->ms = wall_ms() - t0;
  return GBS_OK;
}
