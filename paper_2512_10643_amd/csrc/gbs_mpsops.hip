// MPS-level kernels: precision conversion, gauge scaling, normalisation and
// phase, amplitudes and sequential conditional sampling.
#include "gbs_mpsops.h"

template <typename CD, typename CS>
__global__ void convert_kernel(CD* dst, const CS* src, long n) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) {
    CS v = src[i];
    dst[i] = cmake<CD>((typename real_of<CD>::type)v.re, (typename real_of<CD>::type)v.im);
  }
}

template <typename CD, typename CS>
hipError_t convert(hipStream_t st, CD* dst, const CS* src, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_kernel<CD, CS>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}
template hipError_t convert<cplx32, cplx64>(hipStream_t, cplx32*, const cplx64*, long);
template hipError_t convert<cplx64, cplx32>(hipStream_t, cplx64*, const cplx32*, long);
template hipError_t convert<cplx64, cplx64>(hipStream_t, cplx64*, const cplx64*, long);
template hipError_t convert<cplx32, cplx32>(hipStream_t, cplx32*, const cplx32*, long);

// dst (rows x cols, ld_dst) = src (FP64, ld_src) with column j scaled by
// colscale[j] (or 1/colscale[j] when invert), converted to the target type.
template <typename CD>
__global__ void scaled_copy_kernel(CD* dst, long ld_dst, const cplx64* src, long ld_src, int rows, int cols,
                                   const double* colscale, int invert, int conj_transpose) {
  long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  int i = (int)(e / cols), j = (int)(e % cols);
  cplx64 v;
  double s = 1.0;
  if (conj_transpose) {  // dst(i, j) = conj(src(j, i)) * scale(i)
    v = cconj(src[(long)j * ld_src + i]);
    if (colscale) s = invert ? 1.0 / colscale[i] : colscale[i];
  } else {
    v = src[(long)i * ld_src + j];
    if (colscale) s = invert ? 1.0 / colscale[j] : colscale[j];
  }
  dst[(long)i * ld_dst + j] = cmake<CD>((typename real_of<CD>::type)(v.re * s), (typename real_of<CD>::type)(v.im * s));
}

template <typename CD>
hipError_t scaled_copy(hipStream_t st, CD* dst, long ld_dst, const cplx64* src, long ld_src, int rows, int cols,
                       const double* colscale, int invert, int conj_transpose) {
  long n = (long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((scaled_copy_kernel<CD>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, ld_dst, src,
                     ld_src, rows, cols, colscale, invert, conj_transpose);
  return hipGetLastError();
}
template hipError_t scaled_copy<cplx32>(hipStream_t, cplx32*, long, const cplx64*, long, int, int, const double*, int,
                                        int);
template hipError_t scaled_copy<cplx64>(hipStream_t, cplx64*, long, const cplx64*, long, int, int, const double*, int,
                                        int);

// x (rows x cols) : x[i][j] *= rowscale[i]^(-1) * colscale[j]  (NULL = 1).
// Scales are square roots of the given weights when `sqrt_weights`.
template <typename C>
__global__ void gauge_scale_kernel(C* x, int rows, int d, int cols, const double* wrow, const double* wcol) {
  long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long n = (long)rows * d * cols;
  if (e >= n) return;
  int i = (int)(e / ((long)d * cols));
  int j = (int)(e % cols);
  double s = 1.0;
  if (wrow) s /= sqrt(wrow[i]);
  if (wcol) s *= sqrt(wcol[j]);
  x[e] = cscale(x[e], (typename real_of<C>::type)s);
}

template <typename C>
hipError_t gauge_scale(hipStream_t st, C* x, int rows, int d, int cols, const double* wrow, const double* wcol) {
  long n = (long)rows * d * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((gauge_scale_kernel<C>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, rows, d, cols,
                     wrow, wcol);
  return hipGetLastError();
}
template hipError_t gauge_scale<cplx32>(hipStream_t, cplx32*, int, int, int, const double*, const double*);
template hipError_t gauge_scale<cplx64>(hipStream_t, cplx64*, int, int, int, const double*, const double*);

// Normalise to unit norm and make the vacuum amplitude real > 0: site 1 is
// multiplied by conj(z) / |z| / norm, with z = <0..0|psi> (vac, computed by
// the caller) and norm^2 = *nrm2_in, or the squared norm of site 1 when
// nrm2_in is NULL (exact when sites 2..M are right-canonical).  One workgroup.
template <typename C>
__global__ __launch_bounds__(1024) void normalize_kernel(C* b1, int n1, const cplx64* vac, const double* nrm2_in,
                                                          double* out_norm) {
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double red[64];
  __shared__ double s_re, s_im;
  double part = 0.0;
  for (int e = tid; e < n1; e += nt) {
    C v = b1[e];
    part += (double)v.re * v.re + (double)v.im * v.im;
  }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = part;
  __syncthreads();
  if (tid == 0) {
    double sacc = 0.0;
    for (int i = 0; i < (nt + 63) / 64; ++i) sacc += red[i];
    const double nrm2 = nrm2_in ? *nrm2_in : sacc;
    const double zr = vac->re, zi = vac->im;
    const double az = sqrt(zr * zr + zi * zi);
    const double inv = 1.0 / sqrt(nrm2);
    if (az > 0.0) {
      s_re = zr / az * inv;
      s_im = -zi / az * inv;
    } else {
      s_re = inv;
      s_im = 0.0;
    }
    *out_norm = sqrt(nrm2);
  }
  __syncthreads();
  for (int e = tid; e < n1; e += nt) {
    C x = b1[e];
    double xr = x.re, xi = x.im;
    b1[e] = cmake<C>((typename real_of<C>::type)(xr * s_re - xi * s_im), (typename real_of<C>::type)(xr * s_im + xi * s_re));
  }
}

template <typename C>
hipError_t normalize_mps(hipStream_t st, C* site1, int n1, const cplx64* vac, const double* nrm2_in,
                         double* out_norm) {
  hipLaunchKernelGGL((normalize_kernel<C>), dim3(1), dim3(1024), 0, st, site1, n1, vac, nrm2_in, out_norm);
  return hipGetLastError();
}
template hipError_t normalize_mps<cplx32>(hipStream_t, cplx32*, int, const cplx64*, const double*, double*);
template hipError_t normalize_mps<cplx64>(hipStream_t, cplx64*, int, const cplx64*, const double*, double*);

// ---------------------------------------------------------------------------
// Amplitudes: one workgroup per pattern, FP64 accumulation.
template <typename C>
__global__ __launch_bounds__(256) void amplitude_kernel(C* const* sites, const int* bond, int M, int d,
                                                        const int32_t* pat, int64_t B, double* out, int* bad,
                                                        int maxbond) {
  const int64_t b = blockIdx.x;
  if (b >= B) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  extern __shared__ cplx64 amp_lds[];
  cplx64* v = amp_lds;
  cplx64* w = amp_lds + maxbond;
  __shared__ int invalid;
  if (tid == 0) {
    invalid = 0;
    for (int m = 0; m < M; ++m) {
      int p = pat[b * M + m];
      if (p < 0 || p >= d) invalid = 1;
    }
  }
  __syncthreads();
  if (invalid) {
    if (tid == 0) {
      out[2 * b] = __builtin_nan("");
      out[2 * b + 1] = __builtin_nan("");
      atomicOr(bad, 1);
    }
    return;
  }
  if (tid == 0) v[0] = cmake<cplx64>(1.0, 0.0);
  __syncthreads();
  for (int m = 1; m <= M; ++m) {
    const int rl = bond[m - 1], rr = bond[m];
    const int p = pat[b * M + (m - 1)];
    const C* bm = sites[m - 1];
    for (int j = tid; j < rr; j += nt) {
      double ar = 0.0, ai = 0.0;
      for (int i = 0; i < rl; ++i) {
        C t = bm[((long)i * d + p) * rr + j];
        ar += v[i].re * t.re - v[i].im * t.im;
        ai += v[i].re * t.im + v[i].im * t.re;
      }
      w[j] = cmake<cplx64>(ar, ai);
    }
    __syncthreads();
    for (int j = tid; j < rr; j += nt) v[j] = w[j];
    __syncthreads();
  }
  if (tid == 0) {
    out[2 * b] = v[0].re;
    out[2 * b + 1] = v[0].im;
  }
}

template <typename C>
hipError_t launch_amplitude(hipStream_t st, C* const* sites, const int* bond, int M, int d, const int32_t* pat,
                            int64_t B, double* out, int* bad, int maxbond) {
  if (B <= 0) return hipSuccess;
  size_t lds = 2 * (size_t)maxbond * sizeof(cplx64);
  hipLaunchKernelGGL((amplitude_kernel<C>), dim3((unsigned)B), dim3(256), lds, st, sites, bond, M, d, pat, B, out, bad,
                     maxbond);
  return hipGetLastError();
}
template hipError_t launch_amplitude<cplx32>(hipStream_t, cplx32* const*, const int*, int, int, const int32_t*, int64_t,
                                             double*, int*, int);
template hipError_t launch_amplitude<cplx64>(hipStream_t, cplx64* const*, const int*, int, int, const int32_t*, int64_t,
                                             double*, int*, int);

// ---------------------------------------------------------------------------
// Sampling, one site per launch.  A workgroup owns SHOTS shots; their left
// vectors L (bond[m-1] each) come from `lin`, the next ones go to `lout`.
// For p = 0, 1, ..., T_p = L B[:, p, :] is formed in registers (each thread
// owns a set of columns j for every shot) and its squared norm reduced across
// the workgroup.  L has unit norm and B is right-canonical, so these
// conditional probabilities sum to 1: each shot takes the first p whose
// running sum passes its uniform u (Philox keyed by the seed, counter
// (shot, site)), and the workgroup stops once all its shots are decided.  A
// shot whose u lies above the rounded total keeps the last p of positive
// weight (p = 0 if none).
template <typename C, int SHOTS, int JPT>
__global__ __launch_bounds__(256) void sample_site_kernel(const C* __restrict__ Bm, int rl, int d, int rr,
                                                          const C* __restrict__ lin, C* __restrict__ lout, long ldl,
                                                          int64_t shot0, int64_t nshots, int site, uint32_t k0,
                                                          uint32_t k1, int32_t* __restrict__ out, int M) {
  typedef typename real_of<C>::type R;
  const int tid = threadIdx.x;
  const int64_t sbase = (int64_t)blockIdx.x * SHOTS;
  __shared__ C Ls[SHOTS][64];
  __shared__ R red[SHOTS][4];
  __shared__ R wsum[SHOTS], wsel[SHOTS];
  __shared__ float ush[SHOTS];
  __shared__ int psel[SHOTS], take[SHOTS], left;
  C acc[SHOTS][JPT], sel[SHOTS][JPT];
  for (int s = tid; s < SHOTS; s += 256) {
    wsum[s] = (R)0;
    psel[s] = 0;
    const int64_t gs = sbase + s;
    philox4 c;
    c.v[0] = (uint32_t)(shot0 + gs);
    c.v[1] = (uint32_t)((uint64_t)(shot0 + gs) >> 32);
    c.v[2] = (uint32_t)site;
    c.v[3] = 0u;
    // a shot past the end is decided from the start
    ush[s] = gs < nshots ? u01_24(philox4x32_10(c, k0, k1).v[0]) : -1.f;
  }
  for (int p = 0; p < d; ++p) {
#pragma unroll
    for (int s = 0; s < SHOTS; ++s)
#pragma unroll
      for (int u = 0; u < JPT; ++u) acc[s][u] = cmake<C>((R)0, (R)0);
    for (int i0 = 0; i0 < rl; i0 += 64) {
      __syncthreads();
      for (int e = tid; e < SHOTS * 64; e += 256) {
        int s = e / 64, ii = e % 64;
        int64_t gs = sbase + s;
        Ls[s][ii] = (gs < nshots && i0 + ii < rl) ? lin[gs * ldl + i0 + ii] : cmake<C>((R)0, (R)0);
      }
      __syncthreads();
      const int iend = min(64, rl - i0);
      for (int ii = 0; ii < iend; ++ii) {
        C bv[JPT];
#pragma unroll
        for (int u = 0; u < JPT; ++u) {
          int j = tid + u * 256;
          bv[u] = j < rr ? Bm[((long)(i0 + ii) * d + p) * rr + j] : cmake<C>((R)0, (R)0);
        }
#pragma unroll
        for (int s = 0; s < SHOTS; ++s) {
          C lv = Ls[s][ii];
#pragma unroll
          for (int u = 0; u < JPT; ++u) cfma(acc[s][u], lv, bv[u]);
        }
      }
    }
    // squared norms per shot
#pragma unroll
    for (int s = 0; s < SHOTS; ++s) {
      R part = (R)0;
#pragma unroll
      for (int u = 0; u < JPT; ++u) part += cabs2(acc[s][u]);
      for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
      if ((tid & 63) == 0) red[s][tid >> 6] = part;
    }
    __syncthreads();
    if (tid == 0) left = 0;
    for (int s = tid; s < SHOTS; s += 256) {
      const R wp = red[s][0] + red[s][1] + red[s][2] + red[s][3];
      int tk = 0;
      if (ush[s] >= 0.f) {
        wsum[s] += wp;
        const bool dec = (R)ush[s] < wsum[s];
        // taken, or the provisional choice: the last p of positive weight
        tk = dec || wp > (R)0 || p == 0;
        if (dec) ush[s] = -1.f;
        else left = 1;
      }
      take[s] = tk;
      if (tk) {
        psel[s] = p;
        wsel[s] = wp;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < SHOTS; ++s) {
      if (take[s]) {
#pragma unroll
        for (int u = 0; u < JPT; ++u) sel[s][u] = acc[s][u];
      }
    }
    if (!left) break;  // every shot of the workgroup is decided
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SHOTS; ++s) {
    int64_t gs = sbase + s;
    if (gs >= nshots) continue;
    R inv = wsel[s] > (R)0 ? (R)1 / sqrt(wsel[s]) : (R)0;
#pragma unroll
    for (int u = 0; u < JPT; ++u) {
      int j = tid + u * 256;
      if (j < rr) lout[gs * ldl + j] = cscale(sel[s][u], inv);
    }
    if (tid == 0) out[(shot0 + gs) * (int64_t)M + (site - 1)] = psel[s];
  }
}

template <typename C>
__global__ void fill_first_kernel(C* l, long ldl, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) l[i * ldl] = cmake<C>((typename real_of<C>::type)1, (typename real_of<C>::type)0);
}
template <typename C>
hipError_t launch_fill_first(hipStream_t st, C* l, long ldl, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((fill_first_kernel<C>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, l, ldl, n);
  return hipGetLastError();
}
template hipError_t launch_fill_first<cplx32>(hipStream_t, cplx32*, long, int64_t);
template hipError_t launch_fill_first<cplx64>(hipStream_t, cplx64*, long, int64_t);

template <typename C>
hipError_t launch_sample_site(hipStream_t st, const C* Bm, int rl, int d, int rr, const C* lin, C* lout, long ldl,
                              int64_t shot0, int64_t nshots, int site, uint64_t seed, int32_t* out, int M) {
  constexpr int SHOTS = 8;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  unsigned grid = (unsigned)((nshots + SHOTS - 1) / SHOTS);
  if (rr <= 256)
    hipLaunchKernelGGL((sample_site_kernel<C, SHOTS, 1>), dim3(grid), dim3(256), 0, st, Bm, rl, d, rr, lin, lout, ldl,
                       shot0, nshots, site, k0, k1, out, M);
  else if (rr <= 512)
    hipLaunchKernelGGL((sample_site_kernel<C, SHOTS, 2>), dim3(grid), dim3(256), 0, st, Bm, rl, d, rr, lin, lout, ldl,
                       shot0, nshots, site, k0, k1, out, M);
  else if (rr <= 1024)
    hipLaunchKernelGGL((sample_site_kernel<C, SHOTS, 4>), dim3(grid), dim3(256), 0, st, Bm, rl, d, rr, lin, lout, ldl,
                       shot0, nshots, site, k0, k1, out, M);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
template hipError_t launch_sample_site<cplx32>(hipStream_t, const cplx32*, int, int, int, const cplx32*, cplx32*, long,
                                               int64_t, int64_t, int, uint64_t, int32_t*, int);
template hipError_t launch_sample_site<cplx64>(hipStream_t, const cplx64*, int, int, int, const cplx64*, cplx64*, long,
                                               int64_t, int64_t, int, uint64_t, int32_t*, int);
