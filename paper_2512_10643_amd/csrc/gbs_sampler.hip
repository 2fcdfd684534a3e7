// Sampling sweep on MFMA (FP32), one site per launch.
//
// For every shot s the conditional step at site m computes T_p = L_s B[:, p, :]
// for p < d, draws p with probability |T_p|^2 / sum_p' |T_p'|^2 and continues
// with L_s <- T_p (sequential conditional sampling on a right-canonical MPS).
// The complex products are one real GEMM through the embedding
//   a + ib -> [a, b] (row of the left vector),
//   B -> [[Re B, Im B], [-Im B, Re B]] (2x2 real block per complex entry),
// so the interleaved complex left vectors are the A operand as stored.
//
// Workgroup: 8 waves x 16 shots, two waves per SIMD.  Each wave keeps the
// T_p row block of its 16 shots in MFMA accumulators (v_mfma_f32_16x16x4f32
// tiles), reduces the squared norms across lanes and draws by weighted
// reservoir selection (p replaces the running choice when
// u (W_{p-1} + w_p) < w_p, one Philox uniform per p >= 1 keyed by
// (seed, shot, site)); a replacing T_p row is stored at once to the output
// rows, so no second register set holds the selection.  Rows are left
// unnormalised: the conditional probabilities do not depend on the scale of
// L, and the next site multiplies its A operand by the stored 1/|T_p|.
// B' arrives in LDS in K-chunks of 32 real rows, double buffered by the LDS
// DMA path, in the lane order the B operand needs, four k-steps per 16-byte
// LDS read.
#include "gbs_sampler.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kWaves = 8;              // waves per workgroup
constexpr int kShotsPerWg = 16 * kWaves;

// Packed layout of B' for one site, one 1 KiB block per (c, t, h):
//   P[p][c][t][h][lane][j] = B'[32 c + 8 (lane/16) + 4 h + j][16 t + lane%16]
// c: chunk of 32 real K rows, t: 16-column tile, h: half of the chunk's 8
// k-steps, j: k-step within the half (4 per 16-byte read).
__global__ void pack_kernel(const cplx32* __restrict__ B, int K, int d, int N, int Kp, int Np, float* __restrict__ P) {
  const long NT = (2L * Np) / 16;
  const long per_p = (long)(2 * Kp) * (2 * Np);
  long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= per_p * d) return;
  const int p = (int)(e / per_p);
  long r = e % per_p;
  const int j = (int)(r % 4);
  r /= 4;
  const int lane = (int)(r % 64);
  r /= 64;
  const int h = (int)(r % 2);
  r /= 2;
  const int t = (int)(r % NT);
  const int c = (int)(r / NT);
  const int kr = 32 * c + 8 * (lane / 16) + 4 * h + j;  // real row of B'
  const int nr = 16 * t + (lane % 16);                  // real column of B'
  const int k = kr >> 1, a = kr & 1, jj = nr >> 1, bcol = nr & 1;
  float v = 0.f;
  if (k < K && jj < N) {
    cplx32 z = B[((long)k * d + p) * N + jj];
    v = (a == 0) ? (bcol == 0 ? z.re : z.im) : (bcol == 0 ? -z.im : z.re);
  }
  P[e] = v;
}

template <int NT>
__global__ __launch_bounds__(64 * kWaves) void sample_mfma_kernel(
    const float* __restrict__ P, int nchunk, int d, const float* __restrict__ lin, const float* __restrict__ sin,
    float* __restrict__ lout, float* __restrict__ sout, long ldl2, int ncol_out, int64_t shot0, int64_t nshots,
    int site, uint32_t k0, uint32_t k1, int32_t* __restrict__ out, int M) {
  constexpr int CHUNK = 8 * NT * 64;      // floats per chunk
  constexpr int BLOCKS = CHUNK / 256;     // 1 KiB blocks per chunk (2 NT)
  constexpr int BPW = (BLOCKS + kWaves - 1) / kWaves;
  __shared__ __attribute__((aligned(16))) float Bs[2][CHUNK];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int grp = lane >> 4;   // k sub-block for A, row block for outputs
  const int col = lane & 15;
  const int64_t wbase = (int64_t)blockIdx.x * kShotsPerWg + w * 16;  // first shot of this wave (chunk-local)
  // A operand rows: lane row = col (shot wbase + col), k = 32c + 8 grp + i
  const int64_t arow = wbase + col;
  const bool avalid = arow < nshots;
  const float* arow_ptr = lin + (avalid ? arow : 0) * ldl2 + 8 * grp;
  const float ascale = (sin && avalid) ? sin[arow] : 1.f;
  floatx4 acc[NT];
  float wsum[4], wsel[4], uu[4][4];
  int psel[4];
  bool rowok[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    wsum[v] = 0.f;
    wsel[v] = 0.f;
    psel[v] = 0;
    rowok[v] = wbase + 4 * grp + v < nshots;
  }
  auto load_a = [&](int c, float* a) {
    float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0;
    if (avalid) {
      const float4* ap = (const float4*)(arow_ptr + 32 * c);
      a0 = ap[0];
      a1 = ap[1];
    }
    a[0] = a0.x * ascale; a[1] = a0.y * ascale; a[2] = a0.z * ascale; a[3] = a0.w * ascale;
    a[4] = a1.x * ascale; a[5] = a1.y * ascale; a[6] = a1.z * ascale; a[7] = a1.w * ascale;
  };
  // global -> LDS by the DMA path: lane l carries 16 bytes to block base + 16 l.
  // Chunks run as one sequence over (p, c), so the first chunk of p + 1 is in
  // flight while p's draw is made.
  auto issue = [&](int g, int buf) {
    const float* src = P + (long)g * CHUNK;
#pragma unroll
    for (int q = 0; q < BPW; ++q) {
      const int blk = w + kWaves * q;  // uniform per wave
      if (BLOCKS % kWaves != 0 && blk >= BLOCKS) break;
      __builtin_amdgcn_global_load_lds((const void*)(src + blk * 256 + lane * 4),
                                       (void __attribute__((address_space(3)))*)(&Bs[buf][blk * 256]), 16, 0, 0);
    }
  };
  const int total = d * nchunk;
  float a[8], an[8];
  issue(0, 0);
  load_a(0, a);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int p = 0; p < d; ++p) {
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < nchunk; ++c) {
      const int g = p * nchunk + c;
      const int buf = g & 1;
      if (g + 1 < total) {
        issue(g + 1, buf ^ 1);
        load_a(c + 1 < nchunk ? c + 1 : 0, an);
      }
      const float4* bsrc = (const float4*)Bs[buf];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int t0 = 0; t0 < NT; t0 += 2) {
          const float4 b0 = bsrc[((t0 + 0) * 2 + h) * 64 + lane];
          const float4 b1 = bsrc[((t0 + 1) * 2 + h) * 64 + lane];
          acc[t0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * h + 0], b0.x, acc[t0], 0, 0, 0);
          acc[t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * h + 0], b1.x, acc[t0 + 1], 0, 0, 0);
          acc[t0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * h + 1], b0.y, acc[t0], 0, 0, 0);
          acc[t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * h + 1], b1.y, acc[t0 + 1], 0, 0, 0);
          acc[t0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * h + 2], b0.z, acc[t0], 0, 0, 0);
          acc[t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * h + 2], b1.z, acc[t0 + 1], 0, 0, 0);
          acc[t0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * h + 3], b0.w, acc[t0], 0, 0, 0);
          acc[t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * h + 3], b1.w, acc[t0 + 1], 0, 0, 0);
        }
      }
      // the next chunk (B' in LDS, A in registers) was issued a whole chunk ago
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (g + 1 < total) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = an[i];
      }
    }
    // squared norms of the 4 rows this lane holds (rows 4*grp + v)
    float part[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float s = 0.f;
#pragma unroll
      for (int t = 0; t < NT; ++t) s += acc[t][v] * acc[t][v];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      s += __shfl_xor(s, 8, 64);
      part[v] = s;
    }
    if (p >= 1 && ((p - 1) & 3) == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gs = shot0 + wbase + 4 * grp + v;
        philox4 ctr;
        ctr.v[0] = (uint32_t)gs;
        ctr.v[1] = (uint32_t)((uint64_t)gs >> 32);
        ctr.v[2] = (uint32_t)site;
        ctr.v[3] = (uint32_t)((p - 1) >> 2);
        philox4 rr = philox4x32_10(ctr, k0, k1);
#pragma unroll
        for (int j = 0; j < 4; ++j) uu[v][j] = u01_24(rr.v[j]);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float wp = part[v];
      bool take;
      if (p == 0) {
        take = true;
      } else {
        const float u = uu[v][(p - 1) & 3];
        take = u * (wsum[v] + wp) < wp;
      }
      wsum[v] += wp;
      if (take) {
        psel[v] = p;
        wsel[v] = wp;
        if (rowok[v]) {
          float* orow = lout + (wbase + 4 * grp + v) * ldl2;
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const int cidx = 16 * t + col;
            if (cidx < ncol_out) orow[cidx] = acc[t][v];
          }
        }
      }
    }
  }
  // row scales and samples
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (!rowok[v]) continue;
    const int64_t ls = wbase + 4 * grp + v;
    if (col == 0) {
      sout[ls] = wsel[v] > 0.f ? 1.f / sqrtf(wsel[v]) : 0.f;
      out[(shot0 + ls) * (int64_t)M + (site - 1)] = psel[v];
    }
  }
}

// First left vectors: L = e_0 (the site-1 left bond has dimension 1), as
// `ncols` floats per row (the padded real width of that bond).
__global__ void init_rows_kernel(float* __restrict__ l, long ldl2, int ncols, int64_t n) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t r = e / ncols;
  const int c = (int)(e % ncols);
  l[r * ldl2 + c] = c == 0 ? 1.f : 0.f;
}

}  // namespace

hipError_t launch_sampler_init(hipStream_t st, float* l, long ldl2, int k0, int64_t n) {
  const int ncols = 2 * sampler_pad(k0);
  if (n <= 0) return hipSuccess;
  if (ncols > ldl2) return hipErrorInvalidValue;
  const int64_t tot = n * ncols;
  hipLaunchKernelGGL(init_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, l, ldl2, ncols, n);
  return hipGetLastError();
}

int sampler_pad(int n) { return (n + 15) / 16 * 16; }

int sampler_shots_per_block() { return kShotsPerWg; }

hipError_t launch_pack(hipStream_t st, const cplx32* B, int K, int d, int N, float* P) {
  const int Kp = sampler_pad(K), Np = sampler_pad(N);
  long n = (long)d * (2 * Kp) * (2 * Np);
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, K, d, N, Kp, Np, P);
  return hipGetLastError();
}

hipError_t launch_sample_mfma(hipStream_t st, const float* P, int K, int d, int N, const float* lin,
                              const float* sin, float* lout, float* sout, long ldl2, int64_t shot0, int64_t nshots,
                              int site, uint64_t seed, int32_t* out, int M) {
  const int Kp = sampler_pad(K), Np = sampler_pad(N);
  const int nchunk = (2 * Kp) / 32;
  const int NT = (2 * Np) / 16;
  const int ncol_out = 2 * Np;
  if (ncol_out > ldl2 || 2 * Kp > ldl2) return hipErrorInvalidValue;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  dim3 grid((unsigned)((nshots + kShotsPerWg - 1) / kShotsPerWg));
#define GBS_SAMPLE_CASE(NTV)                                                                                      \
  case NTV:                                                                                                       \
    hipLaunchKernelGGL((sample_mfma_kernel<NTV>), grid, dim3(64 * kWaves), 0, st, P, nchunk, d, lin, sin, lout,   \
                       sout, ldl2, ncol_out, shot0, nshots, site, k0, k1, out, M);                                \
    break;
  switch (NT) {
    GBS_SAMPLE_CASE(2)
    GBS_SAMPLE_CASE(4)
    GBS_SAMPLE_CASE(6)
    GBS_SAMPLE_CASE(8)
    GBS_SAMPLE_CASE(10)
    GBS_SAMPLE_CASE(12)
    GBS_SAMPLE_CASE(14)
    GBS_SAMPLE_CASE(16)
    GBS_SAMPLE_CASE(18)
    GBS_SAMPLE_CASE(20)
    GBS_SAMPLE_CASE(22)
    GBS_SAMPLE_CASE(24)
    GBS_SAMPLE_CASE(26)
    GBS_SAMPLE_CASE(28)
    GBS_SAMPLE_CASE(30)
    GBS_SAMPLE_CASE(32)
    default:
      return hipErrorInvalidValue;
  }
#undef GBS_SAMPLE_CASE
  return hipGetLastError();
}
