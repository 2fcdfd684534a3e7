// Sampling sweep on MFMA (FP32), one site per launch.
//
// For every shot s the conditional step at site m computes T_p = L_s B[:, p, :]
// for p < d, draws p with probability |T_p|^2 / sum_p' |T_p'|^2 and continues
// with L_s <- T_p / |T_p| (sequential conditional sampling on a right-canonical
// MPS).  The complex products are one real GEMM through the embedding
//   a + ib -> [a, b] (row of the left vector),
//   B -> [[Re B, Im B], [-Im B, Re B]] (2x2 real block per complex entry),
// so the interleaved complex left vectors are the A operand as stored.
//
// Workgroup: 4 waves x 16 shots.  Each wave keeps the full T_p row block of its
// 16 shots in MFMA accumulators (v_mfma_f32_16x16x4f32 tiles), reduces the
// squared norms across lanes, and keeps the selected T_p (weighted reservoir
// choice, one Philox uniform per p >= 1 keyed by (seed, shot, site)) in a
// second register set.  B' arrives in LDS in K-chunks of 32 real rows, double
// buffered, in the exact lane order the MFMA B operand needs.
#include "gbs_sampler.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

// Packed layout of B' for one site:
//   P[p][c][i][t][lane] = B'[32 c + 8 (lane/16) + i][16 t + lane%16]
// c: chunk of 32 real K rows, i: MFMA k-step within the chunk (8),
// t: 16-column tile, lane: 0..63.
__global__ void pack_kernel(const cplx32* __restrict__ B, int K, int d, int N, int Kp, int Np, float* __restrict__ P) {
  const long NT = (2L * Np) / 16;
  const long per_p = (long)(2 * Kp) * (2 * Np);
  long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= per_p * d) return;
  const int p = (int)(e / per_p);
  long r = e % per_p;
  const int lane = (int)(r % 64);
  r /= 64;
  const int t = (int)(r % NT);
  r /= NT;
  const int i = (int)(r % 8);
  const int c = (int)(r / 8);
  const int kr = 32 * c + 8 * (lane / 16) + i;  // real row of B'
  const int nr = 16 * t + (lane % 16);          // real column of B'
  const int k = kr >> 1, a = kr & 1, j = nr >> 1, bcol = nr & 1;
  float v = 0.f;
  if (k < K && j < N) {
    cplx32 z = B[((long)k * d + p) * N + j];
    v = (a == 0) ? (bcol == 0 ? z.re : z.im) : (bcol == 0 ? -z.im : z.re);
  }
  P[e] = v;
}

template <int NT>
__global__ __launch_bounds__(256) void sample_mfma_kernel(const float* __restrict__ P, int nchunk, int d,
                                                          const float* __restrict__ lin, float* __restrict__ lout,
                                                          long ldl2, int ncol_out, int64_t shot0, int64_t nshots,
                                                          int site, uint32_t k0, uint32_t k1,
                                                          int32_t* __restrict__ out, int M) {
  constexpr int CHUNK = 8 * NT * 64;  // floats per chunk
  __shared__ float Bs[2][CHUNK];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int grp = lane >> 4;   // k sub-block for A, row block for outputs
  const int col = lane & 15;
  const int64_t wbase = (int64_t)blockIdx.x * 64 + w * 16;  // first shot of this wave (chunk-local)
  // A operand rows: lane row = col (shot wbase + col), k = 32c + 8 grp + i
  const int64_t arow = wbase + col;
  const bool avalid = arow < nshots;
  const float* arow_ptr = lin + (avalid ? arow : 0) * ldl2;
  floatx4 acc[NT], sel[NT];
  float wsum[4], wsel[4], uu[4][4];
  int psel[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    wsum[v] = 0.f;
    wsel[v] = 0.f;
    psel[v] = 0;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) sel[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  // B' chunks are copied global -> LDS by the LDS DMA path (each wave moves
  // 1 KiB blocks: lane l carries 16 bytes to block base + 16 l).
  constexpr int BLOCKS = CHUNK / 256;       // 1 KiB blocks per chunk
  constexpr int BPW = BLOCKS / 4;           // blocks per wave
  for (int p = 0; p < d; ++p) {
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* pbase = P + (long)p * nchunk * CHUNK;
    auto issue = [&](int c, int buf) {
      const float* src = pbase + (long)c * CHUNK;
#pragma unroll
      for (int q = 0; q < BPW; ++q) {
        const int blk = w + 4 * q;
        __builtin_amdgcn_global_load_lds((const void*)(src + blk * 256 + lane * 4),
                                         (void __attribute__((address_space(3)))*)(&Bs[buf][blk * 256]), 16, 0, 0);
      }
    };
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
      const int buf = c & 1;
      if (c + 1 < nchunk) issue(c + 1, buf ^ 1);
      // A operand for this chunk: 8 consecutive floats of the lane's row
      float a[8];
      {
        const float4* ap = (const float4*)(arow_ptr + 32 * c + 8 * grp);
        float4 a0 = avalid ? ap[0] : make_float4(0.f, 0.f, 0.f, 0.f);
        float4 a1 = avalid ? ap[1] : make_float4(0.f, 0.f, 0.f, 0.f);
        a[0] = a0.x; a[1] = a0.y; a[2] = a0.z; a[3] = a0.w;
        a[4] = a1.x; a[5] = a1.y; a[6] = a1.z; a[7] = a1.w;
      }
      const float* bsrc = Bs[buf];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          float b = bsrc[(i * NT + t) * 64 + lane];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b, acc[t], 0, 0, 0);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    // squared norms of the 4 rows this lane holds (rows 4*grp + v)
    float part[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float s = 0.f;
#pragma unroll
      for (int t = 0; t < NT; ++t) s += acc[t][v] * acc[t][v];
      part[v] = s;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float s = part[v];
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
#pragma unroll
        for (int t = 0; t < NT; ++t) sel[t][v] = acc[t][v];
      }
    }
  }
  // write the normalised selected rows and the samples
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t ls = wbase + 4 * grp + v;
    if (ls >= nshots) continue;
    const float inv = wsel[v] > 0.f ? 1.f / sqrtf(wsel[v]) : 0.f;
    float* orow = lout + ls * ldl2;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int cidx = 16 * t + col;
      if (cidx < ncol_out) orow[cidx] = sel[t][v] * inv;
    }
    if (col == 0) out[(shot0 + ls) * (int64_t)M + (site - 1)] = psel[v];
  }
}

}  // namespace

int sampler_pad(int n) { return (n + 15) / 16 * 16; }

hipError_t launch_pack(hipStream_t st, const cplx32* B, int K, int d, int N, float* P) {
  const int Kp = sampler_pad(K), Np = sampler_pad(N);
  long n = (long)d * (2 * Kp) * (2 * Np);
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, K, d, N, Kp, Np, P);
  return hipGetLastError();
}

hipError_t launch_sample_mfma(hipStream_t st, const float* P, int K, int d, int N, const float* lin, float* lout,
                              long ldl2, int64_t shot0, int64_t nshots, int site, uint64_t seed, int32_t* out,
                              int M) {
  const int Kp = sampler_pad(K), Np = sampler_pad(N);
  const int nchunk = (2 * Kp) / 32;
  const int NT = (2 * Np) / 16;
  const int ncol_out = 2 * Np;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  dim3 grid((unsigned)((nshots + 63) / 64));
#define GBS_SAMPLE_CASE(NTV)                                                                                   \
  case NTV:                                                                                                    \
    hipLaunchKernelGGL((sample_mfma_kernel<NTV>), grid, dim3(256), 0, st, P, nchunk, d, lin, lout, ldl2,       \
                       ncol_out, shot0, nshots, site, k0, k1, out, M);                                         \
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
