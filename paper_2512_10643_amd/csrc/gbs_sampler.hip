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
// Photon-parity sectors: every workgroup takes shots of one left sector pi
// (listed by the partition of the previous site's outcomes), so its K rows
// are those of sector pi and outcome p only needs the columns of sector
// pi ^ (p & 1); the blocks B[pi, p, pi ^ (p & 1)] are the only nonzero ones.
//
// Workgroup: 8 waves x 16 shots, two waves per SIMD.  Each wave keeps the
// T_p row block of its 16 shots in MFMA accumulators (v_mfma_f32_16x16x4f32
// tiles), reduces the squared norms across lanes and draws by weighted
// reservoir selection (p replaces the running choice when
// u (W_{p-1} + w_p) < w_p, one Philox uniform per p >= 1 keyed by
// (seed, shot, site)); a replacing T_p row is stored at once to the output
// row of its shot, so no second register set holds the selection.  Rows are
// left unnormalised: the conditional probabilities do not depend on the scale
// of L, and the next site multiplies its A operand by the stored 1/|T_p|.
// B' arrives in LDS in K-chunks of 32 real rows, double buffered by the LDS
// DMA path, in the lane order the B operand needs, four k-steps per 16-byte
// LDS read.
#include "gbs_sampler.h"

#include <algorithm>
#include <climits>

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kWaves = 8;              // waves per workgroup
constexpr int kShotsPerWg = 16 * kWaves;

// Per-launch geometry: for left sector pi, nchunk[pi] K-chunks of 32 real
// rows; right sector s is nt[s] 16-column tiles wide; pbase[pi] is the first
// float of sector pi's block in the packed operand.
struct SampleGeom {
  int nchunk[2];
  int nt[2];
  long pbase[2];
};

// Floats before chunk (p, c) inside a sector block: the outcomes p run in
// order, even p with nte tiles and odd p with nto tiles per chunk.
__host__ __device__ inline long chunk_offset(int nchunk, int nte, int nto, int p, int c) {
  const int ntp = (p & 1) ? nto : nte;
  return 512L * ((long)nchunk * (((p + 1) >> 1) * nte + (p >> 1) * nto) + (long)c * ntp);
}

SampleGeom make_geom(const SamplerSite& s, int d) {
  SampleGeom g;
  for (int i = 0; i < 2; ++i) {
    g.nchunk[i] = sampler_pad(s.nL[i]) / 16;
    g.nt[i] = sampler_pad(s.nR[i]) / 8;
  }
  sampler_site_floats(s, d, g.pbase);
  return g;
}

// Packed layout of B' for one site, per left sector pi and outcome p, one
// 1 KiB block per (c, t, h):
//   P[pi][p][c][t][h][lane][j] = B'_{pi,p}[32 c + 8 (lane/16) + 4 h + j][16 t + lane%16]
// where B'_{pi,p} is the real embedding of B restricted to the rows of left
// sector pi and the columns of right sector pi ^ (p & 1), in sector-local
// order.  c: chunk of 32 real K rows, t: 16-column tile, h: half of the
// chunk's 8 k-steps, j: k-step within the half (4 per 16-byte read).
__global__ void pack_kernel(const cplx32* __restrict__ B, int d, int N, SamplerSite s, SampleGeom g,
                            const int32_t* __restrict__ mapL, const int32_t* __restrict__ mapR,
                            float* __restrict__ P) {
  const int pi = blockIdx.y / d, p = blockIdx.y % d;
  if (s.nL[pi] == 0) return;
  const int sig = pi ^ (p & 1);
  const int ntp = g.nt[sig];
  const long per_chunk = 512L * ntp;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= per_chunk * g.nchunk[pi]) return;
  const int c = (int)(e / per_chunk);
  const int r = (int)(e % per_chunk);
  const int j = r & 3, lane = (r >> 2) & 63, h = (r >> 8) & 1, t = r >> 9;
  const int kr = 32 * c + 8 * (lane >> 4) + 4 * h + j;  // real row of B'
  const int nr = 16 * t + (lane & 15);                  // real column of B'
  const int k = kr >> 1, a = kr & 1, jj = nr >> 1, bcol = nr & 1;
  float v = 0.f;
  if (k < s.nL[pi] && jj < s.nR[sig]) {
    const int al = mapL ? mapL[(pi ? s.nL[0] : 0) + k] : k;
    const int be = mapR ? mapR[(sig ? s.nR[0] : 0) + jj] : jj;
    const cplx32 z = B[((long)al * d + p) * N + be];
    v = (a == 0) ? (bcol == 0 ? z.re : z.im) : (bcol == 0 ? -z.im : z.re);
  }
  P[g.pbase[pi] + chunk_offset(g.nchunk[pi], g.nt[pi], g.nt[pi ^ 1], p, 0) + e] = v;
}

// One thread per column b and a slice of the (a, p) rows; see launch_sector_mask.
__global__ __launch_bounds__(256) void sector_mask_kernel(const cplx32* __restrict__ B, int K, int d, int N,
                                                          const int32_t* __restrict__ mask_l,
                                                          int32_t* __restrict__ mask_r) {
  const int b = blockIdx.x * 64 + (threadIdx.x & 63);
  if (b >= N) return;
  const int rows = K * d;
  int m = 0;
  for (int r = blockIdx.y * 4 + (threadIdx.x >> 6); r < rows; r += 4 * gridDim.y) {
    const cplx32 z = B[(long)r * N + b];
    if (z.re != 0.f || z.im != 0.f) {
      const int a = r / d, p = r - a * d;
      const int pa = (mask_l && mask_l[a] == 2) ? 1 : 0;
      m |= 1 << ((pa + p) & 1);
    }
  }
  if (m) atomicOr(&mask_r[b], m);
}

template <int NT>
__global__ __launch_bounds__(64 * kWaves) void sample_mfma_kernel(
    const float* __restrict__ P, SampleGeom geo, int d, const float* __restrict__ lin,
    const float* __restrict__ sin, float* __restrict__ lout, float* __restrict__ sout, long ldl2,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ cnt, int8_t* __restrict__ par_out,
    int64_t shot0, int64_t nshots, int site, uint32_t k0, uint32_t k1, int32_t* __restrict__ out, int M) {
  __shared__ __attribute__((aligned(16))) float Bs[2][512 * NT];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int grp = lane >> 4;   // k sub-block for A, row block for outputs
  const int col = lane & 15;
  // sector of this workgroup and the end of its slot range
  int pi = 0;
  const int64_t slot0 = (int64_t)blockIdx.x * kShotsPerWg;
  int64_t send = nshots;
  if (perm) {
    const int64_t c0 = cnt[0], c1 = cnt[1];
    const int64_t e = (c0 + kShotsPerWg - 1) / kShotsPerWg * kShotsPerWg;
    if (slot0 < e) {
      send = c0;
    } else {
      pi = 1;
      send = e + c1;
    }
    if (slot0 >= send) return;  // whole workgroup, before any barrier
  }
  const int nchunk = geo.nchunk[pi];
  const int nte = geo.nt[pi], nto = geo.nt[pi ^ 1];
  const float* Pb = P + geo.pbase[pi];
  const int64_t wslot = slot0 + w * 16;  // first slot of this wave
  // A operand rows: lane row = col, k = 32c + 8 grp + i
  const bool avalid = wslot + col < send;
  const int64_t arow = avalid ? (perm ? (int64_t)perm[wslot + col] : wslot + col) : 0;
  const float* arow_ptr = lin + arow * ldl2 + 8 * grp;
  const float ascale = (sin && avalid) ? sin[arow] : 1.f;
  floatx4 acc[NT];
  float wsum[4], wsel[4], uu[4][4];
  int psel[4];
  bool rowok[4];
  int64_t oshot[4];  // chunk-local shot of output row 4 grp + v
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    wsum[v] = 0.f;
    wsel[v] = 0.f;
    psel[v] = 0;
    const int64_t sl = wslot + 4 * grp + v;
    rowok[v] = sl < send;
    oshot[v] = rowok[v] ? (perm ? (int64_t)perm[sl] : sl) : 0;
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
    const int p = g / nchunk, c = g - p * nchunk;
    const int ntp = (p & 1) ? nto : nte;
    const float* src = Pb + chunk_offset(nchunk, nte, nto, p, c);
    for (int blk = w; blk < 2 * ntp; blk += kWaves)  // uniform per wave
      __builtin_amdgcn_global_load_lds((const void*)(src + blk * 256 + lane * 4),
                                       (void __attribute__((address_space(3)))*)(&Bs[buf][blk * 256]), 16, 0, 0);
  };
  const int total = d * nchunk;
  float a[8], an[8];
  if (total > 0) {
    issue(0, 0);
    load_a(0, a);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int p = 0; p < d; ++p) {
    const int ntp = (p & 1) ? nto : nte;
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
          if (t0 < ntp) {
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
      }
      // the next chunk (B' in LDS, A in registers) was issued a whole chunk ago
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (g + 1 < total) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = an[i];
      }
    }
    // squared norms of the 4 rows this lane holds (rows 4*grp + v); tiles at
    // and beyond ntp stay zero
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
        const int64_t gs = shot0 + oshot[v];
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
          float* orow = lout + oshot[v] * ldl2;
#pragma unroll
          for (int t = 0; t < NT; ++t)
            if (t < ntp) orow[16 * t + col] = acc[t][v];
        }
      }
    }
  }
  // row scales, samples and the parity of the new bond index
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (!rowok[v]) continue;
    const int64_t ls = oshot[v];
    if (col == 0) {
      sout[ls] = wsel[v] > 0.f ? 1.f / sqrtf(wsel[v]) : 0.f;
      out[(shot0 + ls) * (int64_t)M + (site - 1)] = psel[v];
      if (par_out) par_out[ls] = (int8_t)((pi + psel[v]) & 1);
    }
  }
}

// Sum over the 256 threads of a block (every thread gets the total).
__device__ inline int block_sum256(int v, int* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

constexpr int kPartElems = 1024;  // parities per partition block (256 threads x 4)

__global__ __launch_bounds__(256) void part_count_kernel(const int8_t* __restrict__ par, int64_t n,
                                                         int32_t* __restrict__ bcnt) {
  __shared__ int sh[4];
  const int64_t base = (int64_t)blockIdx.x * kPartElems + 4 * threadIdx.x;
  int c = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (base + j < n && par[base + j] == 0) ++c;
  c = block_sum256(c, sh);
  if (threadIdx.x == 0) bcnt[blockIdx.x] = c;
}

__global__ __launch_bounds__(256) void part_scatter_kernel(const int8_t* __restrict__ par, int64_t n,
                                                           const int32_t* __restrict__ bcnt, int nblk,
                                                           int32_t* __restrict__ perm, int32_t* __restrict__ cnt) {
  __shared__ int sh[4];
  __shared__ int wtot[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int before = 0, tot = 0;
  for (int i = tid; i < nblk; i += 256) {
    const int v = bcnt[i];
    tot += v;
    if (i < (int)blockIdx.x) before += v;
  }
  before = block_sum256(before, sh);
  tot = block_sum256(tot, sh);
  const int64_t c0 = tot;
  const int64_t e = (c0 + kShotsPerWg - 1) / kShotsPerWg * kShotsPerWg;
  const int64_t blk0 = (int64_t)blockIdx.x * kPartElems;
  const int64_t base = blk0 + 4 * tid;
  int q[4];
  int ne = 0, no = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    q[j] = base + j < n ? (int)par[base + j] : -1;
    ne += q[j] == 0;
    no += q[j] == 1;
  }
  // exclusive scan of (even, odd) counts packed in 16-bit halves
  const int v = ne | (no << 16);
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wtot[w] = x;
  __syncthreads();
  int wpre = 0;
  for (int i = 0; i < w; ++i) wpre += wtot[i];
  const int ex = x - v + wpre;
  int64_t re = before + (ex & 0xffff);
  int64_t ro = e + (blk0 - before) + (ex >> 16);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (q[j] == 0) perm[re++] = (int32_t)(base + j);
    else if (q[j] == 1) perm[ro++] = (int32_t)(base + j);
  }
  if (blockIdx.x == 0 && tid == 0) {
    cnt[0] = (int32_t)c0;
    cnt[1] = (int32_t)(n - c0);
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

long sampler_site_floats(const SamplerSite& s, int d, long pbase[2]) {
  long tot = 0;
  for (int pi = 0; pi < 2; ++pi) {
    if (pbase) pbase[pi] = tot;
    if (s.nL[pi] <= 0) continue;
    const long nchunk = sampler_pad(s.nL[pi]) / 16;
    const long nte = sampler_pad(s.nR[pi]) / 8, nto = sampler_pad(s.nR[pi ^ 1]) / 8;
    tot += 512L * nchunk * (((d + 1) / 2) * nte + (d / 2) * nto);
  }
  return tot;
}

hipError_t launch_sector_mask(hipStream_t st, const cplx32* B, int K, int d, int N, const int32_t* mask_l,
                              int32_t* mask_r) {
  if (K <= 0 || N <= 0 || d <= 0) return hipErrorInvalidValue;
  const int rows = K * d;
  const int gy = std::max(1, std::min(64, (rows + 63) / 64));
  hipLaunchKernelGGL(sector_mask_kernel, dim3((unsigned)((N + 63) / 64), (unsigned)gy), dim3(256), 0, st, B, K, d,
                     N, mask_l, mask_r);
  return hipGetLastError();
}

hipError_t launch_pack(hipStream_t st, const cplx32* B, int K, int d, int N, const SamplerSite& s,
                       const int32_t* mapL, const int32_t* mapR, float* P) {
  if (s.nL[0] + s.nL[1] > K || (mapR && s.nR[0] + s.nR[1] > N) || (!mapR && (s.nR[0] > N || s.nR[1] > N)))
    return hipErrorInvalidValue;
  const SampleGeom g = make_geom(s, d);
  long mx = 0;
  for (int pi = 0; pi < 2; ++pi)
    for (int q = 0; q < 2; ++q) mx = std::max(mx, 512L * g.nchunk[pi] * g.nt[q]);
  if (mx == 0) return hipSuccess;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((mx + 255) / 256), (unsigned)(2 * d)), dim3(256), 0, st, B, d, N,
                     s, g, mapL, mapR, P);
  return hipGetLastError();
}

hipError_t launch_sample_mfma(hipStream_t st, const float* P, int d, const SamplerSite& s, const float* lin,
                              const float* sin, float* lout, float* sout, long ldl2, const int32_t* perm,
                              const int32_t* cnt, int8_t* par_out, int64_t shot0, int64_t nshots, int site,
                              uint64_t seed, int32_t* out, int M) {
  if (nshots <= 0) return hipSuccess;
  if ((perm == nullptr) != (cnt == nullptr)) return hipErrorInvalidValue;
  if (!perm && s.nL[1] != 0) return hipErrorInvalidValue;
  const SampleGeom g = make_geom(s, d);
  for (int i = 0; i < 2; ++i)
    if (32L * g.nchunk[i] > ldl2 || 16L * g.nt[i] > ldl2) return hipErrorInvalidValue;
  const int NT = std::max(g.nt[0], g.nt[1]);
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  // with a partition, sector 1 starts on a fresh workgroup: one more block
  dim3 grid((unsigned)((nshots + kShotsPerWg - 1) / kShotsPerWg + (perm ? 1 : 0)));
#define GBS_SAMPLE_CASE(NTV)                                                                                      \
  case NTV:                                                                                                       \
    hipLaunchKernelGGL((sample_mfma_kernel<NTV>), grid, dim3(64 * kWaves), 0, st, P, g, d, lin, sin, lout, sout, \
                       ldl2, perm, cnt, par_out, shot0, nshots, site, k0, k1, out, M);                           \
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

int64_t sampler_partition_blocks(int64_t nshots) { return (nshots + kPartElems - 1) / kPartElems; }

hipError_t launch_sampler_partition(hipStream_t st, const int8_t* par, int64_t nshots, int32_t* bcnt,
                                    int32_t* perm, int32_t* cnt) {
  if (nshots <= 0) return hipSuccess;
  if (nshots > INT32_MAX - 256) return hipErrorInvalidValue;
  const int nblk = (int)sampler_partition_blocks(nshots);
  hipLaunchKernelGGL(part_count_kernel, dim3((unsigned)nblk), dim3(256), 0, st, par, nshots, bcnt);
  hipLaunchKernelGGL(part_scatter_kernel, dim3((unsigned)nblk), dim3(256), 0, st, par, nshots, bcnt, nblk, perm,
                     cnt);
  return hipGetLastError();
}
