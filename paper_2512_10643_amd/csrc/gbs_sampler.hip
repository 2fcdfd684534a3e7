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
// Draw by inverse CDF with early stopping.  The site tensors are right-
// canonical (sum_p B_p B_p^dag = 1) and each left vector enters with unit
// norm, so the conditional probabilities |T_p|^2 of one shot sum to 1 before
// any of them is known.  With one uniform u per (shot, site) (Philox keyed by
// the seed, counter (shot, site)), outcomes are visited in the order
// 0, 1, 2, ... and the first p whose running sum exceeds u is taken; the
// outcomes after it are never formed.  Outcome 0 is its own first pass, and
// a site runs in two launches: the first pass for every shot, then, for the
// shots still undecided (listed by a partition), the remaining passes, where
// a workgroup stops as soon as all of its shots are decided.  A shot whose u
// lies above the rounded total keeps the last outcome of positive
// probability (outcome 0 if none): each pass stores the row of its taken
// outcome, or of its last positive one as a provisional choice.
//
// Workgroup: 8 waves x 16 shots, two waves per SIMD.  Each wave keeps the
// row block of its 16 shots for all outcomes of a pass in MFMA accumulators
// (v_mfma_f32_16x16x4f32 tiles) and reduces the squared norms across lanes.
// Rows are stored normalised (each scaled by 1/|T_p| as it is written), so
// they enter the next site as they are.  B' arrives in LDS in K-chunks of 32 real rows, double
// buffered by the LDS DMA path into two separate LDS arrays (so reads of one
// need not wait for the DMA into the other), in the lane order the B operand
// needs, four k-steps per 16-byte LDS read.
#include "gbs_sampler.h"

#include <algorithm>
#include <climits>
#include <map>
#include <mutex>

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kWaves = 8;              // waves per workgroup
constexpr int kShotsPerWg = 16 * kWaves;
// Waves per workgroup of the launches after a site's first (the few shots
// the first pass leaves undecided): workgroups of 64 shots stop sooner than
// 128 and spread those shots over more compute units.  Their grid is
// kRestGridMult times the resident workgroups, so the device hands blocks
// to compute units as they free up (blocks of hard shots run longer).
constexpr int kRestWaves = 4;
constexpr int kRestGridMult = 4;
// Key of a shot after a site's first launch: kKeyDone once decided, else
// its left sector and one of kKeyBuckets buckets (see shot_key)
constexpr int kKeyBuckets = 4;
constexpr int8_t kKeyDone = 127;

// Packed layout of B' for one site, per left sector pi and pass q, one 1 KiB
// block per (c, t, h):
//   P[pi][q][c][t][h][lane][j] = B'_{pi,q}[32 c + 16 h + 4 (lane/16) + j][16 t + lane%16]
// where B'_{pi,q} is the real embedding of B restricted to the rows of left
// sector pi (sector-local order) and, side by side, the columns of right
// sector pi ^ (p & 1) of every outcome p of the pass, each padded to whole
// tiles.  c: chunk of 32 real K rows, t: 16-column tile, h: half of the
// chunk (16 rows, 4 k-steps), j: k-step within the half (4 per 16-byte
// read).  A half last chunk stores only its h = 0 blocks.
//
// One thread per complex entry z of B: its 2 x 2 real block [[re, im],
// [-im, re]] (rows a, columns b of the embedding) sits at lanes 2l, 2l + 1
// and k-steps 2m, 2m + 1 of the layout, i.e. two float2 pairs 4 floats
// apart.  Thread order within a chunk is (t, h, l, m), so a wave writes 1 KB
// of P contiguously and reads 8 complex rows of 8 adjacent columns of B.
__device__ __forceinline__ void pack_body(const cplx32* __restrict__ B, int d, int N, const SamplerSite& s,
                                          const SamplerGeom* __restrict__ g, const int32_t* __restrict__ mapL,
                                          const int32_t* __restrict__ mapR, float* __restrict__ P) {
  const int pi = blockIdx.y / kSamplerMaxOutcomes, q = blockIdx.y % kSamplerMaxOutcomes;
  if (s.nL[pi] == 0 || q >= g->npass[pi]) return;
  const int T = g->tiles[pi][q];
  const long per_chunk = 128L * T;  // complex entries of a full chunk
  const int nfull = g->nchunk[pi] - g->half[pi];
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= per_chunk * nfull + (g->half[pi] ? 64L * T : 0)) return;
  int c, r, h, t;
  long o;  // float offset of the thread's first pair within the pass
  if (e < per_chunk * nfull) {
    c = (int)(e / per_chunk);
    r = (int)(e % per_chunk);
    h = (r >> 6) & 1;
    t = r >> 7;
    o = 512L * T * c + ((long)t << 9) + (h << 8);
  } else {  // half chunk: blocks (t, h = 0) only
    c = nfull;
    r = (int)(e - per_chunk * nfull);
    h = 0;
    t = r >> 6;
    o = 512L * T * c + ((long)t << 8);
  }
  const int m = r & 1, l = (r >> 1) & 31;  // k-step pair, lane pair
  o += (l << 3) + (m << 1);
  // the outcome owning tile t
  int p = g->j0[pi][q], sig = pi ^ (p & 1);
  while (t >= g->nt[sig]) {
    t -= g->nt[sig];
    ++p;
    sig = pi ^ (p & 1);
  }
  const int k = 16 * c + 8 * h + 2 * (l >> 3) + m;  // complex row of B restricted to sector pi
  const int jj = 8 * t + (l & 7);                   // complex column within outcome p
  float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
  if (k < s.nL[pi] && jj < s.nR[sig]) {
    const int al = mapL ? mapL[(pi ? s.nL[0] : 0) + k] : k;
    const int be = mapR ? mapR[(sig ? s.nR[0] : 0) + jj] : jj;
    const cplx32 z = B[((long)al * d + p) * N + be];
    lo = make_float2(z.re, -z.im);  // column b = 0: rows a = 0, 1
    hi = make_float2(z.im, z.re);   // column b = 1
  }
  float* dst = P + g->base[pi][q] + o;
  *(float2*)dst = lo;
  *(float2*)(dst + 4) = hi;
}

__global__ void pack_kernel(const cplx32* __restrict__ B, int d, int N, SamplerSite s,
                            const SamplerGeom* __restrict__ g, const int32_t* __restrict__ mapL,
                            const int32_t* __restrict__ mapR, float* __restrict__ P) {
  pack_body(B, d, N, s, g, mapL, mapR, P);
}

// Every site's packing in one launch (site blockIdx.z).
__global__ void pack_batch_kernel(const SamplerPackDesc* __restrict__ desc) {
  const SamplerPackDesc& q = desc[blockIdx.z];
  pack_body(q.B, q.d, q.N, q.s, q.g, q.mapL, q.mapR, q.P);
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

// An undecided shot's bucket measures how far its uniform ur lies past the
// running sum csum, relative to the probability still to come (1 - csum,
// rows being of unit norm): thresholds 1/2, 3/4 and 9/10.  The remaining
// launch takes the shots sorted by bucket, so its workgroups of low buckets,
// which mostly need one more outcome, stop early.
__device__ __forceinline__ int8_t shot_key(bool fin, int pi, float ur, float csum) {
  if (fin) return kKeyDone;
  const float dlt = ur - csum, rest = 1.f - csum;
  const int b = (dlt >= 0.5f * rest) + (dlt >= 0.75f * rest) + (dlt >= 0.9f * rest);
  return (int8_t)(pi * kKeyBuckets + b);
}

// One MFMA step with the B' fragment as the A operand and the left vectors as
// the B operand: the accumulator tile is T^T, so lane (grp, col) holds
// columns 16 t + 4 grp + v (v = 0..3) of shot col.
#define GBS_MF(T_, AV, BV) acc[T_] = __builtin_amdgcn_mfma_f32_16x16x4f32(BV, AV, acc[T_], 0, 0, 0)

// MFMAs of one K-chunk: tiles [0, T) of the accumulators from the B' chunk
// in LDS at bsrc and this lane's eight scaled A values; hc: the chunk holds
// k-half 0 only.
template <int NT>
__device__ __forceinline__ void chunk_mfma(floatx4 (&acc)[NT], const float4* __restrict__ bsrc, const float (&a)[8],
                                           int T, bool hc, int lane) {
        // Tile pairs in order.  The four B' fragments of pair k + 1 (both
        // k-halves) are read while pair k's MFMAs issue, into the other of two
        // register sets; pair k waits only for reads issued a whole pair
        // earlier.  A read past the pass's last pair stays inside the buffer
        // and is not used.
        float4 F[2][4];
        F[0][0] = bsrc[(0 * 2 + 0) * 64 + lane];
        F[0][1] = bsrc[(1 * 2 + 0) * 64 + lane];
        F[0][2] = bsrc[(0 * 2 + 1) * 64 + lane];
        F[0][3] = bsrc[(1 * 2 + 1) * 64 + lane];
  #pragma unroll
        for (int t0 = 0; t0 < NT; t0 += 2) {
          if (t0 < T) {
            const int cs = (t0 >> 1) & 1, ns = cs ^ 1;
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this pair's fragments are in
            if (t0 + 2 < NT) {
              F[ns][0] = bsrc[((t0 + 2) * 2 + 0) * 64 + lane];
              F[ns][1] = bsrc[((t0 + 3) * 2 + 0) * 64 + lane];
              F[ns][2] = bsrc[((t0 + 2) * 2 + 1) * 64 + lane];
              F[ns][3] = bsrc[((t0 + 3) * 2 + 1) * 64 + lane];
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the MFMAs
            GBS_MF(t0, a[0], F[cs][0].x);
            GBS_MF(t0 + 1, a[0], F[cs][1].x);
            GBS_MF(t0, a[1], F[cs][0].y);
            GBS_MF(t0 + 1, a[1], F[cs][1].y);
            GBS_MF(t0, a[2], F[cs][0].z);
            GBS_MF(t0 + 1, a[2], F[cs][1].z);
            GBS_MF(t0, a[3], F[cs][0].w);
            GBS_MF(t0 + 1, a[3], F[cs][1].w);
            if (!hc) {  // k-half 1 (absent from a half chunk)
              GBS_MF(t0, a[4], F[cs][2].x);
              GBS_MF(t0 + 1, a[4], F[cs][3].x);
              GBS_MF(t0, a[5], F[cs][2].y);
              GBS_MF(t0 + 1, a[5], F[cs][3].y);
              GBS_MF(t0, a[6], F[cs][2].z);
              GBS_MF(t0 + 1, a[6], F[cs][3].z);
              GBS_MF(t0, a[7], F[cs][2].w);
              GBS_MF(t0 + 1, a[7], F[cs][3].w);
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
}

// Draws after the last chunk of a pass over outcomes [j0, j1): squared norms
// of this lane's shot per outcome (outcome p owns the accumulator tiles
// [lo, hi), nte / nto tiles for even / odd p), inverse CDF against ur with
// the running sum csum, and the store of the taken or provisional row to
// orow (this lane's column quad of its shot's output row).
template <int NT>
__device__ __forceinline__ void pass_draws(const floatx4 (&acc)[NT], int j0, int j1, int nte, int nto, float ur,
                                           float& csum, bool& done, bool& wrote, int& psel, float& wsel, bool valid,
                                           float* orow0) {
  int lo = 0, slo = 0, shi = 0;
  bool pick = false;
  for (int p = j0; p < j1; ++p) {
    const int hi = lo + ((p & 1) ? nto : nte);
    // squared norm of this lane's shot: its 4 columns per tile, then the
    // four column quads
    float part = 0.f;
    if (j1 - j0 == 1) {
      // the pass's only outcome owns every nonzero tile
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) part = fmaf(acc[t][v], acc[t][v], part);
    } else {
      const uint32_t own = (hi >= 32 ? 0xffffffffu : ((1u << hi) - 1u)) &
                           ~(lo >= 32 ? 0xffffffffu : ((1u << lo) - 1u));
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float f = ((own >> t) & 1u) ? 1.f : 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) part = fmaf(f * acc[t][v], acc[t][v], part);
      }
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (!done) {
      csum += part;
      // taken when the running sum passes u; otherwise the last outcome of
      // positive weight (outcome 0 in any case) is the provisional one
      done = ur < csum;
      if (done || part > 0.f || p == 0) {
        pick = true;
        psel = p;
        wsel = part;
        slo = lo;
        shi = hi;
      }
    }
    lo = hi;
  }
  if (pick) {
    wrote = true;
    if (valid) {
      const uint32_t own = (shi >= 32 ? 0xffffffffu : ((1u << shi) - 1u)) &
                           ~(slo >= 32 ? 0xffffffffu : ((1u << slo) - 1u));
      // the row of outcome psel, normalised (a row of zero weight stays zero)
      const float sc = wsel > 0.f ? 1.f / sqrtf(wsel) : 0.f;
      float* orow = orow0 - 16 * slo;
#pragma unroll
      for (int t = 0; t < NT; ++t)
        if ((own >> t) & 1u)
          *(float4*)(orow + 16 * t) = make_float4(acc[t][0] * sc, acc[t][1] * sc, acc[t][2] * sc, acc[t][3] * sc);
    }
  }
}

// Passes [qbeg, qend) of one site for the 128 slots of workgroup `blk` (used
// for the remaining passes of the shots a site's first launch left
// undecided, and, over all passes, by the batched sweep).  Bs0, Bs1: the
// kernel's two LDS operand buffers (512 NT floats each, two separate arrays
// so the compiler can tell the buffer being read from the one the DMA is
// filling); wdone: W ints of LDS.  W waves of 16 shots per workgroup (W
// divides kWaves, so a block never straddles the 128-aligned start of the
// sector-1 slots).
template <int NT, int W>
__device__ __forceinline__ void sample_passes(
    float* __restrict__ Bs0, float* __restrict__ Bs1, int* __restrict__ wdone, int64_t blk,
    const float* __restrict__ P, const SamplerGeom* __restrict__ geo, const float* __restrict__ lin,
    float* __restrict__ lout, long ldl2, const int32_t* __restrict__ perm, const int32_t* __restrict__ cnt,
    int8_t* __restrict__ par_out, float* __restrict__ cum, int8_t* __restrict__ key, int qbeg, int qend,
    int64_t shot0, int64_t nshots, int site, uint32_t k0, uint32_t k1, int32_t* __restrict__ out, int M) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, scalar
  const int grp = lane >> 4;   // k sub-block of the left vector; column quad of the output
  const int col = lane & 15;   // shot within the wave
  // sector of this workgroup and the end of its slot range
  static_assert(kWaves % W == 0, "W must divide kWaves");
  int pi = 0;
  const int64_t slot0 = blk * 16 * W;
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
  // this lane's shot: left-vector row for the MFMA operand and output row
  const int64_t slot = slot0 + w * 16 + col;
  const bool valid = slot < send;
  const int64_t shot = valid ? (perm ? (int64_t)perm[slot] : slot) : 0;
  const int npass = geo->npass[pi];
  const int qlast = min(qend, npass);
  if (qbeg >= qlast) {
    // no rows in this left sector: outcome 0 with weight zero (a shot cannot
    // reach an empty sector with positive probability)
    if (valid && grp == 0 && qbeg == 0) {
      out[(shot0 + shot) * (int64_t)M + (site - 1)] = 0;
      if (par_out) par_out[shot] = (int8_t)pi;
      if (key) key[shot] = kKeyDone;
    }
    return;  // uniform over the workgroup
  }
  const int nchunk = geo->nchunk[pi];
  const bool halfk = geo->half[pi] != 0;  // last chunk of each pass is half
  const int nte = geo->nt[pi], nto = geo->nt[pi ^ 1];
  const float* arow_ptr = lin + shot * ldl2 + 4 * grp;
  // the shot's uniform (every lane of the shot draws the same one) and the
  // running sum of its conditional probabilities
  float ur, csum = (qbeg > 0 && valid) ? cum[shot] : 0.f;
  {
    const int64_t gs = shot0 + shot;
    philox4 ctr;
    ctr.v[0] = (uint32_t)gs;
    ctr.v[1] = (uint32_t)((uint64_t)gs >> 32);
    ctr.v[2] = (uint32_t)site;
    ctr.v[3] = 0u;
    ur = u01_24(philox4x32_10(ctr, k0, k1).v[0]);
  }
  bool done = false, wrote = false;
  int psel = 0;
  float wsel = 0.f;
  floatx4 acc[NT];
  // A rows are loaded into `an` and copied to the operand only when they
  // become current, so nothing waits on the loads before the end of the
  // chunk.  A lane past the end of the slot range reads row 0 (in bounds); it
  // feeds only its own output column, which is never stored.
  auto load_a = [&](int c, float4* r) {
    r[0] = *(const float4*)(arow_ptr + 32 * c);       // k-half 0: rows 32c + 4 grp + (0..3)
    r[1] = *(const float4*)(arow_ptr + 32 * c + 16);  // k-half 1: 16 rows further
  };
  auto take_a = [&](const float4* r, float* a) {
    a[0] = r[0].x; a[1] = r[0].y; a[2] = r[0].z; a[3] = r[0].w;
    a[4] = r[1].x; a[5] = r[1].y; a[6] = r[1].z; a[7] = r[1].w;
  };
  // global -> LDS by the DMA path: lane l carries 16 bytes to block base + 16 l.
  // Chunks run as one sequence over (pass, c), so the first chunk of the next
  // pass is in flight while this pass's draws are made.
  auto issue = [&](const float* src, int T, float* dst, bool halfc) {
    if (halfc) {  // blocks (t, h = 0) of a half chunk land where a full chunk has them
      for (int blk = w; blk < T; blk += W)
        __builtin_amdgcn_global_load_lds((const void*)(src + blk * 256 + lane * 4),
                                         (void __attribute__((address_space(3)))*)(dst + 2 * blk * 256), 16, 0, 0);
    } else {
      for (int blk = w; blk < 2 * T; blk += W)  // uniform per wave
        __builtin_amdgcn_global_load_lds((const void*)(src + blk * 256 + lane * 4),
                                         (void __attribute__((address_space(3)))*)(dst + blk * 256), 16, 0, 0);
    }
  };
  const int total = (qlast - qbeg) * nchunk;
  // the chunk being multiplied (pass q, chunk c, T tiles) and the one being
  // fetched (nq, nc, nT from nsrc), stepped without divisions; pass
  // parameters are read from the geometry only when a pass starts
  int q = qbeg, c = 0, T = geo->tiles[pi][qbeg];
  int nq = qbeg, nc = 0, nT = T;
  const float* nsrc = P + geo->base[pi][qbeg];
  auto advance_next = [&]() {
    if (++nc == nchunk) {
      nc = 0;
      if (++nq < qlast) {
        nT = geo->tiles[pi][nq];
        nsrc = P + geo->base[pi][nq];
      }
    } else {
      nsrc += 512L * nT;
    }
  };
  float a[8];
  float4 an[2];
  issue(nsrc, nT, Bs0, halfk && nchunk == 1);
  load_a(0, an);
  advance_next();
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  take_a(an, a);
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  // chunk g of the sequence over (pass, c): MFMAs on one buffer while chunk
  // g + 1 streams into the other (u fixes which buffer at compile time); the
  // draws follow the last chunk of each pass
  bool stop = false;
  for (int g0 = 0; g0 < total && !stop; g0 += 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int g = g0 + u;
      if (g >= total) break;
      if (g + 1 < total) issue(nsrc, nT, u ? Bs0 : Bs1, halfk && nc == nchunk - 1);
      if (g + 1 < total) load_a(nc, an);
      const float4* bsrc = (const float4*)(u ? Bs1 : Bs0);
      const bool hc = halfk && c == nchunk - 1;  // this chunk holds k-half 0 only
      chunk_mfma<NT>(acc, bsrc, a, T, hc, lane);
      // every wave's share of chunk g + 1 (and its A rows) has landed, and
      // its LDS reads of chunk g are done, before any wave goes on
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_s_barrier();
      if (g + 1 < total) take_a(an, a);
      if (c == nchunk - 1) {
        pass_draws<NT>(acc, geo->j0[pi][q], geo->j0[pi][q + 1], nte, nto, ur, csum, done, wrote, psel, wsel, valid,
                       lout + shot * ldl2 + 4 * grp);
        // the next pass accumulates from zero
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        if (q + 1 < qlast) {
          // the workgroup stops once every one of its shots is decided; the
          // chunk already in flight is waited for first
          const int wall = __all(done || !valid);
          if (lane == 0) wdone[w] = wall;
          __syncthreads();
          int all = 1;
#pragma unroll
          for (int i = 0; i < W; ++i) all &= wdone[i];
          if (all) {
            __builtin_amdgcn_s_waitcnt(0);
            stop = true;
            break;
          }
        }
      }
      q = nq;
      c = nc;
      T = nT;
      if (g + 1 < total) advance_next();
    }
  }
  if (valid && grp == 0) {
    // sample and the parity of the new bond index of the outcome
    // stored here; an undecided shot hands its running sum to the next launch
    if (wrote) {
      out[(shot0 + shot) * (int64_t)M + (site - 1)] = psel;
      if (par_out) par_out[shot] = (int8_t)((pi + psel) & 1);
    }
    const bool fin = done || qlast >= npass;
    if (key) key[shot] = shot_key(fin, pi, ur, csum);
    if (!fin) cum[shot] = csum;
  }
}

// Passes [qbeg, qend) for blocks of 16 W slots; the workgroups of the grid
// loop over the blocks that hold shots (with a partition, the counts come
// from cnt), so the grid need not match the shot count.
template <int NT, int W>
__global__ __launch_bounds__(64 * W) void sample_mfma_kernel(
    const float* __restrict__ P, const SamplerGeom* __restrict__ geo, const float* __restrict__ lin,
    float* __restrict__ lout, long ldl2, const int32_t* __restrict__ perm, const int32_t* __restrict__ cnt,
    int8_t* __restrict__ par_out, float* __restrict__ cum, int8_t* __restrict__ key, int qbeg, int qend,
    int64_t shot0, int64_t nshots, int site, uint32_t k0, uint32_t k1, int32_t* __restrict__ out, int M) {
  __shared__ __attribute__((aligned(16))) float Bs0[512 * NT];
  __shared__ __attribute__((aligned(16))) float Bs1[512 * NT];
  __shared__ int wdone[W];
  constexpr int kS = 16 * W;
  int64_t nblk = (nshots + kS - 1) / kS;
  if (perm) {
    const int64_t c0 = cnt[0], c1 = cnt[1];
    const int64_t e = (c0 + kShotsPerWg - 1) / kShotsPerWg * kShotsPerWg;
    nblk = e / kS + (c1 + kS - 1) / kS;
  }
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x)
    sample_passes<NT, W>(Bs0, Bs1, wdone, blk, P, geo, lin, lout, ldl2, perm, cnt, par_out, cum, key, qbeg, qend,
                         shot0, nshots, site, k0, k1, out, M);
}

// Batched sweep: one site step of several sampling requests in one launch.
// Workgroup (x, y) takes slot block x of request y at that request's own
// current site (requests join and leave the batch at any step), all passes
// of the site with early stopping.  The arithmetic of every shot is that of
// the single-request sweep.
template <int NT>
__global__ __launch_bounds__(64 * kWaves) void sample_batch_kernel(const SampleBatchDesc* __restrict__ desc) {
  __shared__ __attribute__((aligned(16))) float Bs0[512 * NT];
  __shared__ __attribute__((aligned(16))) float Bs1[512 * NT];
  __shared__ int wdone[kWaves];
  const SampleBatchDesc& D = desc[blockIdx.y];
  const int m = D.site;
  const bool part = D.psplit && m > 1, next = D.psplit && m < D.M;
  const int64_t blocks = (D.nshots + kShotsPerWg - 1) / kShotsPerWg + (part ? 1 : 0);
  if ((int64_t)blockIdx.x >= blocks) return;  // whole workgroup
  const int cur = (m - 1) & 1;
  sample_passes<NT, kWaves>(Bs0, Bs1, wdone, blockIdx.x, D.packed + D.poff[m], D.geo + m, D.fb[cur], D.fb[1 - cur],
                    D.ldl2, part ? D.perm : nullptr, part ? D.cnt : nullptr, next ? D.par : nullptr, nullptr, nullptr,
                    0, kSamplerMaxOutcomes, 0, D.nshots, m, D.k0, D.k1, D.out, D.M);
}

// The first pass of a site (outcome 0, plus any outcomes sharing its pass)
// for every shot, as a persistent launch: each workgroup loops over blocks
// of 128 slots (sector-0 blocks, then sector-1 blocks from slot E) with a
// stride of the grid size, and the chunk sequence runs on across blocks, so
// the next block's first B' chunk and A rows are fetched during the current
// block's last chunk and its row stores drain under the next block's MFMAs.
template <int NT>
__global__ __launch_bounds__(64 * kWaves) void sample_first_kernel(
    const float* __restrict__ P, const SamplerGeom* __restrict__ geo, const float* __restrict__ lin,
    float* __restrict__ lout, long ldl2, const int32_t* __restrict__ perm, const int32_t* __restrict__ cnt,
    int8_t* __restrict__ par_out, float* __restrict__ cum, int8_t* __restrict__ key, int64_t shot0, int64_t nshots,
    int site, uint32_t k0, uint32_t k1, int32_t* __restrict__ out, int M) {
  __shared__ __attribute__((aligned(16))) float Bs0[512 * NT];
  __shared__ __attribute__((aligned(16))) float Bs1[512 * NT];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, scalar
  const int grp = lane >> 4, col = lane & 15;
  int64_t c0 = nshots, c1 = 0;
  if (perm) {
    c0 = cnt[0];
    c1 = cnt[1];
  }
  const int64_t nb0 = (c0 + kShotsPerWg - 1) / kShotsPerWg;
  const int64_t nblk = nb0 + (c1 + kShotsPerWg - 1) / kShotsPerWg;
  const int64_t e = nb0 * kShotsPerWg;
  const int64_t stride = gridDim.x;
  // one block as seen by this lane
  struct Blk {
    int pi, nchunk, T;
    bool halfk, valid;
    long base;
    int64_t shot;
  };
  auto setup = [&](int64_t bb) {
    Blk s;
    const bool one = bb >= nb0;
    s.pi = one ? 1 : 0;
    const int64_t slot = (one ? e + (bb - nb0) * kShotsPerWg : bb * kShotsPerWg) + w * 16 + col;
    s.valid = slot < (one ? e + c1 : c0);
    s.shot = s.valid ? (perm ? (int64_t)perm[slot] : slot) : 0;
    s.nchunk = geo->nchunk[s.pi];
    s.halfk = geo->half[s.pi] != 0;
    s.T = geo->tiles[s.pi][0];
    s.base = geo->base[s.pi][0];
    return s;
  };
  // the first block at or after bb whose sector has rows; the shots of a
  // block in an empty sector get outcome 0 with weight zero (a shot cannot
  // reach an empty sector with positive probability)
  auto next_block = [&](int64_t bb) {
    for (; bb < nblk; bb += stride) {
      const int pb = bb >= nb0 ? 1 : 0;
      if (geo->npass[pb] > 0) break;
      const Blk s = setup(bb);
      if (s.valid && grp == 0) {
        out[(shot0 + s.shot) * (int64_t)M + (site - 1)] = 0;
        if (par_out) par_out[s.shot] = (int8_t)pb;
        if (key) key[s.shot] = kKeyDone;
      }
    }
    return bb;
  };
  auto load_a = [&](const Blk& s, int c, float4* r) {
    const float* row = lin + s.shot * ldl2 + 4 * grp + 32 * c;
    r[0] = *(const float4*)(row);       // k-half 0: rows 32c + 4 grp + (0..3)
    r[1] = *(const float4*)(row + 16);  // k-half 1: 16 rows further
  };
  auto take_a = [&](const float4* r, float* a) {
    a[0] = r[0].x; a[1] = r[0].y; a[2] = r[0].z; a[3] = r[0].w;
    a[4] = r[1].x; a[5] = r[1].y; a[6] = r[1].z; a[7] = r[1].w;
  };
  auto issue = [&](const Blk& s, int c, float* dst) {
    const float* src = P + s.base + 512L * s.T * c;
    if (s.halfk && c == s.nchunk - 1) {  // blocks (t, h = 0) of a half chunk
      for (int blk = w; blk < s.T; blk += kWaves)
        __builtin_amdgcn_global_load_lds((const void*)(src + blk * 256 + lane * 4),
                                         (void __attribute__((address_space(3)))*)(dst + 2 * blk * 256), 16, 0, 0);
    } else {
      for (int blk = w; blk < 2 * s.T; blk += kWaves)
        __builtin_amdgcn_global_load_lds((const void*)(src + blk * 256 + lane * 4),
                                         (void __attribute__((address_space(3)))*)(dst + blk * 256), 16, 0, 0);
    }
  };
  int64_t b = next_block((int64_t)blockIdx.x);
  if (b >= nblk) return;  // uniform over the workgroup
  Blk cur = setup(b);
  int64_t bn = next_block(b + stride);
  bool has_next = bn < nblk;
  Blk nxt = has_next ? setup(bn) : cur;
  floatx4 acc[NT];
  float a[8];
  float4 an[2];
  issue(cur, 0, Bs0);
  load_a(cur, 0, an);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  take_a(an, a);
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  int c = 0;  // chunk of the current block in the buffer being multiplied
  bool last = false;
  while (!last) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      // fetch the chunk that follows: the current block's next one, or the
      // next block's first
      const bool fnext = c + 1 >= cur.nchunk;
      const bool fetch = !fnext || has_next;
      if (fetch) {
        if (fnext) {
          issue(nxt, 0, u ? Bs0 : Bs1);
          load_a(nxt, 0, an);
        } else {
          issue(cur, c + 1, u ? Bs0 : Bs1);
          load_a(cur, c + 1, an);
        }
      }
      chunk_mfma<NT>(acc, (const float4*)(u ? Bs1 : Bs0), a, cur.T, cur.halfk && c == cur.nchunk - 1, lane);
      // every wave's share of the fetched chunk (and its A rows) has landed,
      // and its LDS reads of this chunk are done, before any wave goes on
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_s_barrier();
      if (fetch) take_a(an, a);
      if (!fnext) {
        ++c;
        continue;
      }
      // last chunk of the block: draw and store
      float ur;
      {
        const int64_t gs = shot0 + cur.shot;
        philox4 ctr;
        ctr.v[0] = (uint32_t)gs;
        ctr.v[1] = (uint32_t)((uint64_t)gs >> 32);
        ctr.v[2] = (uint32_t)site;
        ctr.v[3] = 0u;
        ur = u01_24(philox4x32_10(ctr, k0, k1).v[0]);
      }
      float csum = 0.f, wsel = 0.f;
      bool done = false, wrote = false;
      int psel = 0;
      pass_draws<NT>(acc, geo->j0[cur.pi][0], geo->j0[cur.pi][1], geo->nt[cur.pi], geo->nt[cur.pi ^ 1], ur, csum,
                     done, wrote, psel, wsel, cur.valid, lout + cur.shot * ldl2 + 4 * grp);
      if (cur.valid && grp == 0) {
        // outcome 0 is in the first pass, so every shot has a row stored
        out[(shot0 + cur.shot) * (int64_t)M + (site - 1)] = psel;
        if (par_out) par_out[cur.shot] = (int8_t)((cur.pi + psel) & 1);
        const bool fin = done || geo->npass[cur.pi] <= 1;
        if (key) key[cur.shot] = shot_key(fin, cur.pi, ur, csum);
        if (!fin) cum[cur.shot] = csum;
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      if (!has_next) {
        last = true;
        break;
      }
      cur = nxt;
      c = 0;
      bn = next_block(bn + stride);
      has_next = bn < nblk;
      if (has_next) nxt = setup(bn);
    }
  }
}
#undef GBS_MF

constexpr int kPartElems = 1024;  // parities per partition block (256 threads x 4)

// N sums over the 256 threads of a block at once (every thread gets all N):
// one exchange through LDS (sh: 4 N ints) instead of one per value.
template <int N>
__device__ inline void block_sums256(int (&v)[N], int* sh) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) sh[(threadIdx.x >> 6) * N + i] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = sh[i] + sh[N + i] + sh[2 * N + i] + sh[3 * N + i];
}

// Classes k = sector * B + bucket, B buckets per sector; any other value is
// left out.  part_count: per block of kPartElems shots, the count of each
// class; part_scatter: the stable counting sort by class, sector 0's classes
// from slot 0 and sector 1's from slot E (sector 0's total rounded up to a
// whole workgroup), so a workgroup never mixes sectors.
template <int B>
__device__ __forceinline__ void part_count(const int8_t* __restrict__ par, int64_t n, int32_t* __restrict__ bcnt,
                                           int64_t blk, int* sh) {
  constexpr int K = 2 * B;
  const int64_t base = blk * kPartElems + 4 * threadIdx.x;
  int c[K];
#pragma unroll
  for (int k = 0; k < K; ++k) c[k] = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int v = base + j < n ? (int)par[base + j] : -1;
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] += v == k;
  }
  block_sums256<K>(c, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) bcnt[K * blk + k] = c[k];
}

template <int B>
__device__ __forceinline__ void part_scatter(const int8_t* __restrict__ par, int64_t n,
                                             const int32_t* __restrict__ bcnt, int nblk, int32_t* __restrict__ perm,
                                             int32_t* __restrict__ cnt, int blk, int* sh, int* wtot) {
  constexpr int K = 2 * B, KP = (K + 1) / 2;  // classes, 16-bit pairs of them
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int before[K], tot[K];
#pragma unroll
  for (int k = 0; k < K; ++k) before[k] = tot[k] = 0;
  for (int i = tid; i < nblk; i += 256) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int v = bcnt[K * i + k];
      tot[k] += v;
      if (i < blk) before[k] += v;
    }
  }
  block_sums256<K>(before, sh);
  block_sums256<K>(tot, sh);
  int64_t c0 = 0, c1 = 0;
#pragma unroll
  for (int k = 0; k < B; ++k) {
    c0 += tot[k];
    c1 += tot[B + k];
  }
  const int64_t e = (c0 + kShotsPerWg - 1) / kShotsPerWg * kShotsPerWg;
  // first slot of each class for this block's shots
  int64_t start[K];
  {
    int64_t run0 = 0, run1 = e;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      start[k] = run0 + before[k];
      run0 += tot[k];
      start[B + k] = run1 + before[B + k];
      run1 += tot[B + k];
    }
  }
  const int64_t base = (int64_t)blk * kPartElems + 4 * tid;
  int q[4];
  int pk[KP];  // this thread's class counts, two per int in 16-bit halves
#pragma unroll
  for (int i = 0; i < KP; ++i) pk[i] = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    q[j] = base + j < n ? (int)par[base + j] : -1;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (q[j] == k) pk[k >> 1] += 1 << (16 * (k & 1));
  }
  // exclusive scan over the block of the packed counts (at most 1024 per
  // class, so the halves never carry into each other)
  int ex[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    int x = pk[i];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    int wpre = 0;
    for (int v = 0; v < w; ++v) wpre += wtot[v];
    ex[i] = x - pk[i] + wpre;
  }
  int64_t pos[K];
#pragma unroll
  for (int k = 0; k < K; ++k) pos[k] = start[k] + ((ex[k >> 1] >> (16 * (k & 1))) & 0xffff);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (q[j] == k) perm[pos[k]++] = (int32_t)(base + j);
  }
  if (blk == 0 && tid == 0) {
    cnt[0] = (int32_t)c0;
    cnt[1] = (int32_t)c1;
  }
}

template <int B>
__global__ __launch_bounds__(256) void part_count_kernel(const int8_t* __restrict__ par, int64_t n,
                                                         int32_t* __restrict__ bcnt) {
  __shared__ int sh[8 * B];
  part_count<B>(par, n, bcnt, blockIdx.x, sh);
}

template <int B>
__global__ __launch_bounds__(256) void part_scatter_kernel(const int8_t* __restrict__ par, int64_t n,
                                                           const int32_t* __restrict__ bcnt, int nblk,
                                                           int32_t* __restrict__ perm, int32_t* __restrict__ cnt) {
  __shared__ int sh[8 * B];
  __shared__ int wtot[4];
  part_scatter<B>(par, n, bcnt, nblk, perm, cnt, blockIdx.x, sh, wtot);
}

// Partition by the parities of request y's outcomes at its current site,
// for the next site (requests at their last site, or without sectors, skip).
__global__ __launch_bounds__(256) void part_count_batch_kernel(const SampleBatchDesc* __restrict__ desc) {
  __shared__ int sh[8];  // 4 x (2 classes)
  const SampleBatchDesc& D = desc[blockIdx.y];
  const int64_t nblk = (D.nshots + kPartElems - 1) / kPartElems;
  if (!D.psplit || D.site >= D.M || (int64_t)blockIdx.x >= nblk) return;
  part_count<1>(D.par, D.nshots, D.bcnt, blockIdx.x, sh);
}

__global__ __launch_bounds__(256) void part_scatter_batch_kernel(const SampleBatchDesc* __restrict__ desc) {
  __shared__ int sh[8];  // 4 x (2 classes)
  __shared__ int wtot[4];
  const SampleBatchDesc& D = desc[blockIdx.y];
  const int64_t nblk = (D.nshots + kPartElems - 1) / kPartElems;
  if (!D.psplit || D.site >= D.M || (int64_t)blockIdx.x >= nblk) return;
  part_scatter<1>(D.par, D.nshots, D.bcnt, (int)nblk, D.perm, D.cnt, blockIdx.x, sh, wtot);
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

long sampler_geometry(const SamplerSite& s, int d, SamplerGeom* g) {
  if (d < 1 || d > kSamplerMaxOutcomes) return -1;
  SamplerGeom G{};
  for (int i = 0; i < 2; ++i) {
    if (sampler_pad(s.nL[i]) > kSamplerMaxSector || sampler_pad(s.nR[i]) > kSamplerMaxSector) return -1;
    const int nkh = (s.nL[i] + 7) / 8;  // K in halves of 16 real rows (8 complex)
    G.nchunk[i] = (nkh + 1) / 2;
    G.half[i] = nkh & 1;
    G.nt[i] = sampler_pad(s.nR[i]) / 8;
  }
  // accumulator tiles: the widest single outcome, raised towards the budget
  // so that narrow outcomes share passes
  int widest = 2, sum_max = 0;
  for (int pi = 0; pi < 2; ++pi) {
    if (s.nL[pi] <= 0) continue;
    int sum = 0;
    for (int p = 0; p < d; ++p) {
      const int t = G.nt[pi ^ (p & 1)];
      widest = std::max(widest, t);
      sum += t;
    }
    sum_max = std::max(sum_max, sum);
  }
  G.NT = std::max(widest, std::min(kSamplerMaxTiles, sum_max));
  G.NT = (G.NT + 7) / 8 * 8;  // kernel instances: 8, 16, 24, 32 tiles
  long tot = 0;
  for (int pi = 0; pi < 2; ++pi) {
    G.npass[pi] = 0;
    G.j0[pi][0] = 0;
    if (s.nL[pi] <= 0) continue;
    int j = 0;
    while (j < d) {
      const int q = G.npass[pi]++;
      int T = 0;
      while (j < d) {
        const int t = G.nt[pi ^ (j & 1)];
        if (T > 0 && T + t > G.NT) break;
        T += t;
        ++j;
        if (j == 1 && T > 0) break;  // outcome 0 alone: the first launch decides most shots with it
      }
      G.tiles[pi][q] = T;
      G.base[pi][q] = tot;
      G.j0[pi][q + 1] = j;
      tot += (512L * (G.nchunk[pi] - G.half[pi]) + 256L * G.half[pi]) * T;
    }
  }
  if (g) *g = G;
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
                       const SamplerGeom& g, const SamplerGeom* gd, const int32_t* mapL, const int32_t* mapR,
                       float* P) {
  if (s.nL[0] + s.nL[1] > K || (mapR && s.nR[0] + s.nR[1] > N) || (!mapR && (s.nR[0] > N || s.nR[1] > N)))
    return hipErrorInvalidValue;
  long mx = 0;
  for (int pi = 0; pi < 2; ++pi)
    for (int q = 0; q < g.npass[pi]; ++q) mx = std::max(mx, 128L * g.nchunk[pi] * g.tiles[pi][q]);  // bound
  if (mx == 0) return hipSuccess;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((mx + 255) / 256), (unsigned)(2 * kSamplerMaxOutcomes)), dim3(256),
                     0, st, B, d, N, s, gd, mapL, mapR, P);
  return hipGetLastError();
}

hipError_t launch_pack_batch(hipStream_t st, const SamplerPackDesc* host, const SamplerPackDesc* dev, int n,
                             const SamplerGeom* geo_host) {
  long mx = 0;
  for (int i = 0; i < n; ++i) {
    const SamplerPackDesc& q = host[i];
    const SamplerGeom& g = geo_host[i];
    if (q.s.nL[0] + q.s.nL[1] > q.K || (q.mapR && q.s.nR[0] + q.s.nR[1] > q.N) ||
        (!q.mapR && (q.s.nR[0] > q.N || q.s.nR[1] > q.N)))
      return hipErrorInvalidValue;
    for (int pi = 0; pi < 2; ++pi)
      for (int p = 0; p < g.npass[pi]; ++p) mx = std::max(mx, 128L * g.nchunk[pi] * g.tiles[pi][p]);  // bound
  }
  if (mx == 0 || n <= 0) return hipSuccess;
  if (n > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pack_batch_kernel, dim3((unsigned)((mx + 255) / 256), (unsigned)(2 * kSamplerMaxOutcomes),
                                             (unsigned)n),
                     dim3(256), 0, st, dev);
  return hipGetLastError();
}

// Workgroups of a persistent launch: as many as the device runs at once
// (resident workgroups per CU times the CU count), counted once per kernel.
static int64_t persistent_grid(const void* kernel, int threads = 64 * kWaves) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int64_t> known;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  std::lock_guard<std::mutex> lk(mu);
  auto it = known.find({dev, kernel});
  if (it != known.end()) return it->second;
  int ncu = 0, per = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1) per = 1;
  const int64_t g = (int64_t)ncu * per;
  known[{dev, kernel}] = g;
  return g;
}

hipError_t launch_sample_mfma(hipStream_t st, const float* P, const SamplerGeom& g, const SamplerGeom* gd,
                              const float* lin, float* lout, long ldl2,
                              const int32_t* perm, const int32_t* cnt, int8_t* par_out, float* cum, int8_t* key,
                              int qbeg, int qend, int64_t shot0, int64_t nshots, int site, uint64_t seed, int32_t* out,
                              int M) {
  if (nshots <= 0) return hipSuccess;
  if ((perm == nullptr) != (cnt == nullptr)) return hipErrorInvalidValue;
  if (!perm && g.npass[1] != 0) return hipErrorInvalidValue;
  if (qbeg < 0 || qend <= qbeg) return hipErrorInvalidValue;
  // a launch that leaves shots undecided hands them on through cum and key;
  // a later launch reads cum and gets its shots from a partition of key
  const bool leaves = qend < g.npass[0] || qend < g.npass[1];
  if ((leaves && (!cum || !key)) || (qbeg > 0 && (!cum || !perm))) return hipErrorInvalidValue;
  for (int i = 0; i < 2; ++i)
    if (32L * g.nchunk[i] > ldl2 || 16L * g.nt[i] > ldl2) return hipErrorInvalidValue;
  // accumulator tiles of the kernel instance: the widest pass of the range
  int mx = 8;
  for (int pi = 0; pi < 2; ++pi)
    for (int q = 0; q < g.npass[pi]; ++q) {
      if (g.tiles[pi][q] > g.NT) return hipErrorInvalidValue;
      if (q >= qbeg && q < qend) mx = std::max(mx, g.tiles[pi][q]);
    }
  const int nt = (mx + 7) / 8 * 8;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  // with a partition, sector 1 starts on a fresh workgroup: one more block
  dim3 grid((unsigned)((nshots + kShotsPerWg - 1) / kShotsPerWg + (perm ? 1 : 0)));
#define GBS_SAMPLE_CASE(NTV)                                                                                      \
  case NTV:                                                                                                       \
    if (qbeg == 0 && qend == 1) {                                                                                 \
      const dim3 pg((unsigned)std::min<int64_t>(grid.x, persistent_grid((const void*)sample_first_kernel<NTV>))); \
      hipLaunchKernelGGL((sample_first_kernel<NTV>), pg, dim3(64 * kWaves), 0, st, P, gd, lin, lout, ldl2, perm,   \
                         cnt, par_out, cum, key, shot0, nshots, site, k0, k1, out, M);                            \
    } else {                                                                                                      \
      const void* kf = (const void*)sample_mfma_kernel<NTV, kRestWaves>;                                          \
      const int64_t nb = (nshots + 16 * kRestWaves - 1) / (16 * kRestWaves) + (perm ? kWaves / kRestWaves : 0);   \
      const dim3 rg((unsigned)std::min<int64_t>(nb, kRestGridMult * persistent_grid(kf, 64 * kRestWaves)));       \
      hipLaunchKernelGGL((sample_mfma_kernel<NTV, kRestWaves>), rg, dim3(64 * kRestWaves), 0, st, P, gd, lin,     \
                         lout, ldl2, perm, cnt, par_out, cum, key, qbeg, qend, shot0, nshots, site, k0, k1, out, M); \
    }                                                                                                             \
    break;
  switch (nt) {
    GBS_SAMPLE_CASE(8)
    GBS_SAMPLE_CASE(16)
    GBS_SAMPLE_CASE(24)
    GBS_SAMPLE_CASE(32)
    default:
      return hipErrorInvalidValue;
  }
#undef GBS_SAMPLE_CASE
  return hipGetLastError();
}

int64_t sampler_partition_ws(int64_t nshots) {
  return 2 * kKeyBuckets * ((nshots + kPartElems - 1) / kPartElems);
}

hipError_t launch_sampler_partition(hipStream_t st, const int8_t* par, int64_t nshots, int32_t* bcnt,
                                    int32_t* perm, int32_t* cnt, bool buckets) {
  if (nshots <= 0) return hipSuccess;
  if (nshots > INT32_MAX - 256) return hipErrorInvalidValue;
  const int nblk = (int)((nshots + kPartElems - 1) / kPartElems);
  if (buckets) {
    hipLaunchKernelGGL(part_count_kernel<kKeyBuckets>, dim3((unsigned)nblk), dim3(256), 0, st, par, nshots, bcnt);
    hipLaunchKernelGGL(part_scatter_kernel<kKeyBuckets>, dim3((unsigned)nblk), dim3(256), 0, st, par, nshots, bcnt,
                       nblk, perm, cnt);
  } else {
    hipLaunchKernelGGL(part_count_kernel<1>, dim3((unsigned)nblk), dim3(256), 0, st, par, nshots, bcnt);
    hipLaunchKernelGGL(part_scatter_kernel<1>, dim3((unsigned)nblk), dim3(256), 0, st, par, nshots, bcnt, nblk,
                       perm, cnt);
  }
  return hipGetLastError();
}

int sampler_batch_nt(const SamplerGeom& g) {
  int mx = 8;
  for (int pi = 0; pi < 2; ++pi)
    for (int q = 0; q < g.npass[pi]; ++q) mx = std::max(mx, g.tiles[pi][q]);
  return (mx + 7) / 8 * 8;
}

hipError_t launch_sample_batch(hipStream_t st, const SampleBatchDesc* desc, int nreq, int64_t max_blocks, int nt) {
  if (nreq <= 0 || max_blocks <= 0) return hipSuccess;
  if (nreq > 65535 || max_blocks > INT32_MAX) return hipErrorInvalidValue;
  const dim3 grid((unsigned)max_blocks, (unsigned)nreq);
  switch (nt) {
    case 8: hipLaunchKernelGGL((sample_batch_kernel<8>), grid, dim3(64 * kWaves), 0, st, desc); break;
    case 16: hipLaunchKernelGGL((sample_batch_kernel<16>), grid, dim3(64 * kWaves), 0, st, desc); break;
    case 24: hipLaunchKernelGGL((sample_batch_kernel<24>), grid, dim3(64 * kWaves), 0, st, desc); break;
    case 32: hipLaunchKernelGGL((sample_batch_kernel<32>), grid, dim3(64 * kWaves), 0, st, desc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_partition_batch(hipStream_t st, const SampleBatchDesc* desc, int nreq, int64_t max_shots) {
  if (nreq <= 0 || max_shots <= 0) return hipSuccess;
  if (nreq > 65535 || max_shots > INT32_MAX - 256) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((max_shots + kPartElems - 1) / kPartElems), (unsigned)nreq);
  hipLaunchKernelGGL(part_count_batch_kernel, grid, dim3(256), 0, st, desc);
  hipLaunchKernelGGL(part_scatter_batch_kernel, grid, dim3(256), 0, st, desc);
  return hipGetLastError();
}
