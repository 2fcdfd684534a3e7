// Projected-creation-operator mapping on the GPU (Sec. II.C.2, App. B).
//
// All PCOs commute and the kept subspace V is closed under creation
// operators (Eq. pass_projector), so the product of every PCO applied to the
// vacuum equals P exp(X)|0> = sum_k (P X P)^k |0> / k!  with
// X = sum_{z <= z'} (1 - delta/2) Q_{zz'} d_z^dag d_z'^dag.  The term with k
// pair creations lives on the kept states with 2k photons, so
//   A[n] = (1/k) sum_{z <= z'} (1 - delta/2) Q_{zz'} sqrt(n_z (n_z' - delta)) A[n - e_z - e_z']
// for every element n = (alpha, p, beta) with |alpha| + p + |beta| = 2k.
// Elements of one level are independent: one launch per level covers every
// site at once (sites are independent once Q^m and the kept bases are known).
// Source indices come from the lowering maps (first-order vector sets and
// their composition).  Accumulation is in FP64.
#include "gbs_pco.h"

__global__ __launch_bounds__(256) void pco_level_kernel(PcoArgs a, const LevelBlock* __restrict__ blocks, int nblocks,
                                                        long nelem, int k) {
  const long gid0 = blockIdx.x * (long)blockDim.x + threadIdx.x;
  // threads past the last element take element nelem - 1's path without
  // storing, so that every lane of a wave reaches the term count at the end
  const bool live = gid0 < nelem;
  const long gid = live ? gid0 : nelem - 1;
  // locate the block (elem_start ascending)
  int lo = 0, hi = nblocks - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (blocks[mid].elem_start <= gid) lo = mid;
    else hi = mid - 1;
  }
  const LevelBlock bk = blocks[lo];
  const long loc = gid - bk.elem_start;
  const int i = (int)(loc / bk.b_cnt), j = (int)(loc % bk.b_cnt);
  const SiteDesc sd = a.sites[bk.site];
  const int p = bk.p;
  const int alpha = a.perm[sd.off_state_l + bk.a_off + i];
  const int beta = a.perm[sd.off_state_r + bk.b_off + j];
  const int nl = sd.nl, nr = sd.nr, d = sd.d, chiR = sd.chiR, chiL = sd.chiL;
  const cplx64* Q = a.Q + sd.off_q;
  const long ldq = a.ld_q;
  cplx64* T = a.T + sd.off_t;
  const int ia = nl;
  // occupied-mode lists
  const int4* la = a.olist + (sd.off_state_l + alpha) * GBS_K_MAX;
  const int4* lb = a.olist + (sd.off_state_r + beta) * GBS_K_MAX;
  const int sa = a.nocc[sd.off_state_l + alpha] < GBS_K_MAX ? a.nocc[sd.off_state_l + alpha] : GBS_K_MAX;
  const int sb = a.nocc[sd.off_state_r + beta] < GBS_K_MAX ? a.nocc[sd.off_state_r + beta] : GBS_K_MAX;
  const int* lowL = a.low + sd.off_occ_l;  // [q * chiL + state]
  const int* lowR = a.low + sd.off_occ_r;  // [q * chiR + state]
#define TIDX(al, pp, be) (((long)(al) * d + (pp)) * chiR + (be))
  double ar = 0.0, ai = 0.0;
  int nterm = 0;
  auto acc = [&](cplx64 g, double c, long idx) {
    ++nterm;
    cplx64 v = T[idx];
    ar += c * (g.re * v.re - g.im * v.im);
    ai += c * (g.re * v.im + g.im * v.re);
  };
  // incoming-virtual pairs (q <= q')
  for (int u = 0; u < sa; ++u) {
    const int4 ou = la[u];
    if (ou.y >= 2) {
      int src = lowL[(long)ou.x * chiL + ou.z];
      cplx64 g = Q[(long)ou.x * ldq + ou.x];
      acc(g, 0.5 * sqrt((double)ou.y * (ou.y - 1)), TIDX(src, p, beta));
    }
    for (int v = u + 1; v < sa; ++v) {
      const int4 ov = la[v];
      int src = lowL[(long)ov.x * chiL + ou.z];
      cplx64 g = Q[(long)ou.x * ldq + ov.x];
      acc(g, sqrt((double)ou.y * ov.y), TIDX(src, p, beta));
    }
    if (p >= 1) {  // incoming - physical
      cplx64 g = Q[(long)ou.x * ldq + ia];
      acc(g, sqrt((double)ou.y * p), TIDX(ou.z, p - 1, beta));
    }
    for (int v = 0; v < sb; ++v) {  // incoming - outgoing (cross)
      const int4 ov = lb[v];
      cplx64 g = Q[(long)ou.x * ldq + nl + 1 + ov.x];
      acc(g, sqrt((double)ou.y * ov.y), TIDX(ou.z, p, ov.z));
    }
  }
  if (p >= 2) {  // physical duplicate
    cplx64 g = Q[(long)ia * ldq + ia];
    acc(g, 0.5 * sqrt((double)p * (p - 1)), TIDX(alpha, p - 2, beta));
  }
  for (int v = 0; v < sb; ++v) {
    const int4 ov = lb[v];
    if (p >= 1) {  // physical - outgoing
      cplx64 g = Q[(long)ia * ldq + nl + 1 + ov.x];
      acc(g, sqrt((double)p * ov.y), TIDX(alpha, p - 1, ov.z));
    }
    if (ov.y >= 2) {
      int src = lowR[(long)ov.x * chiR + ov.z];
      cplx64 g = Q[(long)(nl + 1 + ov.x) * ldq + nl + 1 + ov.x];
      acc(g, 0.5 * sqrt((double)ov.y * (ov.y - 1)), TIDX(alpha, p, src));
    }
    for (int w = v + 1; w < sb; ++w) {
      const int4 ow = lb[w];
      int src = lowR[(long)ow.x * chiR + ov.z];
      cplx64 g = Q[(long)(nl + 1 + ov.x) * ldq + nl + 1 + ow.x];
      acc(g, sqrt((double)ov.y * ow.y), TIDX(alpha, p, src));
    }
  }
#undef TIDX
  (void)nr;
  const double inv = 1.0 / (double)k;
  if (live) T[((long)alpha * d + p) * chiR + beta] = cmake<cplx64>(ar * inv, ai * inv);
  if (a.terms) {  // source terms of this wave's elements, one atomic per wave
    unsigned long long c = live ? (unsigned long long)nterm : 0ull;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(a.terms, c);
  }
}

__global__ void pco_init_kernel(PcoArgs a, int nsites) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsites) return;
  a.T[a.sites[s].off_t] = cmake<cplx64>(1.0, 0.0);
}

hipError_t launch_pco_init(hipStream_t st, const PcoArgs& a, int nsites) {
  hipLaunchKernelGGL(pco_init_kernel, dim3((nsites + 255) / 256), dim3(256), 0, st, a, nsites);
  return hipGetLastError();
}

hipError_t launch_pco_level(hipStream_t st, const PcoArgs& a, const LevelBlock* blocks, int nblocks, long nelem,
                            int k) {
  if (nelem <= 0) return hipSuccess;
  long grid = (nelem + 255) / 256;
  hipLaunchKernelGGL(pco_level_kernel, dim3((unsigned)grid), dim3(256), 0, st, a, blocks, nblocks, nelem, k);
  return hipGetLastError();
}
