// Kept virtual bases and index maps (Sec. II.C.1, App. B).
//
// Per cut, the D lowest-entanglement-energy Fock states over the active
// virtual modes (E = -sum_q 2 n_q log Lambda_q, Lambda descending) are
// enumerated best-first.  Every state is reached once through a canonical
// parent (the state minus one photon of its highest occupied mode); a heap
// ordered by (E, occupation tuple descending lexicographically) holds at most
// one child and one sibling per popped state.  That tie-break is the one
// consistent with the parent/sibling order, so states come out in key order.
//
// Index maps: an additive 64-bit hash H(n) = sum_q n_q R_q (R_q from
// splitmix64) gives H(n - e_q) = H(n) - R_q, looked up by binary search over
// the sorted hashes and verified against the occupation table.  The dense
// lowering table low[q][beta] = index(beta - e_q) is the first-order content
// of the vector sets of Algorithm 1; pair lowerings are its composition
// (Algorithm 3).
#include "gbs_kept.h"

namespace {

struct HeapNode {
  double E;
  int parent;
  int q;
};

// Compare two candidates (parent + e_q): true if a comes before b.
__device__ bool node_before(const HeapNode& a, const HeapNode& b, const short* occ, int ne) {
  if (a.E != b.E) return a.E < b.E;
  // tie: occupation tuple in descending lexicographic order comes first
  const short* ra = occ + (long)a.parent * ne;
  const short* rb = occ + (long)b.parent * ne;
  for (int j = 0; j < ne; ++j) {
    int na = ra[j] + (j == a.q), nb = rb[j] + (j == b.q);
    if (na != nb) return na > nb;
  }
  return false;
}

__device__ void heap_push(HeapNode* h, int& n, HeapNode x, const short* occ, int ne) {
  int i = n++;
  while (i > 0) {
    int p = (i - 1) >> 1;
    if (!node_before(x, h[p], occ, ne)) break;
    h[i] = h[p];
    i = p;
  }
  h[i] = x;
}

__device__ HeapNode heap_pop(HeapNode* h, int& n, const short* occ, int ne) {
  HeapNode top = h[0];
  HeapNode x = h[--n];
  int i = 0;
  while (true) {
    int l = 2 * i + 1, r = l + 1, s = i;
    HeapNode best = x;
    if (l < n && node_before(h[l], best, occ, ne)) { s = l; best = h[l]; }
    if (r < n && node_before(h[r], best, occ, ne)) { s = r; best = h[r]; }
    if (s == i) break;
    h[i] = h[s];
    i = s;
  }
  if (n > 0) h[i] = x;
  return top;
}

}  // namespace

__global__ __launch_bounds__(256) void kept_kernel(KeptArgs a) {
  const int m = blockIdx.x;  // cuts 0..M (0 and M hold the vacuum)
  const CutDesc cd = a.cuts[m];
  const int ne = cd.ne, chi = cd.chi;
  const int tid = threadIdx.x, nt = blockDim.x;
  extern __shared__ char smem[];
  // heap and sort buffer: LDS, or this cut's slice of a global workspace
  // when they do not fit (large chi)
  char* wbase = a.gws ? a.gws + (long)m * a.gws_stride : smem;
  double* E = a.E + cd.off_state;
  int* parent = a.parent + cd.off_state;
  int* pmode = a.pmode + cd.off_state;
  int* ntot = a.ntot + cd.off_state;
  unsigned long long* H = a.hash + cd.off_state;
  short* occ = a.occ + cd.off_occ;
  int* low = a.low + cd.off_occ;
  int* nocc = a.nocc + cd.off_state;
  int4* olist = a.olist + cd.off_state * GBS_K_MAX;
  const double* lam = a.lam + (long)m * a.ld_lam;

  // zero the occupation table of this cut
  for (long e = tid; e < (long)chi * ne; e += nt) occ[e] = 0;
  __syncthreads();
  if (ne == 0) {
    if (tid == 0) {
      E[0] = 0.0; parent[0] = -1; pmode[0] = -1; ntot[0] = 0; H[0] = 0ull; nocc[0] = 0;
    }
    return;
  }
  // ---- best-first enumeration (thread 0)
  HeapNode* heap = (HeapNode*)wbase;
  if (tid == 0) {
    int hn = 0;
    E[0] = 0.0; parent[0] = -1; pmode[0] = -1; ntot[0] = 0;
    // mode energies e_q = -2 log Lambda_q (Lambda descending => e ascending)
    HeapNode first = {-2.0 * log(lam[0]), 0, 0};
    heap_push(heap, hn, first, occ, ne);
    // D(eps): the kept weight (1/Z) sum exp(-E), log Z = -sum_q log(1 - Lambda_q^2)
    const double tgt = a.eps_target;
    double logz = 0.0;
    for (int q = 0; q < ne; ++q) logz -= log1p(-lam[q] * lam[q]);
    double kw = exp(-logz);  // the vacuum state, E = 0
    int count = 1;
    while (count < chi && hn > 0 && !(tgt > 0.0 && 1.0 - kw <= tgt)) {
      HeapNode t = heap_pop(heap, hn, occ, ne);
      const int b = count++;
      kw += exp(-t.E - logz);
      E[b] = t.E; parent[b] = t.parent; pmode[b] = t.q; ntot[b] = ntot[t.parent] + 1;
      // materialise the occupation row now (needed for later tie-breaks)
      for (int j = 0; j < ne; ++j) occ[(long)b * ne + j] = occ[(long)t.parent * ne + j];
      occ[(long)b * ne + t.q] += 1;
      // child: b + e_q (same mode)
      HeapNode c = {t.E + (-2.0 * log(lam[t.q])), b, t.q};
      heap_push(heap, hn, c, occ, ne);
      // sibling: parent + e_{q+1}
      if (t.q + 1 < ne) {
        HeapNode s = {E[t.parent] + (-2.0 * log(lam[t.q + 1])), t.parent, t.q + 1};
        heap_push(heap, hn, s, occ, ne);
      }
    }
    a.chi_out[m] = count;
  }
  __syncthreads();
  const int nk = a.chi_out[m];
  // ---- hashes along the parent chains, compact occupied lists
  for (int b = tid; b < nk; b += nt) {
    unsigned long long h = 0ull;
    int k = 0;
    for (int j = 0; j < ne; ++j) {
      int n = occ[(long)b * ne + j];
      if (n) {
        h += (unsigned long long)n * splitmix64(0x5eed0000ull + j);
        if (k < GBS_K_MAX) olist[(long)b * GBS_K_MAX + k] = make_int4(j, n, -1, 0);
        ++k;
      }
    }
    H[b] = h;
    nocc[b] = k;
    if (k > GBS_K_MAX) gbs_set_error(a.err, GBS_DEVERR_KMAX);
  }
  __syncthreads();
  // ---- sort (hash, index) pairs (bitonic, padded to a power of two)
  int np2 = 1;
  while (np2 < nk) np2 <<= 1;
  unsigned long long* sh = (unsigned long long*)wbase;
  int* si = (int*)(sh + np2);
  for (int i = tid; i < np2; i += nt) {
    sh[i] = i < nk ? H[i] : ~0ull;
    si[i] = i < nk ? i : -1;
  }
  __syncthreads();
  for (int k = 2; k <= np2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < np2; i += nt) {
        int ixj = i ^ j;
        if (ixj > i) {
          bool up = (i & k) == 0;
          unsigned long long a0 = sh[i], a1 = sh[ixj];
          if ((a0 > a1) == up) {
            sh[i] = a1; sh[ixj] = a0;
            int t = si[i]; si[i] = si[ixj]; si[ixj] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  // ---- lowering table low[q][b] = index(b - e_q), verified
  for (long e = tid; e < (long)ne * nk; e += nt) {
    int q = (int)(e / nk), b = (int)(e % nk);
    int n = occ[(long)b * ne + q];
    int res = -1;
    if (n > 0) {
      unsigned long long target = H[b] - splitmix64(0x5eed0000ull + q);
      int lo = 0, hi = nk - 1;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (sh[mid] < target) lo = mid + 1;
        else hi = mid;
      }
      if (sh[lo] == target) res = si[lo];
      bool ok = res >= 0;
      if (ok) {
        for (int j = 0; j < ne && ok; ++j) {
          int want = occ[(long)b * ne + j] - (j == q);
          ok = occ[(long)res * ne + j] == want;
        }
      }
      if (!ok) {
        gbs_set_error(a.err, GBS_DEVERR_HASH);
        res = -1;
      }
    }
    low[(long)q * nk + b] = res;
  }
  __syncthreads();
  for (int b = tid; b < nk; b += nt) {
    int k = nocc[b] < GBS_K_MAX ? nocc[b] : GBS_K_MAX;
    for (int i = 0; i < k; ++i) {
      int4 o = olist[(long)b * GBS_K_MAX + i];
      o.z = low[(long)o.x * nk + b];
      olist[(long)b * GBS_K_MAX + i] = o;
    }
  }
}

size_t kept_workspace_bytes(int chi) {
  int np2 = 1;
  while (np2 < chi) np2 <<= 1;
  const size_t heap_bytes = (size_t)(2 * chi + 4) * sizeof(HeapNode);
  const size_t sort_bytes = (size_t)np2 * (sizeof(unsigned long long) + sizeof(int));
  const size_t b = heap_bytes > sort_bytes ? heap_bytes : sort_bytes;
  return (b + 255) / 256 * 256;
}

hipError_t launch_kept(hipStream_t st, const KeptArgs& a, int ncuts, int chi) {
  if (ncuts <= 0) return hipSuccess;
  const size_t ws = kept_workspace_bytes(chi);
  if (a.gws ? (long)ws > a.gws_stride : ws > kKeptLdsMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kept_kernel, dim3(ncuts), dim3(256), a.gws ? 0 : ws, st, a);
  return hipGetLastError();
}
