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

  // a basis the parallel enumeration wrote is only indexed here
  const bool enumerated = a.enum_done && a.enum_done[m];
  // zero the occupation table of this cut
  if (!enumerated)
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
  if (tid == 0 && !enumerated) {
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

// ---------------------------------------------------------------------------
// Parallel enumeration of one cut's kept basis (large chi).  The heap pops the
// states in the order of the key (E, occupation tuple descending), with E
// summed along the canonical parent chain: the photons of mode 0 first, then
// those of mode 1, and so on, each adding e_q = -2 log Lambda_q.  The first
// chi states in that order are the states with E below some threshold T plus
// the first of those at T.  Here:
//   1. T is found by doubling and bisection on counts: expanding the vacuum
//      over mode 0, then mode 1, ... (child j of a prefix adds e_q j times,
//      so every E is the heap's sum, bit for bit) and keeping E <= T gives
//      every state with E <= T; a count between chi and the workspace cap
//      stops the search;
//   2. the states with E <= T are expanded once more with their occupation
//      rows and sorted by the key (bitonic, in the workspace);
//   3. the first chi (or, for D(eps), the first whose kept weight reaches
//      1 - eps, summed in key order as the heap does) are written out.
// If the states at one energy are too many for the cap (degenerate modes), the
// cut is left to the heap (enum_done stays 0).
namespace {

constexpr int kEnumThreads = 1024;

__device__ inline long enum_cap(int chi) { return 4L * chi + 1024; }

__device__ int block_scan_excl(int v, int* sh, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (w == 0) {
    int t = lane < nw ? sh[lane] : 0;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(t, off, 64);
      if (lane >= off) t += y;
    }
    if (lane < nw) sh[lane] = t;
  }
  __syncthreads();
  const int base = w > 0 ? sh[w - 1] : 0;
  total = sh[nw - 1];
  __syncthreads();
  return base + x - v;
}

// States over modes 0..ne-1 with E <= T (E summed as the heap sums it), in
// Ea: returns their number, or cap + 1 if there are more than cap.  With
// lv (rows wanted), level q's prefixes record their parent in the previous
// level and their photons in mode q (lv_par / lv_n + q * cap), and *nlev
// receives the number of levels expanded.  On return the energies are in
// *pa.
__device__ long enum_expand(const double* e, int ne, double T, long cap, double* Ea, double* Eb, int* lv_par,
                            short* lv_n, int* nlev, int* sh, double** pa) {
  constexpr int kItems = 8;  // consecutive prefixes per thread and chunk
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) Ea[0] = 0.0;
  __syncthreads();
  long n = 1;
  int q = 0;
  for (; q < ne; ++q) {
    const double eq = e[q];
    // e ascends with q: once one photon of mode q exceeds T (the vacuum
    // prefix has E = 0), no later mode takes a photon either
    if (!(eq <= T)) break;
    long total = 0;
    bool over = false;
    for (long base = 0; base < n; base += (long)nt * kItems) {
      const long i0 = base + (long)tid * kItems;
      int cs[kItems];
      double xs[kItems];
      int tsum = 0;
#pragma unroll
      for (int it = 0; it < kItems; ++it) {
        const long i = i0 + it;
        int c = 0;
        double x = 0.0;
        if (i < n) {
          x = Ea[i];
          c = 1;
          double y = x + eq;
          while (y <= T && c <= cap) {
            ++c;
            y += eq;
          }
        }
        cs[it] = c;
        xs[it] = x;
        tsum += c;
      }
      int ctot;
      const int off = block_scan_excl(tsum, sh, ctot);
      if (total + ctot > cap) over = true;  // the same on every thread
      if (!over) {
        long o = total + off;
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
          double z = xs[it];
          for (int j = 0; j < cs[it]; ++j, ++o) {
            Eb[o] = z;
            if (lv_par) {
              lv_par[(long)q * cap + o] = (int)(i0 + it);
              lv_n[(long)q * cap + o] = (short)j;
            }
            z += eq;
          }
        }
      }
      total += ctot;
      if (over) break;
    }
    __syncthreads();
    if (over) return cap + 1;
    n = total;
    double* t = Ea;
    Ea = Eb;
    Eb = t;
  }
  if (nlev) *nlev = q;
  *pa = Ea;
  return n;
}

// key(ia) < key(ib): E ascending, ties by occupation tuple descending; -1 last
__device__ inline bool enum_less(int ia, int ib, const double* E, const short* R, int ne) {
  if (ib < 0) return ia >= 0;
  if (ia < 0) return false;
  const double ea = E[ia], eb = E[ib];
  if (ea != eb) return ea < eb;
  for (int j = 0; j < ne; ++j) {
    const short na = R[(long)ia * ne + j], nb = R[(long)ib * ne + j];
    if (na != nb) return na > nb;
  }
  return false;
}

}  // namespace

size_t kept_enum_bytes(int chi, int ne) {
  const long cap = 4L * chi + 1024;
  long np2 = 1;
  while (np2 < cap) np2 <<= 1;
  const size_t nn = ne > 0 ? ne : 1;
  // energies (ping-pong), per level parent and photons, rows, sort indices
  const size_t b = 2 * cap * sizeof(double) + nn * cap * (sizeof(int) + sizeof(short)) + cap * nn * sizeof(short) +
                   np2 * sizeof(int) + 64;
  return (b + 255) / 256 * 256;
}

__global__ __launch_bounds__(kEnumThreads) void kept_enum_kernel(KeptArgs a) {
  const int m = blockIdx.x;
  const CutDesc cd = a.cuts[m];
  const int ne = cd.ne, chi = cd.chi;
  if (ne == 0 || chi < kKeptParallelMin || ne > a.ews_ne || ne > kKeptEnumNeMax || cd.eslot < 0) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double e[kKeptEnumNeMax];
  __shared__ int sh[64];
  __shared__ int found;
  __shared__ double Tf;
  const double* lam = a.lam + (long)m * a.ld_lam;
  for (int q = tid; q < ne; q += nt) e[q] = -2.0 * log(lam[q]);
  const long cap = enum_cap(chi);
  long np2 = 1;
  while (np2 < cap) np2 <<= 1;
  char* w = a.ews + (long)cd.eslot * a.ews_stride;
  double* Ea = (double*)w;
  double* Eb = Ea + cap;
  int* lv_par = (int*)(Eb + cap);
  short* lv_n = (short*)(lv_par + (long)ne * cap);
  short* pr = lv_n + (long)ne * cap;  // rows of the final states
  int* idx = (int*)(((uintptr_t)(pr + cap * ne) + 15) & ~(uintptr_t)15);
  __syncthreads();
  // 1. the threshold: a count of states with E <= T near chi (at most
  // chi + chi/4 + 256, so that the sort stays small), or failing that the
  // smallest count in [chi, cap] met on the way
  const long wnd = chi + chi / 4 + 256 < cap ? chi + chi / 4 + 256 : cap;
  double lo = 0.0, hi = -1.0, T = e[0], best_T = -1.0;
  long best_c = cap + 1;
  double* pa;
  for (int it = 0; it < 400; ++it) {
    const long c = enum_expand(e, ne, T, cap, Ea, Eb, nullptr, nullptr, nullptr, sh, &pa);
    if (c >= chi && c <= wnd) {
      best_T = T;
      best_c = c;
      break;
    }
    if (c < chi) {
      lo = T;
    } else {
      hi = T;
      if (c <= cap && c < best_c) {
        best_c = c;
        best_T = T;
      }
    }
    const double nx = hi < 0.0 ? 2.0 * T : 0.5 * (lo + hi);
    if (!(nx > lo) || (hi >= 0.0 && !(nx < hi))) break;  // no double in between
    T = nx;
  }
  if (tid == 0) {
    found = best_T >= 0.0;
    Tf = best_T;
  }
  __syncthreads();
  if (!found) return;  // a tie too wide for the cap: the heap enumerates this cut
  // 2. every state with E <= T, its row rebuilt from the levels, sorted by the key
  __shared__ int nlev_s;
  int nlev = 0;
  const long n = enum_expand(e, ne, Tf, cap, Ea, Eb, lv_par, lv_n, &nlev, sh, &pa);
  if (tid == 0) nlev_s = nlev;
  __syncthreads();
  nlev = nlev_s;
  for (long i = tid; i < n; i += nt) {
    short* row = pr + i * ne;
    for (int j = nlev; j < ne; ++j) row[j] = 0;
    long k = i;
    for (int q = nlev - 1; q >= 0; --q) {
      row[q] = lv_n[(long)q * cap + k];
      k = lv_par[(long)q * cap + k];
    }
  }
  for (long i = tid; i < np2; i += nt) idx[i] = i < n ? (int)i : -1;
  __syncthreads();
  for (long k = 2; k <= np2; k <<= 1) {
    for (long j = k >> 1; j > 0; j >>= 1) {
      for (long i = tid; i < np2; i += nt) {
        const long ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const int x = idx[i], y = idx[ixj];
          if (up ? enum_less(y, x, pa, pr, ne) : enum_less(x, y, pa, pr, ne)) {
            idx[i] = y;
            idx[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // 3. the kept count (D(eps): the heap's running weight, summed in key
  // order by one thread over the energies gathered into key order)
  __shared__ int count;
  const double tgt = a.eps_target;
  if (tgt > 0.0) {
    double* Es = pa == Ea ? Eb : Ea;  // the energy buffer not holding the final states
    for (long b = tid; b < chi; b += nt) Es[b] = pa[idx[b]];
    __syncthreads();
    if (tid == 0) {
      double logz = 0.0;
      for (int q = 0; q < ne; ++q) logz -= log1p(-lam[q] * lam[q]);
      double kw = exp(-logz);
      int cnt = 1;
      while (cnt < chi && !(1.0 - kw <= tgt)) {
        kw += exp(-Es[cnt] - logz);
        ++cnt;
      }
      count = cnt;
    }
  } else if (tid == 0) {
    count = chi;
  }
  __syncthreads();
  if (tid == 0) a.chi_out[m] = count;
  double* E = a.E + cd.off_state;
  int* parent = a.parent + cd.off_state;
  int* pmode = a.pmode + cd.off_state;
  int* ntot = a.ntot + cd.off_state;
  short* occ = a.occ + cd.off_occ;
  for (int b = tid; b < chi; b += nt) {
    // rows past the kept count stay zero, as the heap leaves them
    const int src = b < count ? idx[b] : -1;
    int tot = 0, hm = -1;
    for (int j = 0; j < ne; ++j) {
      const short v = src >= 0 ? pr[(long)src * ne + j] : (short)0;
      occ[(long)b * ne + j] = v;
      tot += v;
      if (v) hm = j;
    }
    if (b < count) {
      E[b] = pa[src];
      ntot[b] = tot;
      parent[b] = -1;  // not needed past the enumeration
      pmode[b] = hm;
    }
  }
  if (tid == 0) a.enum_done[m] = 1;
}

hipError_t launch_kept_enum(hipStream_t st, const KeptArgs& a, int ncuts) {
  if (ncuts <= 0 || !a.ews) return hipSuccess;
  hipLaunchKernelGGL(kept_enum_kernel, dim3(ncuts), dim3(kEnumThreads), 0, st, a);
  return hipGetLastError();
}
