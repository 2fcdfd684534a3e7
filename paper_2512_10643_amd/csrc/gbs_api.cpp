// Host orchestration of the build, amplitude and sampling paths behind the
// C ABI declared in include/gbs_mps.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gbs_mps.h"
#include "gbs_common.h"
#include "gbs_gsvd.h"
#include "gbs_internal.h"
#include "gbs_kept.h"
#include "gbs_linalg.h"
#include "gbs_mpsops.h"
#include "gbs_pco.h"
#include "gbs_sampler.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int set_hip_error(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return fail(e == hipErrorOutOfMemory ? GBS_E_NOMEM : GBS_E_DEVICE,
              std::string("HIP error '") + hipGetErrorString(e) + "' in " + what);
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Stream-ordered allocations come from the device's default memory pool,
// which keeps up to this many freed bytes cached instead of returning them to
// the driver (repeated builds then allocate without a driver call).
constexpr uint64_t kPoolKeepBytes = 32ull << 30;

hipError_t ensure_pool(hipStream_t st) {
  static std::mutex mu;
  static std::vector<int> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  (void)st;
  std::lock_guard<std::mutex> lk(mu);
  if (std::find(done.begin(), done.end(), dev) != done.end()) return hipSuccess;
  hipMemPool_t pool;
  e = hipDeviceGetDefaultMemPool(&pool, dev);
  if (e != hipSuccess) return e;
  uint64_t keep = kPoolKeepBytes;
  e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  if (e != hipSuccess) return e;
  done.push_back(dev);
  return hipSuccess;
}

// Owning device allocation list.  With a stream, allocations are stream
// ordered (hipMallocAsync / hipFreeAsync on that stream), so releasing a
// temporary arena never waits for other streams; without one they are plain
// hipMalloc / hipFree (buffers owned by a handle).  A temporary arena (made
// with a stream) hands out buffers below kArenaChunk from chunks of that
// size by a bump pointer, so a build makes a few pool calls instead of one
// allocation and one free per buffer (each costs tens of microseconds of
// host time, and the frees at the end of a build leave the device idle);
// its buffers are all freed together.
constexpr size_t kArenaChunk = 64ull << 20;
struct DevArena {
  std::vector<void*> ptrs;
  int64_t bytes = 0;
  hipStream_t st = nullptr;
  bool ordered = false;
  bool pack = false;         // sub-allocate small buffers (temporary arenas)
  char* cur = nullptr;       // free space left in the current chunk
  size_t left = 0;
  DevArena() = default;
  explicit DevArena(hipStream_t s) : st(s), ordered(true), pack(true) {}
  DevArena(const DevArena&) = delete;
  DevArena& operator=(const DevArena&) = delete;
  hipError_t alloc(void** p, size_t n) {
    if (n == 0) n = 16;
    n = (n + 255) & ~(size_t)255;
    if (pack && n <= kArenaChunk / 2) {
      if (n > left) {
        void* c = nullptr;
        hipError_t e = hipMallocAsync(&c, kArenaChunk, st);
        if (e != hipSuccess) return e;
        ptrs.push_back(c);
        cur = (char*)c;
        left = kArenaChunk;
      }
      *p = cur;
      cur += n;
      left -= n;
      bytes += (int64_t)n;
      return hipSuccess;
    }
    hipError_t e = ordered ? hipMallocAsync(p, n, st) : hipMalloc(p, n);
    if (e == hipSuccess) {
      ptrs.push_back(*p);
      bytes += (int64_t)n;
    }
    return e;
  }
  void release(void* p) {  // one buffer of an arena that does not sub-allocate
    if (pack) return;       // its buffers go with the arena
    for (size_t i = 0; i < ptrs.size(); ++i)
      if (ptrs[i] == p) {
        (void)(ordered ? hipFreeAsync(p, st) : hipFree(p));
        ptrs.erase(ptrs.begin() + (long)i);
        return;
      }
  }
  void release_all() {
    for (void* p : ptrs) (void)(ordered ? hipFreeAsync(p, st) : hipFree(p));
    ptrs.clear();
    bytes = 0;
    cur = nullptr;
    left = 0;
  }
  ~DevArena() { release_all(); }
};

template <typename T>
hipError_t dalloc(DevArena& ar, T** p, size_t count) {
  return ar.alloc((void**)p, count * sizeof(T));
}

const char* deverr_msg(int code) {
  switch (code) {
    case GBS_DEVERR_NOT_PD: return "covariance block not positive definite (Cholesky pivot <= 0)";
    case GBS_DEVERR_NOT_PURE: return "covariance matrix is not pure";
    case GBS_DEVERR_WILLIAMSON: return "symplectic pairing of the Williamson form failed";
    case GBS_DEVERR_SINGULAR: return "Bogoliubov matrix U is singular";
    case GBS_DEVERR_HASH: return "kept-basis index lookup failed";
    case GBS_DEVERR_KMAX: return "size limit exceeded (too many occupied modes or entangled pairs)";
    case GBS_DEVERR_JACOBI: return "Jacobi eigensolver of a Williamson form did not converge";
    case GBS_DEVERR_JACOBI_BOND: return "Hermitian Jacobi eigensolver of a bond environment did not converge";
    default: return "unknown device error";
  }
}

}  // namespace

struct gbs_mps_s {
  int M = 0, d = 0, chi = 0, prec = 0;
  double dstar = 0, trunc_rel = 0;
  uint32_t flags = 0;
  DevArena keep;                 // buffers that live with the handle
  std::vector<int> ne, kept, bond;
  std::vector<double> eps, entropy;
  std::vector<std::vector<double>> lam;   // active Lambda per cut
  std::vector<std::vector<double>> svals; // singular values per bond
  double norm_raw = 0;
  int64_t pco_updates = 0;
  int64_t pco_terms = 0;          // source terms summed by the PCO level gather
  double t_pco_kernels = 0;       // device time of the level launches (HIP events)
  double t_gsvd = 0, t_kept = 0, t_pco = 0, t_svd = 0;
  int eig_sweeps = 0;            // sweeps of the bond eigensolver
  int single_site = 0;           // > 0: the handle holds that site's PCO tensor only
  int gsvd_independent = 0;      // 1: each site's Gaussian SVD ran on its own (bond modes aligned)
  // canonical tensors
  void* tens = nullptr;          // contiguous, element size esz
  size_t esz = 16;
  std::vector<long> toff;        // per site offset (elements)
  void** site_ptrs = nullptr;    // device array of per-site pointers
  int* bond_dev = nullptr;
  int maxbond = 1;
  // pair matrices: while building, Q^m in slot m - 1 - q_slot0 of a strided
  // buffer of the build's scratch arena (Q, q_stride, ld_q); afterwards
  // compact, Q^m (n_m x n_m) at Qc + qc_off[m], or qc_off[m] < 0 if not formed
  cplx64* Q = nullptr;
  long q_stride = 0, ld_q = 0;
  int q_slot0 = 0;
  cplx64* Qc = nullptr;
  std::vector<long> qc_off;
  float* packed = nullptr;       // MFMA sampler operand layout (FP32 builds)
  std::vector<long> poff;        // per site offset into `packed` (floats)
  long* poff_dev = nullptr;      // the same on the device, M + 1 entries
  std::vector<SamplerSite> ssite;  // per site sector sizes of the packed operand
  std::vector<SamplerGeom> sgeo;   // per site launch geometry (host copy)
  SamplerGeom* sgeo_dev = nullptr; // the same on the device, M + 1 entries
  bool psplit = false;           // bonds split into photon-parity sectors
  std::vector<int32_t> secn;     // (M+1) x 2 sector sizes when psplit
  long ldl2 = 0;                 // sampler row stride (floats)
  cplx64* raw = nullptr;         // PCO tensors (GBS_KEEP_RAW)
  std::vector<long> raw_off;
  short* occ = nullptr;
  std::vector<long> occ_off;
  int* err = nullptr;
};

namespace {

// Shots per sampling sweep.  The MFMA sweep takes up to 2^20 rows per
// ping-pong buffer (2 GB each at a 256-wide bond), so that a 10^6-shot call is
// one launch per site and the last, partly filled round of workgroups is a
// small part of it; the generic sweep keeps 2^18 (rows there are up to 16 KB).
constexpr int64_t kSampleChunk = (int64_t)1 << 20;
constexpr int64_t kSampleChunkGeneric = (int64_t)1 << 18;

template <typename C>
C cone() {
  return cmake<C>(1, 0);
}
template <typename C>
C czero() {
  return cmake<C>(0, 0);
}

// Truncation sweep and canonical form.  The Gram / environment matrices whose
// eigenvalues are the squared singular values, and their eigen-decompositions,
// are FP64; the gauge transforms that produce the stored tensors run in the
// build precision CT.
// A second stream of the calling thread on the current device (default
// priority), kept for the life of the thread, for work that overlaps a
// build's own stream.
hipError_t side_stream(hipStream_t* out) {
  thread_local std::vector<std::pair<int, hipStream_t>> own;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  for (auto& pr : own)
    if (pr.first == dev) {
      *out = pr.second;
      return hipSuccess;
    }
  hipStream_t s = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  own.push_back({dev, s});
  *out = s;
  return hipSuccess;
}

// The sampler's photon-parity masks of a reduced-precision build (a chain of
// small launches, bond after bond) run on a side stream while the build's
// own stream runs the FP64 norm chain; the normalisation of site 1 waits for
// the side stream to be done reading site 1.  The destructor waits for the
// side stream, so its work never outlives the build's temporaries.
struct MaskJob {
  hipStream_t side = nullptr;
  int32_t* mask = nullptr;      // (M + 1) x maxbond ints
  hipEvent_t ready = nullptr;   // final tensors on the build's stream
  hipEvent_t site1 = nullptr;   // side stream past site 1
  bool launched = false;
  MaskJob() = default;
  MaskJob(const MaskJob&) = delete;
  MaskJob& operator=(const MaskJob&) = delete;
  ~MaskJob() {
    if (launched) (void)hipStreamSynchronize(side);
    if (ready) (void)hipEventDestroy(ready);
    if (site1) (void)hipEventDestroy(site1);
  }
};

hipError_t launch_masks(gbs_mps_s* h, hipStream_t st, DevArena& tmp, MaskJob& mj) {
  const int M = h->M, d = h->d, mb = h->maxbond;
  const size_t bytes = (size_t)(M + 1) * mb * sizeof(int32_t);
  hipError_t e = tmp.alloc((void**)&mj.mask, bytes);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&mj.ready, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&mj.site1, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(mj.ready, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(mj.side, mj.ready, 0);
  if (e != hipSuccess) return e;
  mj.launched = true;
  e = hipMemsetAsync(mj.mask, 0, bytes, mj.side);
  for (int m = 1; m <= M && e == hipSuccess; ++m) {
    e = launch_sector_mask(mj.side, (const cplx32*)h->tens + h->toff[m], h->bond[m - 1], d, h->bond[m],
                           m == 1 ? nullptr : mj.mask + (long)(m - 1) * mb, mj.mask + (long)m * mb);
    if (e == hipSuccess && m == 1) e = hipEventRecord(mj.site1, mj.side);
  }
  return e;
}

template <typename CT>
int canonicalize(gbs_mps_s* h, hipStream_t st, DevArena& tmp, const cplx64* T64, const std::vector<long>& t64off,
                 MaskJob* mj) {
  typedef cplx64 C;
  const int M = h->M, d = h->d;
  const double tau = h->trunc_rel > 0 ? h->trunc_rel * h->trunc_rel : (std::is_same<CT, cplx64>::value ? 1e-24 : 1e-16);
  // working tensors A^m (FP64), dims (cl, d, cr)
  std::vector<int> cl(M + 1), cr(M + 1);
  std::vector<C*> A(M + 1, nullptr);
  for (int m = 1; m <= M; ++m) {
    cl[m] = h->kept[m - 1];
    cr[m] = h->kept[m];
    A[m] = (C*)(T64 + t64off[m]);
  }
  const int chi_ld = *std::max_element(h->kept.begin(), h->kept.end()) * d + 1;
  cplx64 *G64, *Vtmp, *Vec;
  double* w64;
  int* jerr = h->err;
  HIP_CHECK_RET(dalloc(tmp, &G64, (size_t)chi_ld * chi_ld));
  HIP_CHECK_RET(dalloc(tmp, &Vtmp, (size_t)chi_ld * chi_ld));
  HIP_CHECK_RET(dalloc(tmp, &Vec, (size_t)chi_ld * chi_ld));
  HIP_CHECK_RET(dalloc(tmp, &w64, (size_t)chi_ld));
  C *Gc, *Uc, *Xc;
  HIP_CHECK_RET(dalloc(tmp, &Gc, (size_t)chi_ld * chi_ld));
  HIP_CHECK_RET(dalloc(tmp, &Uc, (size_t)chi_ld * chi_ld));
  HIP_CHECK_RET(dalloc(tmp, &Xc, (size_t)chi_ld * chi_ld * d));
  std::vector<double> wh(chi_ld);

  // small Hermitian eigenproblem: Gc (n x n, ld n) -> w (desc), Vec (ld n)
  auto eig_small = [&](int n) -> int {
    HIP_CHECK_RET(convert<cplx64, C>(st, G64, Gc, (long)n * n));
    HIP_CHECK_RET(jacobi_herm(st, G64, Vtmp, w64, nullptr, n, 0, 1, jerr, Vec));
    HIP_CHECK_RET(hipMemcpyAsync(wh.data(), w64, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK_RET(hipStreamSynchronize(st));
    return 0;
  };
  auto keep_count = [&](int n) {
    int r = 0;
    for (int k = 0; k < n; ++k)
      if (wh[k] > tau * wh[0] && wh[k] > 0.0) ++r;
    return std::max(r, 1);
  };
  double* wdev;  // per-eigenproblem weights
  HIP_CHECK_RET(dalloc(tmp, &wdev, (size_t)chi_ld));

  // (1) left edge: bond m may be cut to rank(A^m as (cl d) x cr) when cl d < cr.
  for (int m = 1; m < M; ++m) {
    int rows = cl[m] * d, cols = cr[m];
    if (rows >= cols) break;
    // G = M M^H (rows x rows)
    HIP_CHECK_RET(zgemm<C>(st, rows, rows, cols, cone<C>(), A[m], cols, 0, 0, A[m], cols, 0, 2, czero<C>(), Gc, rows,
                           0, 1));
    if (int rc = eig_small(rows)) return rc;
    int r = keep_count(rows);
    HIP_CHECK_RET(hipMemcpyAsync(wdev, w64, r * sizeof(double), hipMemcpyDeviceToDevice, st));
    // X = U_r^H M (r x cols); new A^m = U_r S (rows x r); A^{m+1} <- S^-1 X A^{m+1}
    HIP_CHECK_RET(scaled_copy<C>(st, Uc, r, Vec, rows, rows, r, nullptr, 0, 0));      // U_r (rows x r)
    HIP_CHECK_RET(zgemm<C>(st, r, cols, rows, cone<C>(), Uc, r, 0, 2, A[m], cols, 0, 0, czero<C>(), Xc, cols, 0, 1));
    C* An;
    HIP_CHECK_RET(dalloc(tmp, &An, (size_t)rows * r));
    HIP_CHECK_RET(hipMemcpyAsync(An, Uc, sizeof(C) * rows * r, hipMemcpyDeviceToDevice, st));
    HIP_CHECK_RET(gauge_scale<C>(st, An, rows, 1, r, nullptr, wdev));                // * S
    HIP_CHECK_RET(gauge_scale<C>(st, Xc, r, 1, cols, wdev, nullptr));                // S^-1 *
    int n2 = d * cr[m + 1];
    C* Bn;
    HIP_CHECK_RET(dalloc(tmp, &Bn, (size_t)r * n2));
    HIP_CHECK_RET(zgemm<C>(st, r, n2, cols, cone<C>(), Xc, cols, 0, 0, A[m + 1], n2, 0, 0, czero<C>(), Bn, n2, 0, 1));
    A[m] = An;
    A[m + 1] = Bn;
    cr[m] = r;
    cl[m + 1] = r;
  }
  // (2) right edge: bond m-1 may be cut when d cr < cl.
  for (int m = M; m > 1; --m) {
    int rows = cl[m], cols = d * cr[m];
    if (cols >= rows) break;
    // G = M^H M (cols x cols)
    HIP_CHECK_RET(zgemm<C>(st, cols, cols, rows, cone<C>(), A[m], cols, 0, 2, A[m], cols, 0, 0, czero<C>(), Gc, cols,
                           0, 1));
    if (int rc = eig_small(cols)) return rc;
    int r = keep_count(cols);
    HIP_CHECK_RET(hipMemcpyAsync(wdev, w64, r * sizeof(double), hipMemcpyDeviceToDevice, st));
    // new A^m = S U_r^H (r x cols); X = M U_r S^-1 (rows x r); A^{m-1} <- A^{m-1} X
    C* An;
    HIP_CHECK_RET(dalloc(tmp, &An, (size_t)r * cols));
    HIP_CHECK_RET(scaled_copy<C>(st, An, cols, Vec, cols, r, cols, nullptr, 0, 1));   // U_r^H
    HIP_CHECK_RET(scaled_copy<C>(st, Uc, r, Vec, cols, cols, r, nullptr, 0, 0));      // U_r (cols x r)
    HIP_CHECK_RET(zgemm<C>(st, rows, r, cols, cone<C>(), A[m], cols, 0, 0, Uc, r, 0, 0, czero<C>(), Xc, r, 0, 1));
    {
      // rows of An times S = sqrt(w), columns of X times S^-1 (weights 1/w)
      std::vector<double> wi(r);
      for (int k = 0; k < r; ++k) wi[k] = 1.0 / wh[k];
      double* winv;
      HIP_CHECK_RET(dalloc(tmp, &winv, r));
      HIP_CHECK_RET(hipMemcpyAsync(winv, wi.data(), r * sizeof(double), hipMemcpyHostToDevice, st));
      HIP_CHECK_RET(gauge_scale<C>(st, Xc, rows, 1, r, nullptr, winv));
      HIP_CHECK_RET(gauge_scale<C>(st, An, r, 1, cols, winv, nullptr));
      HIP_CHECK_RET(hipStreamSynchronize(st));
    }
    int nl = cl[m - 1] * d;
    C* Bn;
    HIP_CHECK_RET(dalloc(tmp, &Bn, (size_t)nl * r));
    HIP_CHECK_RET(zgemm<C>(st, nl, r, rows, cone<C>(), A[m - 1], rows, 0, 0, Xc, r, 0, 0, czero<C>(), Bn, r, 0, 1));
    A[m] = An;
    A[m - 1] = Bn;
    cl[m] = r;
    cr[m - 1] = r;
  }
  // (3) right environments E_{m-1} = sum_p A^m[p] E_m A^m[p]^H, bonds 1..M-1.
  int emax = 1;
  for (int m = 1; m < M; ++m) emax = std::max(emax, cr[m]);
  const long eld = emax;
  cplx64 *E64, *EV64, *EVt;
  double* W64;
  C* Ec;
  C* Tb;
  HIP_CHECK_RET(dalloc(tmp, &E64, (size_t)(M + 1) * eld * eld));
  HIP_CHECK_RET(dalloc(tmp, &EV64, (size_t)(M + 1) * eld * eld));
  HIP_CHECK_RET(dalloc(tmp, &EVt, (size_t)(M + 1) * eld * eld));
  HIP_CHECK_RET(dalloc(tmp, &W64, (size_t)(M + 1) * eld));
  HIP_CHECK_RET(dalloc(tmp, &Ec, (size_t)2 * eld * eld));
  HIP_CHECK_RET(dalloc(tmp, &Tb, (size_t)eld * d * eld));
  std::vector<int> edim(M + 1, 1);
  // split-K workspace for the chain products (few output tiles, K = d chi)
  const long gws_elems = 8 * eld * eld;
  C* gws;
  HIP_CHECK_RET(dalloc(tmp, &gws, (size_t)gws_elems));
  {
    C one = cone<C>();
    HIP_CHECK_RET(hipMemcpyAsync(Ec, &one, sizeof(C), hipMemcpyHostToDevice, st));
    int cur = 0;
    // FP64 environments are written straight into their slots of E64 (and
    // read back from there for the next step); others go through Ec
    constexpr bool direct = std::is_same<C, cplx64>::value;
    for (int m = M; m >= 2; --m) {
      int a = cl[m], b = cr[m];
      C* Ein = Ec + (long)cur * eld * eld;
      C* Eout = Ec + (long)(1 - cur) * eld * eld;
      if (direct) {
        if (m < M) Ein = (C*)(E64 + (long)m * eld * eld);
        Eout = (C*)(E64 + (long)(m - 1) * eld * eld);
      }
      // Tb[:, p, :] = A^m[:, p, :] E_m   (batched over p)
      HIP_CHECK_RET(zgemm<C>(st, a, b, b, cone<C>(), A[m], (long)d * b, b, 0, Ein, eld, 0, 0, czero<C>(), Tb,
                             (long)d * b, b, d));
      // E_{m-1} = Tb (a x d b) * A^m^H, stored with leading dimension eld
      HIP_CHECK_RET(zgemm<C>(st, a, a, d * b, cone<C>(), Tb, (long)d * b, 0, 0, A[m], (long)d * b, 0, 2, czero<C>(),
                             Eout, eld, 0, 1, gws, gws_elems));
      if (!direct) HIP_CHECK_RET(convert<cplx64, C>(st, E64 + (long)(m - 1) * eld * eld, Eout, (long)a * eld));
      edim[m - 1] = a;
      cur = 1 - cur;
    }
  }
  // (4) all bond eigenproblems in parallel (FP64 Jacobi), bonds 1..M-1
  int* edim_dev;
  HIP_CHECK_RET(dalloc(tmp, &edim_dev, M + 1));
  {
    // the Jacobi kernel needs a contiguous square leading dimension per matrix:
    // matrices are stored with leading dimension eld (row stride) already.
    HIP_CHECK_RET(hipMemcpyAsync(edim_dev, edim.data(), (M + 1) * sizeof(int), hipMemcpyHostToDevice, st));
    if (M > 1) {
      // blocked Jacobi over all bonds at once
      const int nb = M - 1;
      const long off = eld * eld;
      cplx64* vsub;
      int* active;
      double* dmx;
      int* vid;
      HIP_CHECK_RET(dalloc(tmp, &vsub, (size_t)jacobi_blocked_ws_elems((int)eld, nb)));
      HIP_CHECK_RET(dalloc(tmp, &vid, (size_t)jacobi_blocked_ws_elems((int)eld, nb) / 1024 + 1));
      HIP_CHECK_RET(dalloc(tmp, &active, nb));
      HIP_CHECK_RET(dalloc(tmp, &dmx, nb));
      int sweeps = 0;
      HIP_CHECK_RET(jacobi_herm_blocked(st, E64 + off, EVt + off, W64 + eld, edim_dev + 1, (int)eld, eld, eld * eld, nb,
                                        jerr, EV64 + off, vsub, active, vid, dmx, 60, &sweeps));
      if (sweeps < 0) return fail(GBS_E_INTERNAL, deverr_msg(GBS_DEVERR_JACOBI_BOND));
      h->eig_sweeps = sweeps;
    }
  }
  std::vector<double> wall((size_t)(M + 1) * eld);
  HIP_CHECK_RET(hipMemcpyAsync(wall.data(), W64, wall.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  int herr = 0;
  HIP_CHECK_RET(hipMemcpyAsync(&herr, jerr, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipStreamSynchronize(st));
  if (herr) return fail(GBS_E_INTERNAL, deverr_msg(herr));
  std::vector<int> r(M + 1, 1);
  h->svals.assign(M + 1, {});
  for (int m = 1; m < M; ++m) {
    const double* w = &wall[(size_t)m * eld];
    int n = edim[m], k = 0;
    for (int i = 0; i < n; ++i)
      if (w[i] > tau * w[0] && w[i] > 0.0) ++k;
    k = std::max(1, std::min(k, h->chi));
    r[m] = k;
    h->svals[m].resize(k);
    for (int i = 0; i < k; ++i) h->svals[m][i] = std::sqrt(w[i]);
  }
  // (5) B^m = S_{m-1}^-1 U_{m-1}^H A^m[p] U_m S_m, in the build precision
  long total = 0;
  h->toff.assign(M + 1, 0);
  for (int m = 1; m <= M; ++m) {
    h->toff[m] = total;
    total += (long)r[m - 1] * d * r[m];
  }
  CT* out;
  HIP_CHECK_RET(dalloc(h->keep, &out, (size_t)total));
  h->tens = out;
  h->esz = sizeof(CT);
  CT *Ub, *Am, *Tc;  // U_m in precision CT (eld x eld), one site tensor, scratch
  HIP_CHECK_RET(dalloc(tmp, &Ub, (size_t)(M + 1) * eld * eld));
  HIP_CHECK_RET(dalloc(tmp, &Am, (size_t)eld * d * eld + d));
  HIP_CHECK_RET(dalloc(tmp, &Tc, (size_t)eld * d * eld + d));
  for (int m = 1; m < M; ++m)
    HIP_CHECK_RET(scaled_copy<CT>(st, Ub + (long)m * eld * eld, eld, EV64 + (long)m * eld * eld, eld, edim[m], r[m],
                                  nullptr, 0, 0));
  // site transforms in the build precision: FP64 or FP32 MFMA, or split-BF16x3
  auto gemm_ct = [&](int Mr, int Nc, int K, const CT* Ap, long lda, long sAp, int opA, const CT* Bp, long ldb,
                     long sBp, CT* Cp, long ldc, long sCp, int batch) -> hipError_t {
    if (h->prec == GBS_BF16X3)
      return zgemm_bf16x3(st, Mr, Nc, K, cone<cplx32>(), (const cplx32*)Ap, lda, sAp, opA, (const cplx32*)Bp, ldb,
                          sBp, 0, czero<cplx32>(), (cplx32*)Cp, ldc, sCp, batch);
    return zgemm<CT>(st, Mr, Nc, K, cone<CT>(), Ap, lda, sAp, opA, Bp, ldb, sBp, 0, czero<CT>(), Cp, ldc, sCp, batch);
  };
  // Interior sites of equal shape whose FP64 tensors lie back to back in
  // the PCO buffer go through in runs of up to kRun: one conversion and two
  // batched products per run (Y = A^m U_m as one (a d) x b by b x r_m
  // product per site, then U_{m-1}^H Y), instead of a launch sequence per
  // site.
  constexpr int kRun = 16;
  CT *AmR = nullptr, *TcR = nullptr;
  auto run_end = [&](int m0) {
    int e = m0;
    while (e < M && e - m0 < kRun && cl[e] == cl[m0] && cr[e] == cr[m0] && r[e - 1] == r[m0 - 1] &&
           r[e] == r[m0] && A[e] == (C*)(T64 + t64off[e]) &&
           (e == m0 || t64off[e] - t64off[e - 1] == (long)cl[m0] * d * cr[m0]))
      ++e;
    return e;
  };
  for (int m = 1; m <= M; ++m) {
    if (m > 1 && m < M) {
      const int e = run_end(m);
      if (e - m >= 2) {
        const int a = cl[m], b = cr[m], ra = r[m - 1], rb = r[m], ns = e - m;
        if (!AmR) {
          HIP_CHECK_RET(dalloc(tmp, &AmR, (size_t)kRun * eld * d * eld));
          HIP_CHECK_RET(dalloc(tmp, &TcR, (size_t)kRun * eld * d * eld));
        }
        HIP_CHECK_RET(convert<CT, cplx64>(st, AmR, A[m], (long)ns * a * d * b));
        HIP_CHECK_RET(gemm_ct(a * d, rb, b, AmR, b, (long)a * d * b, 0, Ub + (long)m * eld * eld, eld, eld * eld, TcR,
                              rb, (long)a * d * rb, ns));
        HIP_CHECK_RET(gemm_ct(ra, d * rb, a, Ub + (long)(m - 1) * eld * eld, eld, eld * eld, 2, TcR, (long)d * rb,
                              (long)a * d * rb, out + h->toff[m], (long)d * rb, (long)ra * d * rb, ns));
        for (int k = m; k < e; ++k)
          HIP_CHECK_RET(gauge_scale<CT>(st, out + h->toff[k], ra, d, rb, W64 + (long)(k - 1) * eld, W64 + (long)k * eld));
        m = e - 1;
        continue;
      }
    }
    int a = cl[m], b = cr[m], ra = r[m - 1], rb = r[m];
    HIP_CHECK_RET(convert<CT, cplx64>(st, Am, A[m], (long)a * d * b));
    // Y = A^m[p] U_m  (a x d x rb)
    const CT* Y = Am;
    if (m < M) {
      HIP_CHECK_RET(gemm_ct(a, rb, b, Am, (long)d * b, b, 0, Ub + (long)m * eld * eld, eld, 0, Tc, (long)d * rb, rb,
                            d));
      Y = Tc;
    }
    CT* Bm = out + h->toff[m];
    if (m > 1) {
      HIP_CHECK_RET(gemm_ct(ra, d * rb, a, Ub + (long)(m - 1) * eld * eld, eld, 0, 2, Y, (long)d * rb, 0, Bm,
                            (long)d * rb, 0, 1));
    } else {
      HIP_CHECK_RET(hipMemcpyAsync(Bm, Y, sizeof(CT) * (long)a * d * rb, hipMemcpyDeviceToDevice, st));
    }
    const double* wl = m > 1 ? W64 + (long)(m - 1) * eld : nullptr;
    const double* wr = m < M ? W64 + (long)m * eld : nullptr;
    HIP_CHECK_RET(gauge_scale<CT>(st, Bm, ra, d, rb, wl, wr));
  }
  // (6) normalise and fix the phase
  h->bond = r;
  h->maxbond = *std::max_element(r.begin(), r.end());
  if (mj && mj->side && !std::is_same<CT, cplx64>::value && h->maxbond <= 2 * kSamplerMaxSector &&
      d <= kSamplerMaxOutcomes && !(h->flags & GBS_DENSE_SAMPLER))
    HIP_CHECK_RET(launch_masks(h, st, tmp, *mj));
  HIP_CHECK_RET(dalloc(h->keep, &h->bond_dev, M + 1));
  HIP_CHECK_RET(hipMemcpyAsync(h->bond_dev, r.data(), (M + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  std::vector<void*> ptrs(M);
  for (int m = 1; m <= M; ++m) ptrs[m - 1] = out + h->toff[m];
  HIP_CHECK_RET(dalloc(h->keep, &h->site_ptrs, M));
  HIP_CHECK_RET(hipMemcpyAsync(h->site_ptrs, ptrs.data(), M * sizeof(void*), hipMemcpyHostToDevice, st));
  double* nrm;
  HIP_CHECK_RET(dalloc(tmp, &nrm, 1));
  // Vacuum amplitude z = <0..0|psi> = B^1[0, 0, :] ... B^M[:, 0, 0] (FP64
  // chain of vector-matrix products), for the global phase.  Reduced-precision
  // tensors are right-canonical only to their rounding level, and those
  // deviations add up along the chain; their squared norm is therefore taken
  // from the full FP64 transfer chain
  //   L_m = sum_p B^m[p]^H L_{m-1} B^m[p],  L_0 = 1,  norm^2 = L_M.
  const double* nrm2_dev = nullptr;
  C *vac, *Lb = nullptr, *B64 = nullptr, *X64 = nullptr;
  C one = cone<C>();
  HIP_CHECK_RET(dalloc(tmp, &vac, (size_t)2 * eld));
  HIP_CHECK_RET(hipMemcpyAsync(vac, &one, sizeof(C), hipMemcpyHostToDevice, st));
  const bool reduced = !std::is_same<CT, cplx64>::value;
  if (reduced) {
    HIP_CHECK_RET(dalloc(tmp, &Lb, (size_t)2 * eld * eld));
    HIP_CHECK_RET(dalloc(tmp, &B64, (size_t)eld * d * eld + d));
    HIP_CHECK_RET(dalloc(tmp, &X64, (size_t)eld * d * eld + d));
    HIP_CHECK_RET(hipMemcpyAsync(Lb, &one, sizeof(C), hipMemcpyHostToDevice, st));
  }
  int cur = 0;
  for (int m = 1; m <= M; ++m) {
    const int a = r[m - 1], b = r[m];
    const C* Bs;
    if (reduced) {
      HIP_CHECK_RET(convert<cplx64, CT>(st, B64, out + h->toff[m], (long)a * d * b));
      Bs = B64;
    } else {
      Bs = (const C*)(out + h->toff[m]);
    }
    // z chain: v (1 x a) * B[:, 0, :] (a x b, row stride d b)
    HIP_CHECK_RET(zgemm<C>(st, 1, b, a, one, vac + (long)cur * eld, a, 0, 0, Bs, (long)d * b, 0, 0, czero<C>(),
                           vac + (long)(1 - cur) * eld, b, 0, 1));
    if (reduced) {
      C* Lin = Lb + (long)cur * eld * eld;
      C* Lout = Lb + (long)(1 - cur) * eld * eld;
      // X = L_{m-1} B (a x d b), then L_m = B^H X over the (a, p) rows
      HIP_CHECK_RET(zgemm<C>(st, a, d * b, a, one, Lin, eld, 0, 0, B64, (long)d * b, 0, 0, czero<C>(), X64,
                             (long)d * b, 0, 1));
      HIP_CHECK_RET(zgemm<C>(st, b, b, a * d, one, B64, b, 0, 2, X64, b, 0, 0, czero<C>(), Lout, eld, 0, 1, gws,
                             gws_elems));
    }
    cur = 1 - cur;
  }
  if (reduced) nrm2_dev = (const double*)(Lb + (long)cur * eld * eld);  // real part of the 1 x 1 L_M
  if (mj && mj->launched) HIP_CHECK_RET(hipStreamWaitEvent(st, mj->site1, 0));
  HIP_CHECK_RET(normalize_mps<CT>(st, out + h->toff[1], d * r[1], vac + (long)cur * eld, nrm2_dev, nrm));
  HIP_CHECK_RET(hipMemcpyAsync(&h->norm_raw, nrm, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipStreamSynchronize(st));
  return GBS_OK;
}

// Every site's Gaussian data on its own, all sites in one batch (Sec. III.A):
// site m starts the chain at cut m - 1 straight from Gamma and takes one step
// to cut m, forming Q^m; then the bond modes of every cut are aligned between
// its two neighbours (a phase per mode, put into Q^m), so the tensors fit
// together as the sequential chain's do.  Fills h->Q (leading dimension
// h->ld_q), ne (host, M + 1), and the Lambda of every cut on the device
// (*lam, row stride ld_lam) and on the host (lamh).  Returns GBS_DEVERR_ALIGN
// through *dev_err when the two sides of a cut count different entangled
// pairs (a D within rounding of D*), and the caller then runs the chain.
int gsvd_independent(gbs_mps_s* h, const double* gamma, int M, double dstar, hipStream_t st, DevArena& tmp, int* err,
                     std::vector<int>& ne, std::vector<double>& lamh, double** lam, long ld_lam, int* dev_err) {
  // one pool of doubles and one of ints, carved per site: site m's blocks are
  // at most 2m wide (cut m - 1 from Gamma: 2(m - 1); its step: 2(n_e + 1)).
  // carve(m, base, ...) lays site m's buffers out from `base` (NULL: count).
  std::vector<GsvdArgs> a0(M), a1(M);
  std::vector<int> c0(M), c1(M);
  std::vector<double*> keep(M);
  std::vector<long> keep_ld(M);
  auto carve = [&](int m, double* base, int* ip) -> long {
    const long n2 = 2L * m, lu = m + 1;
    long used = 0;
    auto take = [&](long n) {
      double* r = base ? base + used : nullptr;
      used += (n + 31) / 32 * 32;
      return r;
    };
    GsvdArgs g{};
    g.M = M;
    g.dstar = dstar;
    g.gamma = gamma;
    g.err = err;
    g.ne = ip;
    g.ws_ord = ip ? ip + (M + 1) : nullptr;
    g.ld_dsym = lu;
    g.dsym = take((long)(M + 1) * lu);
    g.lam = take((long)(M + 1) * lu);
    g.ld_drr = n2;
    g.ld_cr = 2L * M;
    double* drr0 = take(n2 * n2);
    double* drr1 = take(n2 * n2);
    double* cr0 = take(n2 * 2L * M);
    double* cr1 = take(n2 * 2L * M);
    g.Q = h->Q;
    g.q_stride = h->q_stride;
    g.ld_q = h->ld_q;
    g.ld_ws = n2;
    g.ws_G = take(n2 * n2);
    g.ws_L = take(n2 * n2);
    g.ws_A = take(n2 * n2);
    g.ws_B = take(n2 * n2);
    g.ws_E = take(n2 * n2);
    g.ws_O = take(n2 * n2);
    g.ws_S = take(n2 * n2);
    g.ws_W = take(n2 * n2);
    double* kp = take(n2 * n2);
    g.ws_vec = take(3 * n2);
    g.ws_pack = take(n2 * (n2 + 1) / 2);
    g.ws_w = take(n2);
    g.ld_glr = 2L * M;
    g.ws_glr = take(n2 * 2L * M);
    g.ws_tri = take(2 * n2 * n2 + 4 * n2);
    g.ld_u = lu;
    g.ws_U = (cplx64*)take(2 * lu * lu);
    g.ws_V = (cplx64*)take(2 * lu * lu);
    g.ws_aug = (cplx64*)take(2 * lu * 2 * lu);
    g.q_first = m;
    if (base) {
      keep[m - 1] = kp;
      keep_ld[m - 1] = n2;
      a0[m - 1] = g;
      a0[m - 1].drr_in = drr0;
      a0[m - 1].cr_in = cr0;
      a0[m - 1].drr_out = drr1;
      a0[m - 1].cr_out = cr1;
      a1[m - 1] = g;
      a1[m - 1].drr_in = drr1;
      a1[m - 1].cr_in = cr1;
      a1[m - 1].drr_out = drr0;
      a1[m - 1].cr_out = cr0;
      c0[m - 1] = m - 1;
      c1[m - 1] = m;
    }
    return used;
  };
  std::vector<long> dof(M + 1), iof(M + 1);
  long dtot = 0, itot = 0;
  for (int m = 1; m <= M; ++m) {
    dof[m] = dtot;
    dtot += carve(m, nullptr, nullptr);
    iof[m] = itot;
    itot += (M + 1) + 2L * m + 64;  // ne, ord
  }
  double* dpool;
  int* ipool;
  HIP_CHECK_RET(dalloc(tmp, &dpool, (size_t)dtot));
  HIP_CHECK_RET(dalloc(tmp, &ipool, (size_t)itot));
  HIP_CHECK_RET(hipMemsetAsync(ipool, 0, (size_t)itot * sizeof(int), st));
  for (int m = 1; m <= M; ++m) carve(m, dpool + dof[m], ipool + iof[m]);
  std::vector<GsvdAlign> al(M - 1);
  for (int m = 1; m < M; ++m) {
    GsvdAlign& x = al[m - 1];
    x.t0 = m >= 2 ? keep[m - 1] : nullptr;
    x.ldt0 = keep_ld[m - 1];
    x.ne_e = a0[m - 1].ne;
    x.t1 = a0[m - 1].ws_A;
    x.ldt1 = a0[m - 1].ld_ws;
    x.tr = keep[m];
    x.ldtr = keep_ld[m];
    x.ne_r = a0[m].ne;
    x.Q = h->Q + (long)(m - 1) * h->q_stride;
    x.ld_q = h->ld_q;
    x.m = m;
  }
  GsvdArgs *a0d, *a1d;
  int *c0d, *c1d;
  double** keepd;
  long* keepld;
  GsvdAlign* ald;
  HIP_CHECK_RET(dalloc(tmp, &a0d, M));
  HIP_CHECK_RET(dalloc(tmp, &a1d, M));
  HIP_CHECK_RET(dalloc(tmp, &c0d, M));
  HIP_CHECK_RET(dalloc(tmp, &c1d, M));
  HIP_CHECK_RET(dalloc(tmp, &keepd, M));
  HIP_CHECK_RET(dalloc(tmp, &keepld, M));
  HIP_CHECK_RET(dalloc(tmp, &ald, std::max(M - 1, 1)));
  HIP_CHECK_RET(hipMemcpyAsync(a0d, a0.data(), M * sizeof(GsvdArgs), hipMemcpyHostToDevice, st));
  HIP_CHECK_RET(hipMemcpyAsync(a1d, a1.data(), M * sizeof(GsvdArgs), hipMemcpyHostToDevice, st));
  HIP_CHECK_RET(hipMemcpyAsync(c0d, c0.data(), M * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_CHECK_RET(hipMemcpyAsync(c1d, c1.data(), M * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_CHECK_RET(hipMemcpyAsync(keepd, keep.data(), M * sizeof(double*), hipMemcpyHostToDevice, st));
  HIP_CHECK_RET(hipMemcpyAsync(keepld, keep_ld.data(), M * sizeof(long), hipMemcpyHostToDevice, st));
  if (M > 1) HIP_CHECK_RET(hipMemcpyAsync(ald, al.data(), (M - 1) * sizeof(GsvdAlign), hipMemcpyHostToDevice, st));
  HIP_CHECK_RET(launch_gsvd_independent(st, a0d, a1d, c0d, c1d, M, keepd, keepld, ald, M - 1, err));
  int* ne_d;
  HIP_CHECK_RET(dalloc(tmp, &ne_d, M + 1));
  HIP_CHECK_RET(dalloc(tmp, lam, (size_t)(M + 1) * ld_lam));
  HIP_CHECK_RET(hipMemsetAsync(ne_d, 0, (M + 1) * sizeof(int), st));
  HIP_CHECK_RET(hipMemsetAsync(*lam, 0, (M + 1) * ld_lam * sizeof(double), st));
  HIP_CHECK_RET(launch_gsvd_gather_cuts(st, a1d, M, ne_d, *lam, ld_lam));
  ne.assign(M + 1, 0);
  lamh.assign((size_t)(M + 1) * ld_lam, 0.0);
  HIP_CHECK_RET(hipMemcpyAsync(ne.data(), ne_d, (M + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipMemcpyAsync(lamh.data(), *lam, lamh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipMemcpyAsync(dev_err, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipStreamSynchronize(st));
  return GBS_OK;
}

int build_impl(const double* gamma, int M, const gbs_build_opts* opt, hipStream_t st, gbs_mps_s* h, int only_site) {
  // kept states per cut (D_build); the truncation sweep caps bonds at h->chi
  const int d = opt->d, chi = only_site ? opt->chi : std::max(opt->chi, opt->chi_build);
  HIP_CHECK_RET(ensure_pool(st));
  DevArena tmp(st);
  int* err;
  HIP_CHECK_RET(dalloc(h->keep, &err, 4));
  h->err = err;
  HIP_CHECK_RET(hipMemsetAsync(err, 0, 4 * sizeof(int), st));
  // ---- validation
  {
    double* scal;
    double* wsM;
    HIP_CHECK_RET(dalloc(tmp, &scal, 4));
    HIP_CHECK_RET(dalloc(tmp, &wsM, (size_t)M * M));
    HIP_CHECK_RET(launch_validate(st, gamma, M, scal, wsM, err));
    double hs[3];
    int herr = 0;
    HIP_CHECK_RET(hipMemcpyAsync(hs, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK_RET(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK_RET(hipStreamSynchronize(st));
    double scale = std::max(1.0, 2.0 * hs[1]);
    if (!(hs[0] <= 1e-10 * scale)) return fail(GBS_E_NOT_PD, "Gamma is not symmetric");
    if (herr) return fail(GBS_E_NOT_PD, "Gamma is not positive definite");
    if (!(hs[2] <= 1e-8 * scale * scale)) {
      char buf[128];
      snprintf(buf, sizeof buf, "Gamma is not pure: |(2 Gamma Omega)^2 + 1|_max = %.3e", hs[2]);
      return fail(GBS_E_NOT_PURE, buf);
    }
  }
  // ---- Gaussian SVD chain
  double t0 = now_ms();
  // A single-site build starts the chain at cut k = s - 1 straight from Gamma
  // (a_1..a_{k-1} stand in for r_{k-1}, Sec. III.A): two steps instead of
  // s.  Its first L block is 2 k wide, so k is capped at what one workgroup
  // takes; beyond that the chain runs from the cap to s.
  const int restart = only_site >= 3 ? std::min(only_site - 1, GBS_GSVD_N2_MAX / 2) : 0;
  const int n2max = std::min(GBS_GSVD_N2_MAX, std::max(M + 2, 2 * restart));
  GsvdArgs ga{};
  ga.M = M;
  ga.dstar = opt->dstar;
  ga.gamma = gamma;
  ga.err = err;
  HIP_CHECK_RET(dalloc(tmp, &ga.ne, M + 1));
  HIP_CHECK_RET(hipMemsetAsync(ga.ne, 0, (M + 1) * sizeof(int), st));
  ga.ld_dsym = n2max / 2 + 1;
  HIP_CHECK_RET(dalloc(tmp, &ga.dsym, (size_t)(M + 1) * ga.ld_dsym));
  HIP_CHECK_RET(dalloc(tmp, &ga.lam, (size_t)(M + 1) * ga.ld_dsym));
  ga.ld_drr = n2max;
  ga.ld_cr = 2 * M;
  double *drr[2], *cr[2];
  for (int i = 0; i < 2; ++i) {
    HIP_CHECK_RET(dalloc(tmp, &drr[i], (size_t)n2max * n2max));
    HIP_CHECK_RET(dalloc(tmp, &cr[i], (size_t)n2max * 2 * M));
  }
  h->ld_q = n2max;  // n_modes <= nL + ne <= n2max
  h->q_stride = (long)h->ld_q * h->ld_q;
  h->q_slot0 = only_site ? only_site - 1 : 0;  // a single-site build forms Q^s alone
  HIP_CHECK_RET(dalloc(tmp, &h->Q, (size_t)(only_site ? 1 : M) * h->q_stride));
  ga.Q = h->Q;
  ga.q_stride = h->q_stride;
  ga.ld_q = h->ld_q;
  ga.q_slot0 = h->q_slot0;
  ga.ld_ws = n2max;
  const size_t wsz = (size_t)n2max * n2max;
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_G, wsz));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_L, wsz));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_A, wsz));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_B, wsz));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_E, wsz));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_O, wsz));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_S, wsz));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_vec, (size_t)3 * n2max));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_W, wsz));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_pack, (size_t)n2max * (n2max + 1) / 2));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_w, (size_t)n2max));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_ord, (size_t)n2max));
  ga.ld_glr = 2 * M;
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_glr, (size_t)n2max * 2 * M));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_tri, (size_t)2 * n2max * n2max + 4 * n2max));
  ga.ld_u = n2max / 2 + 1;
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_U, (size_t)ga.ld_u * ga.ld_u));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_V, (size_t)ga.ld_u * ga.ld_u));
  HIP_CHECK_RET(dalloc(tmp, &ga.ws_aug, (size_t)ga.ld_u * 2 * ga.ld_u));
  ga.q_first = only_site;  // a single-site build forms Q^s alone
  std::vector<int> ne(M + 1);
  std::vector<double> lamh((size_t)(M + 1) * ga.ld_dsym);
  int herr = 0;
  // Full builds whose every first block fits one workgroup (2 (M - 1) wide
  // for the last site) build each site's Gaussian data on its own; otherwise,
  // or on request, the sequential chain runs.
  bool chain = only_site || M < 3 || 2 * (M - 1) > GBS_GSVD_N2_MAX || (opt->flags & GBS_CHAIN_GSVD);
  if (!chain) {
    double* lam_ind = nullptr;
    if (int rc = gsvd_independent(h, gamma, M, opt->dstar, st, tmp, err, ne, lamh, &lam_ind, ga.ld_dsym, &herr))
      return rc;
    // The two sides of a cut fix a bond mode's (x, p) rotation separately.  A
    // mode with D close to 1 sits next to the vacuum cluster of its block
    // (D = 1 exactly), so each side's mode carries an admixture of vacuum
    // modes of order eps / (D - 1) that a per-mode phase cannot align; its
    // weight in the state is Lambda ~ sqrt((D - 1) / 2), so amplitudes move
    // by about eps n / Lambda.  Below Lambda = 1e-3 (D - 1 < 2e-6) that
    // exceeds the FP64 accuracy the chain keeps (1e-10 at 2 M = 600), and
    // the chain runs instead.
    bool weak = false;
    if (!herr)
      for (int m = 1; m < M && !weak; ++m)
        for (int q = 0; q < ne[m]; ++q)
          if (lamh[(size_t)m * ga.ld_dsym + q] < GBS_GSVD_INDEP_LAMBDA_MIN) weak = true;
    if (herr == GBS_DEVERR_ALIGN || weak) {  // a cut counted differently on its two sides, or a weak mode
      HIP_CHECK_RET(hipMemsetAsync(err, 0, sizeof(int), st));
      herr = 0;
      chain = true;
    } else {
      ga.lam = lam_ind;
      h->gsvd_independent = 1;
    }
  }
  if (chain && restart) {
    ga.drr_in = drr[(restart + 1) & 1];
    ga.cr_in = cr[(restart + 1) & 1];
    HIP_CHECK_RET(launch_gsvd_restart(st, ga, restart));
  }
  if (chain) {
    const int m_first = restart ? restart : 1, m_last = only_site ? only_site : M;
    for (int m = m_first; m <= m_last; ++m) {
      ga.drr_in = drr[(m + 1) & 1];
      ga.drr_out = drr[m & 1];
      ga.cr_in = cr[(m + 1) & 1];
      ga.cr_out = cr[m & 1];
      HIP_CHECK_RET(launch_gsvd_cut(st, ga, m, n2max));
    }
    if (only_site && only_site < M)
      HIP_CHECK_RET(launch_gsvd_q(st, ga, only_site));
    else
      HIP_CHECK_RET(launch_gsvd_last_q(st, ga));
    HIP_CHECK_RET(hipMemcpyAsync(ne.data(), ga.ne, (M + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK_RET(hipMemcpyAsync(lamh.data(), ga.lam, lamh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK_RET(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK_RET(hipStreamSynchronize(st));
  }
  if (herr)
    return fail(herr == GBS_DEVERR_NOT_PD ? GBS_E_NOT_PD : herr == GBS_DEVERR_KMAX ? GBS_E_INVAL : GBS_E_INTERNAL,
                deverr_msg(herr));
  if (only_site)  // only the two cuts of the site were formed
    for (int m = 0; m <= M; ++m)
      if (m != only_site - 1 && m != only_site) ne[m] = 0;
  h->ne = ne;
  h->lam.assign(M + 1, {});
  h->entropy.assign(M + 1, 0.0);
  for (int m = 1; m < M; ++m) {
    h->lam[m].assign(&lamh[(size_t)m * ga.ld_dsym], &lamh[(size_t)m * ga.ld_dsym] + ne[m]);
    double s = 0;
    for (double l : h->lam[m]) {
      double l2 = l * l;
      if (l2 > 0) s += -std::log1p(-l2) - l2 / (1 - l2) * std::log(l2);
    }
    h->entropy[m] = s;
  }
  double t1 = now_ms();
  h->t_gsvd = t1 - t0;
  // ---- kept bases and maps
  std::vector<CutDesc> cuts(M + 1);
  long off_state = 0, off_occ = 0;
  for (int m = 0; m <= M; ++m) {
    // a single-site build needs the kept bases of the two cuts of its site
    const bool need = only_site == 0 || m == only_site - 1 || m == only_site;
    cuts[m].ne = ne[m];
    cuts[m].chi = ne[m] > 0 && need ? chi : 1;
    cuts[m].off_state = off_state;
    cuts[m].off_occ = off_occ;
    cuts[m].eslot = -1;
    off_state += cuts[m].chi;
    off_occ += (long)cuts[m].chi * ne[m];
  }
  KeptArgs ka{};
  CutDesc* cuts_dev;
  HIP_CHECK_RET(dalloc(tmp, &cuts_dev, M + 1));
  HIP_CHECK_RET(hipMemcpyAsync(cuts_dev, cuts.data(), (M + 1) * sizeof(CutDesc), hipMemcpyHostToDevice, st));
  ka.cuts = cuts_dev;
  ka.lam = ga.lam;
  ka.ld_lam = ga.ld_dsym;
  HIP_CHECK_RET(dalloc(tmp, &ka.E, off_state));
  HIP_CHECK_RET(dalloc(tmp, &ka.parent, off_state));
  HIP_CHECK_RET(dalloc(tmp, &ka.pmode, off_state));
  HIP_CHECK_RET(dalloc(tmp, &ka.ntot, off_state));
  HIP_CHECK_RET(dalloc(tmp, &ka.nocc, off_state));
  HIP_CHECK_RET(dalloc(tmp, &ka.hash, off_state));
  HIP_CHECK_RET(dalloc(h->keep, &ka.occ, std::max(off_occ, 1L)));
  HIP_CHECK_RET(dalloc(tmp, &ka.low, std::max(off_occ, 1L)));
  HIP_CHECK_RET(dalloc(tmp, &ka.olist, (size_t)off_state * GBS_K_MAX));
  HIP_CHECK_RET(dalloc(tmp, &ka.chi_out, M + 1));
  ka.err = err;
  ka.eps_target = opt->eps_target;
  if (kept_workspace_bytes(chi) > kKeptLdsMax) {
    // large chi: the enumeration's heap and sort buffer go to global memory
    ka.gws_stride = (long)kept_workspace_bytes(chi);
    HIP_CHECK_RET(tmp.alloc((void**)&ka.gws, (size_t)(M + 1) * ka.gws_stride));
  }
  // large bases: the parallel enumeration, one workspace slot per such cut
  {
    int nslot = 0, ne_max = 0;
    for (int m = 0; m <= M; ++m)
      if (cuts[m].ne > 0 && cuts[m].chi >= kKeptParallelMin && cuts[m].ne <= kKeptEnumNeMax &&
          !(opt->flags & GBS_KEPT_HEAP)) {
        cuts[m].eslot = nslot++;
        ne_max = std::max(ne_max, cuts[m].ne);
      }
    if (nslot > 0) {
      ka.ews_ne = ne_max;
      ka.ews_stride = (long)kept_enum_bytes(chi, ne_max);
      HIP_CHECK_RET(tmp.alloc((void**)&ka.ews, (size_t)nslot * ka.ews_stride));
      HIP_CHECK_RET(dalloc(tmp, &ka.enum_done, M + 1));
      HIP_CHECK_RET(hipMemsetAsync(ka.enum_done, 0, (M + 1) * sizeof(int), st));
      HIP_CHECK_RET(hipMemcpyAsync(cuts_dev, cuts.data(), (M + 1) * sizeof(CutDesc), hipMemcpyHostToDevice, st));
    }
  }
  h->occ = ka.occ;
  // vacuum cuts report one state
  {
    std::vector<int> ones(M + 1, 1);
    HIP_CHECK_RET(hipMemcpyAsync(ka.chi_out, ones.data(), (M + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  }
  HIP_CHECK_RET(launch_kept_enum(st, ka, M + 1));
  HIP_CHECK_RET(launch_kept(st, ka, M + 1, chi));
  std::vector<int> kept(M + 1), ntot(off_state);
  std::vector<double> Eh(off_state);
  HIP_CHECK_RET(hipMemcpyAsync(kept.data(), ka.chi_out, (M + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipMemcpyAsync(ntot.data(), ka.ntot, off_state * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipMemcpyAsync(Eh.data(), ka.E, off_state * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipStreamSynchronize(st));
  if (herr) return fail(herr == GBS_DEVERR_KMAX ? GBS_E_INVAL : GBS_E_INTERNAL, deverr_msg(herr));
  for (int m = 0; m <= M; ++m) kept[m] = ne[m] > 0 ? kept[m] : 1;
  h->kept = kept;
  h->occ_off.resize(M + 1);
  for (int m = 0; m <= M; ++m) h->occ_off[m] = cuts[m].off_occ;
  // truncation error per cut: eps_m = 1 - (1/Z) sum_kept exp(-E)
  h->eps.assign(M + 1, 0.0);
  for (int m = 1; m < M; ++m) {
    if (ne[m] == 0 || (only_site && m != only_site - 1 && m != only_site)) continue;
    double logz = 0;
    for (double l : h->lam[m]) logz += -std::log1p(-l * l);
    double acc = 0;
    for (int b = 0; b < kept[m]; ++b) acc += std::exp(-Eh[cuts[m].off_state + b] - logz);
    h->eps[m] = std::max(0.0, 1.0 - acc);
  }
  double t2 = now_ms();
  h->t_kept = t2 - t1;
  // ---- PCO schedule: states of each cut grouped by total photon number
  std::vector<int> perm(off_state);
  std::vector<std::vector<int>> grp_off(M + 1), grp_cnt(M + 1), grp_n(M + 1);
  for (int m = 0; m <= M; ++m) {
    const long o = cuts[m].off_state;
    const int nk = kept[m];
    int nmax = 0;
    for (int b = 0; b < nk; ++b) nmax = std::max(nmax, ntot[o + b]);
    std::vector<int> cnt(nmax + 1, 0);
    for (int b = 0; b < nk; ++b) cnt[ntot[o + b]]++;
    std::vector<int> start(nmax + 2, 0);
    for (int n = 0; n <= nmax; ++n) start[n + 1] = start[n] + cnt[n];
    std::vector<int> pos(start.begin(), start.end() - 1);
    for (int b = 0; b < nk; ++b) perm[o + pos[ntot[o + b]]++] = b;
    for (int n = 0; n <= nmax; ++n)
      if (cnt[n]) {
        grp_off[m].push_back(start[n]);
        grp_cnt[m].push_back(cnt[n]);
        grp_n[m].push_back(n);
      }
  }
  std::vector<SiteDesc> sites(M);
  std::vector<long> t64off(M + 1, 0);
  long ttot = 0;
  for (int m = 1; m <= M; ++m) {
    SiteDesc& s = sites[m - 1];
    s.nl = ne[m - 1];
    s.nr = ne[m];
    s.d = d;
    s.chiL = kept[m - 1];
    s.chiR = kept[m];
    s.off_state_l = cuts[m - 1].off_state;
    s.off_state_r = cuts[m].off_state;
    s.off_occ_l = cuts[m - 1].off_occ;
    s.off_occ_r = cuts[m].off_occ;
    s.off_q = (only_site && m != only_site) ? 0 : (long)(m - 1 - h->q_slot0) * h->q_stride;
    s.off_t = ttot;
    t64off[m] = ttot;
    ttot += (long)s.chiL * d * s.chiR;
  }
  // blocks per level
  std::vector<std::vector<LevelBlock>> lv;
  for (int m = 1; m <= M; ++m) {
    if (only_site && m != only_site) continue;
    for (size_t ia = 0; ia < grp_n[m - 1].size(); ++ia)
      for (size_t ib = 0; ib < grp_n[m].size(); ++ib)
        for (int p = 0; p < d; ++p) {
          int tot = grp_n[m - 1][ia] + p + grp_n[m][ib];
          if (tot == 0 || (tot & 1)) continue;
          int k = tot / 2;
          if ((int)lv.size() <= k) lv.resize(k + 1);
          LevelBlock b;
          b.site = m - 1;
          b.p = p;
          b.a_off = grp_off[m - 1][ia];
          b.a_cnt = grp_cnt[m - 1][ia];
          b.b_off = grp_off[m][ib];
          b.b_cnt = grp_cnt[m][ib];
          b.elem_start = 0;
          lv[k].push_back(b);
        }
  }
  std::vector<LevelBlock> allb;
  std::vector<size_t> lv_first(lv.size() + 1, 0);
  std::vector<long> lv_nelem(lv.size(), 0);
  int64_t updates = 0;
  for (size_t k = 0; k < lv.size(); ++k) {
    lv_first[k] = allb.size();
    long acc = 0;
    for (auto& b : lv[k]) {
      b.elem_start = acc;
      acc += (long)b.a_cnt * b.b_cnt;
      allb.push_back(b);
    }
    lv_nelem[k] = acc;
  }
  lv_first[lv.size()] = allb.size();
  cplx64* T64;
  HIP_CHECK_RET(dalloc((h->flags & GBS_KEEP_RAW) || only_site ? h->keep : tmp, &T64, (size_t)std::max(ttot, 1L)));
  HIP_CHECK_RET(hipMemsetAsync(T64, 0, sizeof(cplx64) * ttot, st));
  PcoArgs pa{};
  SiteDesc* sites_dev;
  int* perm_dev;
  LevelBlock* blk_dev;
  HIP_CHECK_RET(dalloc(tmp, &sites_dev, M));
  HIP_CHECK_RET(dalloc(tmp, &perm_dev, off_state));
  HIP_CHECK_RET(dalloc(tmp, &blk_dev, std::max<size_t>(allb.size(), 1)));
  HIP_CHECK_RET(hipMemcpyAsync(sites_dev, sites.data(), M * sizeof(SiteDesc), hipMemcpyHostToDevice, st));
  HIP_CHECK_RET(hipMemcpyAsync(perm_dev, perm.data(), off_state * sizeof(int), hipMemcpyHostToDevice, st));
  if (!allb.empty())
    HIP_CHECK_RET(hipMemcpyAsync(blk_dev, allb.data(), allb.size() * sizeof(LevelBlock), hipMemcpyHostToDevice, st));
  pa.sites = sites_dev;
  pa.perm = perm_dev;
  pa.olist = ka.olist;
  pa.nocc = ka.nocc;
  pa.low = ka.low;
  pa.Q = h->Q;
  pa.ld_q = h->ld_q;
  pa.T = T64;
  unsigned long long* terms_dev;
  HIP_CHECK_RET(dalloc(tmp, &terms_dev, 1));
  HIP_CHECK_RET(hipMemsetAsync(terms_dev, 0, sizeof(unsigned long long), st));
  pa.terms = terms_dev;
  HIP_CHECK_RET(launch_pco_init(st, pa, M));
  hipEvent_t ev[2];
  HIP_CHECK_RET(hipEventCreate(&ev[0]));
  HIP_CHECK_RET(hipEventCreate(&ev[1]));
  HIP_CHECK_RET(hipEventRecord(ev[0], st));
  for (size_t k = 1; k < lv.size(); ++k) {
    int nb = (int)(lv_first[k + 1] - lv_first[k]);
    if (nb == 0) continue;
    HIP_CHECK_RET(launch_pco_level(st, pa, blk_dev + lv_first[k], nb, lv_nelem[k], (int)k));
    updates += lv_nelem[k];
  }
  HIP_CHECK_RET(hipEventRecord(ev[1], st));
  h->pco_updates = updates;
  unsigned long long terms_h = 0;
  HIP_CHECK_RET(hipMemcpyAsync(&terms_h, terms_dev, sizeof terms_h, hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipEventSynchronize(ev[1]));
  {
    float ms = 0.f;
    HIP_CHECK_RET(hipEventElapsedTime(&ms, ev[0], ev[1]));
    h->t_pco_kernels = ms;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if ((h->flags & GBS_KEEP_RAW) || only_site) {
    h->raw = T64;
    h->raw_off = t64off;
  }
  {
    // the pair matrices move to compact storage that lives with the handle
    std::vector<int> qs, qn;
    std::vector<long> qo;
    long qtot = 0;
    h->qc_off.assign(M + 1, -1);
    for (int m = 1; m <= M; ++m) {
      if (only_site && m != only_site) continue;
      const int n = ne[m - 1] + 1 + ne[m];
      qs.push_back(m);
      qn.push_back(n);
      qo.push_back(qtot);
      h->qc_off[m] = qtot;
      qtot += (long)n * n;
    }
    int *qs_d, *qn_d;
    long* qo_d;
    HIP_CHECK_RET(dalloc(h->keep, &h->Qc, (size_t)std::max(qtot, 1L)));
    HIP_CHECK_RET(dalloc(tmp, &qs_d, qs.size()));
    HIP_CHECK_RET(dalloc(tmp, &qn_d, qn.size()));
    HIP_CHECK_RET(dalloc(tmp, &qo_d, qo.size()));
    HIP_CHECK_RET(hipMemcpyAsync(qs_d, qs.data(), qs.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_CHECK_RET(hipMemcpyAsync(qn_d, qn.data(), qn.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_CHECK_RET(hipMemcpyAsync(qo_d, qo.data(), qo.size() * sizeof(long), hipMemcpyHostToDevice, st));
    HIP_CHECK_RET(launch_q_compact(st, h->Q, h->q_stride, h->ld_q, h->q_slot0, qs_d, qn_d, qo_d, (int)qs.size(),
                                   h->Qc));
  }
  HIP_CHECK_RET(hipStreamSynchronize(st));
  h->pco_terms = (int64_t)terms_h;
  h->Q = nullptr;  // the strided buffer goes with the build's scratch arena
  double t3 = now_ms();
  h->t_pco = t3 - t2;
  if (only_site) {
    // the raw PCO tensor of one site: no truncation sweep or normalisation
    h->single_site = only_site;
    h->bond = kept;
    h->maxbond = *std::max_element(kept.begin(), kept.end());
    return GBS_OK;
  }
  // ---- truncation sweep and canonical form
  // (served builds, whose keep arena is stream ordered, stay on their own
  // stream: concurrent slots already share the device's hardware queues)
  MaskJob mj;
  if (h->prec != GBS_FP64 && !h->keep.ordered) HIP_CHECK_RET(side_stream(&mj.side));
  int rc = (h->prec == GBS_FP64) ? canonicalize<cplx64>(h, st, tmp, T64, t64off, nullptr)
                                 : canonicalize<cplx32>(h, st, tmp, T64, t64off, &mj);
  if (rc) return rc;
  if (h->prec != GBS_FP64 && h->maxbond <= 2 * kSamplerMaxSector && d <= kSamplerMaxOutcomes) {
    // Photon-parity sector of every bond index, read off the site tensors
    // (a zero-mean Gaussian state has definite total photon parity, so the
    // canonical tensors are block sparse); any tensor that breaks the
    // structure sends the sampler to the dense layout.
    const int mb = h->maxbond;
    bool split = !(h->flags & GBS_DENSE_SAMPLER);
    std::vector<int32_t> hm((size_t)(M + 1) * mb, 0);
    if (split && mj.launched) {
      // the masks ran beside the norm chain
      HIP_CHECK_RET(hipMemcpyAsync(hm.data(), mj.mask, hm.size() * sizeof(int32_t), hipMemcpyDeviceToHost, mj.side));
      HIP_CHECK_RET(hipStreamSynchronize(mj.side));
    } else if (split) {
      int32_t* mask = nullptr;
      HIP_CHECK_RET(tmp.alloc((void**)&mask, hm.size() * sizeof(int32_t)));
      HIP_CHECK_RET(hipMemsetAsync(mask, 0, hm.size() * sizeof(int32_t), st));
      for (int m = 1; m <= M; ++m)
        HIP_CHECK_RET(launch_sector_mask(st, (const cplx32*)h->tens + h->toff[m], h->bond[m - 1], d, h->bond[m],
                                         m == 1 ? nullptr : mask + (long)(m - 1) * mb, mask + (long)m * mb));
      HIP_CHECK_RET(hipMemcpyAsync(hm.data(), mask, hm.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_CHECK_RET(hipStreamSynchronize(st));
    }
    std::vector<int32_t> maps((size_t)(M + 1) * mb, 0);
    std::vector<int> n0(M + 1, 0), n1(M + 1, 0);
    n0[0] = h->bond[0];
    for (int i = 0; i < h->bond[0]; ++i) maps[i] = i;
    for (int m = 1; m <= M && split; ++m) {
      const int32_t* mk = hm.data() + (size_t)m * mb;
      int32_t* mp = maps.data() + (size_t)m * mb;
      for (int b = 0; b < h->bond[m]; ++b)
        if (mk[b] == 3) split = false;
      for (int b = 0; b < h->bond[m]; ++b)
        if (mk[b] != 2) mp[n0[m]++] = b;  // sector 0, zero columns included
      for (int b = 0; b < h->bond[m]; ++b)
        if (mk[b] == 2) mp[n0[m] + n1[m]++] = b;
      if (sampler_pad(std::max(n0[m], n1[m])) > kSamplerMaxSector) split = false;
    }
    if (split || mb <= kSamplerMaxSector) {
      h->psplit = split;
      if (split) {
        h->secn.resize(2 * (size_t)(M + 1));
        for (int m = 0; m <= M; ++m) {
          h->secn[2 * m] = n0[m];
          h->secn[2 * m + 1] = n1[m];
        }
      }
      int32_t* dmaps = nullptr;
      if (split) {
        HIP_CHECK_RET(dalloc(tmp, &dmaps, maps.size()));
        HIP_CHECK_RET(hipMemcpyAsync(dmaps, maps.data(), maps.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
      }
      h->ssite.assign(M + 1, SamplerSite{});
      h->sgeo.assign(M + 1, SamplerGeom{});
      h->poff.assign(M + 1, 0);
      int widest = 1;
      long tot = 0;
      for (int m = 1; m <= M; ++m) {
        SamplerSite s;
        if (split) {
          s = SamplerSite{{n0[m - 1], n1[m - 1]}, {n0[m], n1[m]}};
          widest = std::max(widest, std::max(std::max(n0[m - 1], n1[m - 1]), std::max(n0[m], n1[m])));
        } else {
          s = SamplerSite{{h->bond[m - 1], 0}, {h->bond[m], h->bond[m]}};
          widest = std::max(widest, std::max(h->bond[m - 1], h->bond[m]));
        }
        h->ssite[m] = s;
        h->poff[m] = tot;
        const long f = sampler_geometry(s, d, &h->sgeo[m]);
        if (f < 0) return fail(GBS_E_INTERNAL, "sampler geometry");  // sizes were checked above
        tot += f;
      }
      h->ldl2 = 2L * sampler_pad(widest);
      HIP_CHECK_RET(dalloc(h->keep, &h->sgeo_dev, (size_t)(M + 1)));
      HIP_CHECK_RET(hipMemcpyAsync(h->sgeo_dev, h->sgeo.data(), (M + 1) * sizeof(SamplerGeom),
                                   hipMemcpyHostToDevice, st));
      HIP_CHECK_RET(dalloc(h->keep, &h->packed, (size_t)tot));
      HIP_CHECK_RET(dalloc(h->keep, &h->poff_dev, (size_t)(M + 1)));
      HIP_CHECK_RET(hipMemcpyAsync(h->poff_dev, h->poff.data(), (M + 1) * sizeof(long), hipMemcpyHostToDevice, st));
      // every site's operand in one launch
      std::vector<SamplerPackDesc> pd(M);
      for (int m = 1; m <= M; ++m)
        pd[m - 1] = SamplerPackDesc{(const cplx32*)h->tens + h->toff[m], h->bond[m - 1], d, h->bond[m], 0,
                                    h->ssite[m], h->sgeo_dev + m, split ? dmaps + (long)(m - 1) * mb : nullptr,
                                    split ? dmaps + (long)m * mb : nullptr, h->packed + h->poff[m]};
      SamplerPackDesc* pd_dev = nullptr;
      HIP_CHECK_RET(dalloc(tmp, &pd_dev, (size_t)M));
      HIP_CHECK_RET(hipMemcpyAsync(pd_dev, pd.data(), M * sizeof(SamplerPackDesc), hipMemcpyHostToDevice, st));
      HIP_CHECK_RET(launch_pack_batch(st, pd.data(), pd_dev, M, h->sgeo.data() + 1));
      HIP_CHECK_RET(hipStreamSynchronize(st));  // pd is read by the copy
    }
  }
  h->t_svd = now_ms() - t3;
  return GBS_OK;
}

}  // namespace

// <psi1|psi2> by the transfer chain E <- sum_p A1[p]^H E A2[p], E_0 = 1, in
// arithmetic C (FP64, FP32 MFMA, or split-BF16x3 on FP32 data).
template <typename C>
int overlap_impl(gbs_mps_s* h1, gbs_mps_s* h2, hipStream_t st, int prec, double* out) {
  const int M = h1->M, d = h1->d;
  const int rmax = std::max(h1->maxbond, h2->maxbond);
  DevArena tmp(st);
  C *E[2], *X, *A1, *A2;
  for (int i = 0; i < 2; ++i) HIP_CHECK_RET(dalloc(tmp, &E[i], (size_t)rmax * rmax));
  HIP_CHECK_RET(dalloc(tmp, &X, (size_t)rmax * d * rmax));
  HIP_CHECK_RET(dalloc(tmp, &A1, (size_t)rmax * d * rmax));
  HIP_CHECK_RET(dalloc(tmp, &A2, (size_t)rmax * d * rmax));
  const long gws_elems = 8L * rmax * rmax;
  C* gws;
  HIP_CHECK_RET(dalloc(tmp, &gws, (size_t)gws_elems));
  auto site = [&](gbs_mps_s* h, int m, C* dst) -> hipError_t {
    long n = (long)h->bond[m - 1] * d * h->bond[m];
    if (h->esz == sizeof(cplx64)) return convert<C, cplx64>(st, dst, (cplx64*)h->tens + h->toff[m], n);
    return convert<C, cplx32>(st, dst, (cplx32*)h->tens + h->toff[m], n);
  };
  auto gemm = [&](int Mr, int Nc, int K, const C* A, long lda, int opA, const C* B, long ldb, C* Cm,
                  long ldc) -> hipError_t {
    if (prec == GBS_BF16X3)
      return zgemm_bf16x3(st, Mr, Nc, K, cone<cplx32>(), (const cplx32*)A, lda, 0, opA, (const cplx32*)B, ldb, 0, 0,
                          czero<cplx32>(), (cplx32*)Cm, ldc, 0, 1, (cplx32*)gws, gws_elems);
    return zgemm<C>(st, Mr, Nc, K, cone<C>(), A, lda, 0, opA, B, ldb, 0, 0, czero<C>(), Cm, ldc, 0, 1, gws,
                    gws_elems);
  };
  const C one = cone<C>();
  HIP_CHECK_RET(hipMemcpyAsync(E[0], &one, sizeof(C), hipMemcpyHostToDevice, st));
  int cur = 0;
  for (int m = 1; m <= M; ++m) {
    const int a1 = h1->bond[m - 1], b1 = h1->bond[m], a2 = h2->bond[m - 1], b2 = h2->bond[m];
    HIP_CHECK_RET(site(h1, m, A1));
    HIP_CHECK_RET(site(h2, m, A2));
    // X = E (a1 x a2) * A2 (a2 x d b2);  E' = A1^H ((a1 d) x b1)^H * X ((a1 d) x b2)
    HIP_CHECK_RET(gemm(a1, d * b2, a2, E[cur], a2, 0, A2, (long)d * b2, X, (long)d * b2));
    HIP_CHECK_RET(gemm(b1, b2, a1 * d, A1, b1, 2, X, b2, E[1 - cur], b2));
    cur = 1 - cur;
  }
  C r;
  HIP_CHECK_RET(hipMemcpyAsync(&r, E[cur], sizeof(C), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipStreamSynchronize(st));
  out[0] = (double)r.re;
  out[1] = (double)r.im;
  return GBS_OK;
}

__attribute__((visibility("hidden"))) int gbs_fail(int code, const std::string& msg) { return fail(code, msg); }

namespace {

// A single-site build of site s past the middle ran on the mode-reversed
// state as site M + 1 - s: number its cuts back (cut m there is cut M - m
// here), transpose its tensor's two bonds, move the Schmidt weights back to
// the bond the forward chain puts them on, and put its pair matrix in the
// mode order (left bond, a_s, right bond) of site s.
int mirror_single_site(gbs_mps_s* h, hipStream_t st) {
  const int M = h->M, d = h->d, sr = h->single_site, s = M + 1 - sr;
  std::reverse(h->ne.begin(), h->ne.end());
  std::reverse(h->kept.begin(), h->kept.end());
  std::reverse(h->bond.begin(), h->bond.end());
  std::reverse(h->eps.begin(), h->eps.end());
  std::reverse(h->entropy.begin(), h->entropy.end());
  std::reverse(h->lam.begin(), h->lam.end());
  std::reverse(h->occ_off.begin(), h->occ_off.end());
  // tensor: kept[s] x d x kept[s-1] in the reversed numbering's bond order
  const long A = h->kept[s], B = h->kept[s - 1];
  cplx64* t;
  HIP_CHECK_RET(dalloc(h->keep, &t, (size_t)std::max(A * d * B, 1L)));
  HIP_CHECK_RET(launch_transpose_bonds(st, h->raw + h->raw_off[sr], A, d, B, t));
  // The reversed chain absorbs each Schmidt weight Lambda_q into the state
  // left of its cut, the forward chain into the state right of it (Eq.
  // SVD3): move them back, element (alpha, p, beta) times
  // prod Lambda_{s-1}^alpha / prod Lambda_s^beta = exp(-E_alpha/2 + E_beta/2)
  // with the entanglement energies of the two bond states.
  auto energies = [&](int cut, std::vector<double>& E) -> int {
    const int n = h->kept[cut], ne = h->ne[cut];
    E.assign((size_t)n, 0.0);
    if (ne == 0) return GBS_OK;
    std::vector<short> oc((size_t)n * ne);
    HIP_CHECK_RET(hipMemcpy(oc.data(), h->occ + h->occ_off[cut], oc.size() * sizeof(short), hipMemcpyDeviceToHost));
    std::vector<double> e(ne);
    for (int q = 0; q < ne; ++q) e[q] = -2.0 * std::log(h->lam[cut][q]);
    for (int b = 0; b < n; ++b)
      for (int q = 0; q < ne; ++q) E[b] += oc[(size_t)b * ne + q] * e[q];
    return GBS_OK;
  };
  std::vector<double> wl, wr;
  if (int rc = energies(s - 1, wl)) return rc;
  if (int rc = energies(s, wr)) return rc;
  for (double& x : wl) x = std::exp(x);  // gauge_scale divides row i by sqrt(wl[i]) and
  for (double& x : wr) x = std::exp(x);  // multiplies column j by sqrt(wr[j])
  DevArena wtmp(st);
  double *wl_d, *wr_d;
  HIP_CHECK_RET(dalloc(wtmp, &wl_d, wl.size()));
  HIP_CHECK_RET(dalloc(wtmp, &wr_d, wr.size()));
  HIP_CHECK_RET(hipMemcpyAsync(wl_d, wl.data(), wl.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_CHECK_RET(hipMemcpyAsync(wr_d, wr.data(), wr.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_CHECK_RET(gauge_scale<cplx64>(st, t, (int)B, d, (int)A, wl_d, wr_d));
  HIP_CHECK_RET(hipStreamSynchronize(st));
  h->keep.release(h->raw);
  h->raw = t;
  h->raw_off.assign(M + 1, 0);
  // pair matrix: modes (r', a, l') = (cut s modes, a_s, cut s-1 modes), in
  // place of the mirrored site's (same size)
  const int nr = h->ne[s], nl = h->ne[s - 1], n = nl + 1 + nr;
  const long qoff = h->qc_off[sr];
  if (qoff < 0) return fail(GBS_E_INTERNAL, "mirrored pair matrix missing");
  std::vector<cplx64> qa((size_t)n * n), qb((size_t)n * n);
  HIP_CHECK_RET(hipMemcpy(qa.data(), h->Qc + qoff, qa.size() * sizeof(cplx64), hipMemcpyDeviceToHost));
  auto src = [&](int i) { return i < nl ? nr + 1 + i : (i == nl ? nr : i - nl - 1); };  // new index -> old
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) qb[(size_t)i * n + j] = qa[(size_t)src(i) * n + src(j)];
  HIP_CHECK_RET(hipMemcpy(h->Qc + qoff, qb.data(), qb.size() * sizeof(cplx64), hipMemcpyHostToDevice));
  h->qc_off.assign(M + 1, -1);
  h->qc_off[s] = qoff;
  h->single_site = s;
  return GBS_OK;
}

}  // namespace

__attribute__((visibility("hidden"))) int gbs_build_handle(const double* gamma, int M, const gbs_build_opts* opt, hipStream_t stream, bool ordered_keep,
                     gbs_mps* out, int only_site) {
  if (!out) return fail(GBS_E_INVAL, "out_handle is NULL");
  *out = nullptr;
  if (!gamma || !opt) return fail(GBS_E_INVAL, "NULL gamma or options");
  if (M < 1) return fail(GBS_E_INVAL, "M must be >= 1");
  if (opt->d < 1) return fail(GBS_E_INVAL, "d must be >= 1");
  if (opt->chi < 1 || opt->chi > (only_site ? GBS_CHI_MAX_SITE : GBS_CHI_MAX))
    return fail(GBS_E_INVAL, only_site ? "chi must be in [1, 16384]" : "chi must be in [1, 4096]");
  if (!(opt->dstar > 1.0)) return fail(GBS_E_INVAL, "dstar must be > 1");
  if (!(opt->eps_target >= 0.0 && opt->eps_target < 1.0)) return fail(GBS_E_INVAL, "eps_target must be in [0, 1)");
  if (opt->prec != GBS_FP64 && opt->prec != GBS_FP32 && opt->prec != GBS_BF16X3)
    return fail(GBS_E_INVAL, "unknown precision");
  if (only_site < 0 || only_site > M) return fail(GBS_E_INVAL, "site out of range");
  if (!only_site && (long)opt->chi * opt->d > 2 * GBS_CHI_MAX) return fail(GBS_E_INVAL, "chi * d too large");
  if (opt->chi_build < 0 || opt->chi_build > GBS_CHI_MAX) return fail(GBS_E_INVAL, "chi_build must be in [0, 4096]");
  if (!only_site && (long)opt->chi_build * opt->d > 2 * GBS_CHI_MAX) return fail(GBS_E_INVAL, "chi_build * d too large");
  if (opt->d > 64) return fail(GBS_E_INVAL, "d must be <= 64");
  if (opt->flags & ~(GBS_KEEP_RAW | GBS_DENSE_SAMPLER | GBS_CHAIN_GSVD | GBS_KEPT_HEAP))
    return fail(GBS_E_INVAL, "unknown build flag");
  gbs_mps_s* h = new (std::nothrow) gbs_mps_s();
  if (!h) return fail(GBS_E_NOMEM, "host allocation failed");
  h->M = M;
  h->d = opt->d;
  h->chi = opt->chi;
  h->prec = opt->prec;
  h->dstar = opt->dstar;
  h->flags = opt->flags;
  h->trunc_rel = opt->trunc_rel;
  if (ordered_keep) {
    h->keep.st = stream;
    h->keep.ordered = true;
  }
  // Past the middle a single site is built on the mode-reversed state, where
  // it lies before the middle: its first Gaussian SVD block, 2(s-1) wide in
  // the given order, is then at most M wide.
  const bool mirror = only_site > 0 && M - only_site < only_site - 1;
  int rc;
  try {
    DevArena rev(stream);
    const double* g = gamma;
    if (mirror) {
      double* gr;
      if (rev.alloc((void**)&gr, sizeof(double) * 4 * (size_t)M * M) != hipSuccess)
        rc = fail(GBS_E_NOMEM, "device allocation of the reversed covariance failed");
      else if (launch_reverse_modes(stream, gamma, M, gr) != hipSuccess)
        rc = fail(GBS_E_INTERNAL, "launch of the mode reversal failed");
      else
        rc = GBS_OK;
      g = gr;
    } else {
      rc = GBS_OK;
    }
    if (rc == GBS_OK) rc = build_impl(g, M, opt, stream, h, mirror ? M + 1 - only_site : only_site);
    if (rc == GBS_OK && mirror) rc = mirror_single_site(h, stream);
  } catch (...) {
    rc = fail(GBS_E_INTERNAL, "unexpected host exception");
  }
  if (rc != GBS_OK) {
    (void)hipStreamSynchronize(stream);
    delete h;
    return rc;
  }
  *out = h;
  return GBS_OK;
}

extern "C" {

int gbs_mps_build(const double* gamma, int32_t M, const gbs_build_opts* opt, void* stream, gbs_mps* out) {
  return gbs_build_handle(gamma, M, opt, (hipStream_t)stream, false, out, 0);
}

int gbs_mps_build_site(const double* gamma, int32_t M, const gbs_build_opts* opt, int32_t site, void* stream,
                       gbs_mps* out) {
  if (out) *out = nullptr;
  if (site < 1 || site > M) return fail(GBS_E_INVAL, "site out of range");
  return gbs_build_handle(gamma, M, opt, (hipStream_t)stream, false, out, site);
}


int gbs_mps_amplitude(gbs_mps h, const int32_t* patterns, int64_t B, double* out, void* stream) {
  if (!h) return fail(GBS_E_INVAL, "NULL handle");
  if (h->single_site) return fail(GBS_E_INVAL, "the handle holds one site's tensor only");
  if (B < 0) return fail(GBS_E_INVAL, "B < 0");
  if (B == 0) return GBS_OK;
  if (!patterns || !out) return fail(GBS_E_INVAL, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  int* bad;
  DevArena tmp(st);
  HIP_CHECK_RET(dalloc(tmp, &bad, 1));
  HIP_CHECK_RET(hipMemsetAsync(bad, 0, sizeof(int), st));
  if (h->esz == sizeof(cplx64))
    HIP_CHECK_RET(launch_amplitude<cplx64>(st, (cplx64* const*)h->site_ptrs, h->bond_dev, h->M, h->d, patterns, B, out,
                                           bad, h->maxbond));
  else
    HIP_CHECK_RET(launch_amplitude<cplx32>(st, (cplx32* const*)h->site_ptrs, h->bond_dev, h->M, h->d, patterns, B, out,
                                           bad, h->maxbond));
  int hb = 0;
  HIP_CHECK_RET(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK_RET(hipStreamSynchronize(st));
  if (hb) return fail(GBS_E_INVAL, "pattern entry outside [0, d)");
  return GBS_OK;
}

}  // extern "C"

namespace {

// HIP events around the sampling launches of one call (measurement only).
struct SampleClock {
  std::vector<hipEvent_t> first, rest;  // start / end pairs
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipStream_t st;
  explicit SampleClock(hipStream_t s) : st(s) {}
  ~SampleClock() {
    for (auto e : first) hipEventDestroy(e);
    for (auto e : rest) hipEventDestroy(e);
    if (t0) hipEventDestroy(t0);
    if (t1) hipEventDestroy(t1);
  }
  hipError_t mark(std::vector<hipEvent_t>& v) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    v.push_back(e);
    return hipEventRecord(e, st);
  }
  hipError_t edge(hipEvent_t* e) {
    hipError_t r = hipEventCreate(e);
    if (r != hipSuccess) return r;
    return hipEventRecord(*e, st);
  }
};

double pair_ms(const std::vector<hipEvent_t>& v) {
  double s = 0;
  for (size_t i = 0; i + 1 < v.size(); i += 2) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, v[i], v[i + 1]) == hipSuccess) s += ms;
  }
  return s;
}

int sample_impl(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, void* stream, SampleClock* clk);

}  // namespace

extern "C" {

int gbs_mps_sample(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, void* stream) {
  return sample_impl(h, shots, seed, out, stream, nullptr);
}

int gbs_mps_sample_timed(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, void* stream,
                         gbs_sample_timing_t* t) {
  if (!t) return fail(GBS_E_INVAL, "NULL timing output");
  *t = gbs_sample_timing_t{};
  SampleClock clk((hipStream_t)stream);
  HIP_CHECK_RET(clk.edge(&clk.t0));
  int rc = sample_impl(h, shots, seed, out, stream, &clk);
  if (rc != GBS_OK) return rc;
  HIP_CHECK_RET(clk.edge(&clk.t1));
  HIP_CHECK_RET(hipStreamSynchronize((hipStream_t)stream));
  float ms = 0;
  HIP_CHECK_RET(hipEventElapsedTime(&ms, clk.t0, clk.t1));
  t->total_ms = ms;
  t->first_launches = (int32_t)(clk.first.size() / 2);
  t->rest_launches = (int32_t)(clk.rest.size() / 2);
  t->first_ms = pair_ms(clk.first);
  t->rest_ms = pair_ms(clk.rest);
  return GBS_OK;
}

}  // extern "C"

namespace {

// Device buffers of one sampling call, sized for `chunk` shots per sweep.
struct SampleBufs {
  float* fb[2] = {nullptr, nullptr};  // MFMA sweep: left vectors (ping-pong), unit norm
  int8_t *par = nullptr, *key = nullptr;
  float* cum = nullptr;
  int32_t *perm = nullptr, *cnt = nullptr, *perm2 = nullptr, *cnt2 = nullptr, *bcnt = nullptr;
  void* lbuf[2] = {nullptr, nullptr};  // vector sweep: left vectors (ping-pong)
};

// Source of those buffers: stream-ordered allocations from an arena, or
// consecutive 256-byte aligned pieces of a region the caller provides.  With
// neither (base == nullptr and no arena) it only counts the bytes.
struct SampleAlloc {
  DevArena* ar = nullptr;
  char* base = nullptr;
  size_t cap = 0, used = 0;
  hipError_t get(void** p, size_t n) {
    n = (std::max<size_t>(n, 16) + 255) & ~(size_t)255;
    if (ar) return ar->alloc(p, n);
    if (base && used + n > cap) return hipErrorOutOfMemory;
    *p = base ? base + used : nullptr;
    used += n;
    return hipSuccess;
  }
};

hipError_t sample_buffers(const gbs_mps_s* h, int64_t chunk, SampleAlloc& a, SampleBufs& b) {
  if (h->packed) {
    // MFMA path: left vectors as interleaved floats in sector-local indices,
    // rows padded to 16 complex; parities
    // and their partition (sector layout); key, running sums and the
    // partition of the shots left undecided by a site's first pass
    for (int i = 0; i < 2; ++i) {
      hipError_t e = a.get((void**)&b.fb[i], (size_t)chunk * h->ldl2 * sizeof(float));
      if (e != hipSuccess) return e;
    }
    const size_t permb = (size_t)(chunk + sampler_shots_per_block()) * sizeof(int32_t);
    hipError_t e = hipSuccess;
    if (h->psplit) {
      e = a.get((void**)&b.par, (size_t)chunk);
      if (e == hipSuccess) e = a.get((void**)&b.perm, permb);
      if (e == hipSuccess) e = a.get((void**)&b.cnt, 2 * sizeof(int32_t));
    }
    if (e == hipSuccess) e = a.get((void**)&b.key, (size_t)chunk);
    if (e == hipSuccess) e = a.get((void**)&b.cum, (size_t)chunk * sizeof(float));
    if (e == hipSuccess) e = a.get((void**)&b.perm2, permb);
    if (e == hipSuccess) e = a.get((void**)&b.cnt2, 2 * sizeof(int32_t));
    if (e == hipSuccess) e = a.get((void**)&b.bcnt, (size_t)sampler_partition_ws(chunk) * sizeof(int32_t));
    return e;
  }
  const size_t rowbytes = (size_t)h->maxbond * h->esz;
  for (int i = 0; i < 2; ++i) {
    hipError_t e = a.get(&b.lbuf[i], (size_t)chunk * rowbytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Largest shot count per sweep for this handle: 2^20 on the MFMA path (one
// launch per site for 10^6 shots), 2^18 on the vector path (rows up to 16 KB).
int64_t sample_chunk_max(const gbs_mps_s* h) { return h->packed ? kSampleChunk : kSampleChunkGeneric; }

int sample_checks(gbs_mps h, int64_t shots, int32_t* out) {
  if (!h) return fail(GBS_E_INVAL, "NULL handle");
  if (h->single_site) return fail(GBS_E_INVAL, "the handle holds one site's tensor only");
  if (shots < 0) return fail(GBS_E_INVAL, "shots < 0");
  if (shots > 0 && !out) return fail(GBS_E_INVAL, "NULL output");
  if (h->maxbond > 1024) return fail(GBS_E_INVAL, "sampler supports bond dimension <= 1024");
  return GBS_OK;
}

// The sweep itself, `chunk` shots at a time, on buffers `b`.
int sample_sweep(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, hipStream_t st, SampleClock* clk,
                 int64_t chunk, const SampleBufs& b) {
  const int M = h->M, d = h->d;
  const long ldl = h->maxbond;
  if (h->packed) {
    const long ldl2 = h->ldl2;
    for (int64_t s0 = 0; s0 < shots; s0 += chunk) {
      const int64_t n = std::min(chunk, shots - s0);
      HIP_CHECK_RET(launch_sampler_init(st, b.fb[0], ldl2, h->bond[0], n));
      int cur = 0;
      for (int m = 1; m <= M; ++m) {
        // site 1: every shot starts in sector 0 of the one-dimensional bond
        const bool part = h->psplit && m > 1;
        const bool next = h->psplit && m < M;
        const SamplerGeom& G = h->sgeo[m];
        const bool more = G.npass[0] > 1 || G.npass[1] > 1;
        const float* P = h->packed + h->poff[m];
        // first pass (outcome 0) for every shot
        if (clk) HIP_CHECK_RET(clk->mark(clk->first));
        HIP_CHECK_RET(launch_sample_mfma(st, P, G, h->sgeo_dev + m, b.fb[cur], b.fb[1 - cur], ldl2,
                                         part ? b.perm : nullptr, part ? b.cnt : nullptr, next ? b.par : nullptr,
                                         more ? b.cum : nullptr, more ? b.key : nullptr, 0, 1, s0, n, m, seed, out, M));
        if (clk) HIP_CHECK_RET(clk->mark(clk->first));
        if (more) {
          // the other passes for the shots the first one left undecided
          HIP_CHECK_RET(launch_sampler_partition(st, b.key, n, b.bcnt, b.perm2, b.cnt2, true));
          if (clk) HIP_CHECK_RET(clk->mark(clk->rest));
          HIP_CHECK_RET(launch_sample_mfma(st, P, G, h->sgeo_dev + m, b.fb[cur], b.fb[1 - cur], ldl2, b.perm2,
                                           b.cnt2, next ? b.par : nullptr, b.cum, nullptr, 1, kSamplerMaxOutcomes, s0,
                                           n, m, seed, out, M));
          if (clk) HIP_CHECK_RET(clk->mark(clk->rest));
        }
        if (next) HIP_CHECK_RET(launch_sampler_partition(st, b.par, n, b.bcnt, b.perm, b.cnt, false));
        cur = 1 - cur;
      }
    }
    return GBS_OK;
  }
  for (int64_t s0 = 0; s0 < shots; s0 += chunk) {
    const int64_t n = std::min(chunk, shots - s0);
    int cur = 0;
    if (h->esz == sizeof(cplx64)) {
      HIP_CHECK_RET(launch_fill_first<cplx64>(st, (cplx64*)b.lbuf[0], ldl, n));
      for (int m = 1; m <= M; ++m) {
        const cplx64* Bm = (const cplx64*)h->tens + h->toff[m];
        HIP_CHECK_RET(launch_sample_site<cplx64>(st, Bm, h->bond[m - 1], d, h->bond[m], (const cplx64*)b.lbuf[cur],
                                                 (cplx64*)b.lbuf[1 - cur], ldl, s0, n, m, seed, out, M));
        cur = 1 - cur;
      }
    } else {
      HIP_CHECK_RET(launch_fill_first<cplx32>(st, (cplx32*)b.lbuf[0], ldl, n));
      for (int m = 1; m <= M; ++m) {
        const cplx32* Bm = (const cplx32*)h->tens + h->toff[m];
        HIP_CHECK_RET(launch_sample_site<cplx32>(st, Bm, h->bond[m - 1], d, h->bond[m], (const cplx32*)b.lbuf[cur],
                                                 (cplx32*)b.lbuf[1 - cur], ldl, s0, n, m, seed, out, M));
        cur = 1 - cur;
      }
    }
  }
  return GBS_OK;
}

int sample_impl(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, void* stream, SampleClock* clk) {
  if (int rc = sample_checks(h, shots, out)) return rc;
  if (shots == 0) return GBS_OK;
  hipStream_t st = (hipStream_t)stream;
  HIP_CHECK_RET(ensure_pool(st));
  const int64_t chunk = std::min<int64_t>(shots, sample_chunk_max(h));
  DevArena tmp(st);
  SampleAlloc a;
  a.ar = &tmp;
  SampleBufs b;
  HIP_CHECK_RET(sample_buffers(h, chunk, a, b));
  return sample_sweep(h, shots, seed, out, st, clk, chunk, b);  // temporaries are freed in stream order
}

}  // namespace

// Sampling on a caller-provided device region of `cap` bytes instead of
// stream-ordered allocations: the shots go through in sweeps of the largest
// multiple of 128 shots whose buffers fit the region (at most the usual
// sweep size).  Allocates nothing.
__attribute__((visibility("hidden"))) int gbs_sample_in_region(gbs_mps h, int64_t shots, uint64_t seed,
                                                               int32_t* out, hipStream_t st, void* region,
                                                               size_t cap) {
  if (int rc = sample_checks(h, shots, out)) return rc;
  if (shots == 0) return GBS_OK;
  if (!region) return fail(GBS_E_INVAL, "NULL workspace region");
  const int64_t blk = sampler_shots_per_block();
  auto bytes = [&](int64_t c) {
    SampleAlloc a;  // counting only
    SampleBufs b;
    (void)sample_buffers(h, c, a, b);
    return a.used;
  };
  const int64_t want = std::min<int64_t>(shots, sample_chunk_max(h));
  int64_t chunk = 0;
  if (bytes(want) <= cap) {
    chunk = want;
  } else {
    int64_t lo = 0, hi = want / blk;  // largest multiple of blk that fits
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (bytes(mid * blk) <= cap) lo = mid;
      else hi = mid - 1;
    }
    chunk = lo * blk;
  }
  if (chunk <= 0) {
    char buf[160];
    snprintf(buf, sizeof buf, "workspace of %zu bytes holds fewer than %lld shots of this handle (%zu bytes needed)",
             cap, (long long)std::min<int64_t>(blk, shots), bytes(std::min<int64_t>(blk, shots)));
    return fail(GBS_E_NOMEM, buf);
  }
  SampleAlloc a;
  a.base = (char*)region;
  a.cap = cap;
  SampleBufs b;
  HIP_CHECK_RET(sample_buffers(h, chunk, a, b));
  return sample_sweep(h, shots, seed, out, st, nullptr, chunk, b);
}

// ---- batched sampling of several handles (used by the server)

__attribute__((visibility("hidden"))) bool gbs_batch_supported(gbs_mps h, int64_t shots) {
  return h && !h->single_site && h->packed && h->poff_dev && shots > 0 && shots <= kSampleChunk;
}

__attribute__((visibility("hidden"))) int64_t gbs_batch_bytes(gbs_mps h, int64_t shots) {
  SampleAlloc a;  // counting only
  SampleBufs b;
  (void)sample_buffers(h, shots, a, b);
  return (int64_t)a.used;
}

__attribute__((visibility("hidden"))) int gbs_batch_prepare(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out,
                                                            hipStream_t st, void* region, size_t cap,
                                                            SampleBatchDesc* d) {
  if (!gbs_batch_supported(h, shots) || !out) return fail(GBS_E_INVAL, "request not sampled by the batched sweep");
  SampleAlloc a;
  a.base = (char*)region;
  a.cap = cap;
  SampleBufs b;
  HIP_CHECK_RET(sample_buffers(h, shots, a, b));
  HIP_CHECK_RET(launch_sampler_init(st, b.fb[0], h->ldl2, h->bond[0], shots));
  *d = SampleBatchDesc{};
  d->packed = h->packed;
  d->poff = h->poff_dev;
  d->geo = h->sgeo_dev;
  for (int i = 0; i < 2; ++i) d->fb[i] = b.fb[i];
  d->par = b.par;
  d->perm = b.perm;
  d->cnt = b.cnt;
  d->bcnt = b.bcnt;
  d->out = out;
  d->ldl2 = h->ldl2;
  d->nshots = shots;
  d->k0 = (uint32_t)seed;
  d->k1 = (uint32_t)(seed >> 32);
  d->M = h->M;
  d->site = 1;
  d->psplit = h->psplit ? 1 : 0;
  return GBS_OK;
}

__attribute__((visibility("hidden"))) int gbs_batch_site_nt(gbs_mps h, int site) {
  return sampler_batch_nt(h->sgeo[site]);
}

__attribute__((visibility("hidden"))) int64_t gbs_mps_device_bytes(gbs_mps h) { return h ? h->keep.bytes : 0; }

extern "C" {

int gbs_mps_overlap(gbs_mps h1, gbs_mps h2, double* out, void* stream) {
  return gbs_mps_overlap_prec(h1, h2, GBS_FP64, out, stream);
}

int gbs_mps_overlap_prec(gbs_mps h1, gbs_mps h2, int32_t prec, double* out, void* stream) {
  if (!h1 || !h2 || !out) return fail(GBS_E_INVAL, "NULL argument");
  if (h1->single_site || h2->single_site) return fail(GBS_E_INVAL, "a handle holds one site's tensor only");
  if (h1->M != h2->M || h1->d != h2->d) return fail(GBS_E_INVAL, "overlap needs equal M and d");
  if (prec != GBS_FP64 && prec != GBS_FP32 && prec != GBS_BF16X3) return fail(GBS_E_INVAL, "unknown precision");
  hipStream_t st = (hipStream_t)stream;
  double r[2];
  int rc = prec == GBS_FP64 ? overlap_impl<cplx64>(h1, h2, st, prec, r) : overlap_impl<cplx32>(h1, h2, st, prec, r);
  if (rc != GBS_OK) return rc;
  out[0] = r[0];
  out[1] = r[1];
  return GBS_OK;
}

int gbs_mps_info(gbs_mps h, gbs_mps_info_t* info, int32_t* bond, int32_t* ne, double* eps, double* entropy) {
  if (!h || !info) return fail(GBS_E_INVAL, "NULL argument");
  info->M = h->M;
  info->d = h->d;
  info->chi = h->chi;
  info->prec = h->prec;
  info->max_bond = h->maxbond;
  info->max_ne = *std::max_element(h->ne.begin(), h->ne.end());
  info->eps_max = *std::max_element(h->eps.begin(), h->eps.end());
  info->norm_raw = h->norm_raw;
  info->bytes = h->keep.bytes;
  info->pco_updates = h->pco_updates;
  info->t_gsvd_ms = h->t_gsvd;
  info->t_kept_ms = h->t_kept;
  info->t_pco_ms = h->t_pco;
  info->t_svd_ms = h->t_svd;
  info->eig_sweeps = h->eig_sweeps;
  info->sampler_layout = h->packed ? (h->psplit ? 2 : 1) : 0;
  info->gsvd_mode = h->gsvd_independent;
  info->pco_terms = h->pco_terms;
  info->t_pco_kernel_ms = h->t_pco_kernels;
  for (int m = 0; m <= h->M; ++m) {
    if (bond) bond[m] = h->bond[m];
    if (ne) ne[m] = h->ne[m];
    if (eps) eps[m] = h->eps[m];
    if (entropy) entropy[m] = h->entropy[m];
  }
  return GBS_OK;
}

int gbs_mps_export(gbs_mps h, int32_t m, int32_t what, void* dst, int64_t cap, int64_t* written) {
  if (!h || !dst) return fail(GBS_E_INVAL, "NULL argument");
  const int M = h->M, d = h->d;
  std::vector<char> buf;
  auto put = [&](const void* p, size_t n) -> int {
    if ((int64_t)n > cap) return fail(GBS_E_INVAL, "export buffer too small");
    std::memcpy(dst, p, n);
    if (written) *written = (int64_t)n;
    return GBS_OK;
  };
  if (h->single_site && (what == GBS_EXPORT_TENSOR || what == GBS_EXPORT_SVALS || what == GBS_EXPORT_SECTORS))
    return fail(GBS_E_INVAL, "the handle holds one site's PCO tensor only");
  if (h->single_site && (what == GBS_EXPORT_RAW || what == GBS_EXPORT_Q) && m != h->single_site)
    return fail(GBS_E_INVAL, "the handle holds the tensor of another site");
  if (what == GBS_EXPORT_TENSOR) {
    if (m < 1 || m > M) return fail(GBS_E_INVAL, "site out of range");
    long n = (long)h->bond[m - 1] * d * h->bond[m];
    std::vector<cplx64> out(n);
    if (h->esz == sizeof(cplx64)) {
      HIP_CHECK_RET(hipMemcpy(out.data(), (cplx64*)h->tens + h->toff[m], n * sizeof(cplx64), hipMemcpyDeviceToHost));
    } else {
      std::vector<cplx32> tmp(n);
      HIP_CHECK_RET(hipMemcpy(tmp.data(), (cplx32*)h->tens + h->toff[m], n * sizeof(cplx32), hipMemcpyDeviceToHost));
      for (long i = 0; i < n; ++i) out[i] = cmake<cplx64>(tmp[i].re, tmp[i].im);
    }
    return put(out.data(), n * sizeof(cplx64));
  }
  if (what == GBS_EXPORT_RAW) {
    if (!h->raw) return fail(GBS_E_INVAL, "raw tensors not kept (build with GBS_KEEP_RAW)");
    if (m < 1 || m > M) return fail(GBS_E_INVAL, "site out of range");
    long n = (long)h->kept[m - 1] * d * h->kept[m];
    std::vector<cplx64> out(n);
    HIP_CHECK_RET(hipMemcpy(out.data(), h->raw + h->raw_off[m], n * sizeof(cplx64), hipMemcpyDeviceToHost));
    return put(out.data(), n * sizeof(cplx64));
  }
  if (what == GBS_EXPORT_Q) {
    if (m < 1 || m > M) return fail(GBS_E_INVAL, "site out of range");
    if (h->qc_off.empty() || h->qc_off[m] < 0) return fail(GBS_E_INVAL, "pair matrix of this site not formed");
    int n = h->ne[m - 1] + 1 + h->ne[m];
    std::vector<cplx64> out((size_t)n * n);
    HIP_CHECK_RET(hipMemcpy(out.data(), h->Qc + h->qc_off[m], out.size() * sizeof(cplx64), hipMemcpyDeviceToHost));
    return put(out.data(), out.size() * sizeof(cplx64));
  }
  if (what == GBS_EXPORT_BASIS) {
    if (m < 0 || m > M) return fail(GBS_E_INVAL, "cut out of range");
    long n = (long)h->kept[m] * h->ne[m];
    std::vector<short> tmp(std::max(n, 1L));
    std::vector<int32_t> out(n);
    if (n) HIP_CHECK_RET(hipMemcpy(tmp.data(), h->occ + h->occ_off[m], n * sizeof(short), hipMemcpyDeviceToHost));
    for (long i = 0; i < n; ++i) out[i] = tmp[i];
    if (written) *written = 0;
    return n ? put(out.data(), n * sizeof(int32_t)) : GBS_OK;
  }
  if (what == GBS_EXPORT_LAMBDA) {
    if (m < 1 || m >= M) return fail(GBS_E_INVAL, "cut out of range");
    if (written) *written = 0;
    return h->lam[m].empty() ? GBS_OK : put(h->lam[m].data(), h->lam[m].size() * sizeof(double));
  }
  if (what == GBS_EXPORT_SVALS) {
    if (m < 1 || m >= M) return fail(GBS_E_INVAL, "bond out of range");
    return put(h->svals[m].data(), h->svals[m].size() * sizeof(double));
  }
  if (what == GBS_EXPORT_SECTORS) {
    std::vector<int32_t> out(2 * (size_t)(M + 1), 0);
    if (h->psplit) out = h->secn;
    return put(out.data(), out.size() * sizeof(int32_t));
  }
  return fail(GBS_E_INVAL, "unknown export kind");
}

int gbs_mps_export_elements(gbs_mps h, int32_t m, int32_t what, const int64_t* idx, int64_t n, double* out) {
  if (!h || (n > 0 && (!idx || !out))) return fail(GBS_E_INVAL, "NULL argument");
  if (n < 0) return fail(GBS_E_INVAL, "n < 0");
  if (what != GBS_EXPORT_TENSOR && what != GBS_EXPORT_RAW) return fail(GBS_E_INVAL, "elements of TENSOR or RAW only");
  if (m < 1 || m > h->M) return fail(GBS_E_INVAL, "site out of range");
  if (what == GBS_EXPORT_TENSOR && h->single_site) return fail(GBS_E_INVAL, "the handle holds one site's PCO tensor only");
  if (what == GBS_EXPORT_RAW && !h->raw) return fail(GBS_E_INVAL, "raw tensors not kept (build with GBS_KEEP_RAW)");
  if (what == GBS_EXPORT_RAW && h->single_site && m != h->single_site)
    return fail(GBS_E_INVAL, "the handle holds the tensor of another site");
  const int d = h->d;
  const long a = what == GBS_EXPORT_RAW ? h->kept[m - 1] : h->bond[m - 1];
  const long b = what == GBS_EXPORT_RAW ? h->kept[m] : h->bond[m];
  for (int64_t k = 0; k < n; ++k) {
    const int64_t i = idx[3 * k], p = idx[3 * k + 1], j = idx[3 * k + 2];
    if (i < 0 || i >= a || p < 0 || p >= d || j < 0 || j >= b) return fail(GBS_E_INVAL, "element index out of range");
    const long e = (i * d + p) * b + j;
    if (what == GBS_EXPORT_RAW || h->esz == sizeof(cplx64)) {
      const cplx64* src = what == GBS_EXPORT_RAW ? h->raw + h->raw_off[m] : (const cplx64*)h->tens + h->toff[m];
      cplx64 v;
      HIP_CHECK_RET(hipMemcpy(&v, src + e, sizeof v, hipMemcpyDeviceToHost));
      out[2 * k] = v.re;
      out[2 * k + 1] = v.im;
    } else {
      cplx32 v;
      HIP_CHECK_RET(hipMemcpy(&v, (const cplx32*)h->tens + h->toff[m] + e, sizeof v, hipMemcpyDeviceToHost));
      out[2 * k] = v.re;
      out[2 * k + 1] = v.im;
    }
  }
  return GBS_OK;
}

void gbs_mps_free(gbs_mps h) {
  if (!h) return;
  delete h;
}

// Upper estimate of the device bytes one build (plus one sampling call of
// `shots`) holds at its peak: every buffer is sized from M, d and chi alone.
int64_t gbs_mps_footprint(int32_t M, const gbs_build_opts* opt, int64_t shots) {
  if (!opt || M < 1 || opt->d < 1 || opt->chi < 1) return -1;
  if (opt->chi_build < 0) return -1;
  const int64_t d = opt->d, chi = std::min<int64_t>(std::max(opt->chi, opt->chi_build), GBS_CHI_MAX), m = M;
  const int64_t esz = opt->prec == GBS_FP64 ? 16 : 8;
  const int64_t n2 = std::min<int64_t>(m + 2, GBS_GSVD_N2_MAX);
  int64_t b = 0;
  // Gaussian SVD chain: residual blocks, stage workspaces, the strided Q^m
  // of the build (n2^2 each), and the compact copy kept with the handle
  b += 2 * (n2 * n2 + n2 * 2 * m) * 8 + 10 * n2 * n2 * 8 + (2 * n2 * n2 + 4 * n2) * 8;
  b += m * n2 * n2 * 16 + m * (n2 / 2 + 2) * (n2 / 2 + 2) * 16 * 4;
  // every site on its own (2 (M - 1) <= 600): per-site pools of doubles
  if (m >= 3 && 2 * (m - 1) <= GBS_GSVD_N2_MAX && !(opt->flags & GBS_CHAIN_GSVD)) {
    int64_t pool = 0;
    for (int64_t k = 1; k <= m; ++k) {
      const int64_t w = 2 * k, lu = k + 1;
      pool += 2 * (m + 1) * lu + 13 * w * w + 3 * w * 2 * m + 8 * w + w * (w + 1) / 2 + 8 * lu * lu + 23 * 32;
    }
    b += pool * 8;
  }
  // kept bases and maps
  b += (m + 1) * chi * (40 + 16 * GBS_K_MAX + 6 * (n2 / 2 + 1));
  if (chi >= kKeptParallelMin && !(opt->flags & GBS_KEPT_HEAP))
    b += (m + 1) * (int64_t)kept_enum_bytes((int)chi, (int)std::min<int64_t>(n2 / 2, kKeptEnumNeMax));
  // PCO tensors (FP64) and the truncation sweep
  const int64_t site = d * chi * chi;
  const int64_t chld = chi * d + 1;
  b += m * site * 16;
  b += 5 * chld * chld * 16 + chld * chld * d * 16;
  b += 3 * (m + 1) * chi * chi * 16 + 3 * site * 16;
  b += (int64_t)jacobi_blocked_ws_elems((int)chi, (int)std::max<int64_t>(m - 1, 1)) * 16 + 16 * m;
  b += m * site * esz + (m + 1) * chi * chi * esz + 2 * site * esz;
  const int64_t pad = (chi + 15) / 16 * 16;
  // sampler operand: sector blocks pad at most 16 rows and columns each
  if (opt->prec != GBS_FP64 && chi <= 512) b += m * 16 * d * (pad + 16) * (pad + 16) + (m + 1) * chi * 8;
  // sampling buffers: rows, scales, parities, running sums and partitions
  const bool mfma = opt->prec != GBS_FP64 && chi <= 512 && d <= 32;
  const int64_t chunk = std::min<int64_t>(std::max<int64_t>(shots, 0), mfma ? kSampleChunk : kSampleChunkGeneric);
  b += 2 * chunk * std::max<int64_t>(chi * esz, 8 * pad) + 32 * chunk + 4096;
  return b + b / 8 + (64LL << 20);
}

const char* gbs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
