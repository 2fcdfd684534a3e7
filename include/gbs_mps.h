/* gbs_mps.h -- C ABI of the MI355X Gaussian-state -> MPS library.
 *
 * Converts a pure M-mode bosonic Gaussian state, given by its covariance
 * matrix, into a matrix product state with photon cutoff d and bond
 * dimension chi, following arXiv 2512.10643 (Liu, Jin, Xiang, Tu):
 * per-cut Gaussian SVD (Sec. II.B), kept virtual bases by entanglement
 * energy (Sec. II.C.1), local tensors by projected creation operators
 * (Sec. II.C.2, App. B), then SVD truncation / canonicalisation, and the MPS
 * consumers: amplitudes and photon-number samples (Sec. I, Sec. III).
 *
 * Conventions
 *   - All array arguments are DEVICE pointers on the current HIP device
 *     unless marked "host".  `stream` is a hipStream_t (may be NULL for the
 *     default stream).
 *   - Matrices are row-major.  Complex outputs are interleaved (re, im).
 *   - Return value: GBS_OK (0) or a negative GBS_E_* code; the library never
 *     aborts and never throws across this boundary.  gbs_last_error() gives a
 *     thread-local message for the last failure.
 *   - Thread safety: distinct handles may be used concurrently; one handle
 *     is read-only after gbs_mps_build and may serve concurrent
 *     amplitude/sample calls on different streams.
 */
#ifndef GBS_MPS_H
#define GBS_MPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gbs_mps_s* gbs_mps;

enum {
  GBS_OK = 0,
  GBS_E_INVAL = -1,     /* bad argument: M<1, d<1, chi<1 or > 4096, dstar<=1, NULL pointer, pattern outside [0,d) */
  GBS_E_NOT_PD = -2,    /* Gamma not symmetric positive definite (Sec. II.A) */
  GBS_E_NOT_PURE = -3,  /* Gamma is not the covariance of a pure state: (2 Gamma Omega)^2 != -1 */
  GBS_E_NOMEM = -4,     /* device allocation failed or footprint above budget */
  GBS_E_DEVICE = -5,    /* HIP runtime error */
  GBS_E_BUSY = -6,      /* serving queue full */
  GBS_E_INTERNAL = -7   /* numerical failure (Jacobi non-convergence, index map) */
};

typedef enum {
  GBS_FP64 = 0,   /* complex FP64 tensors and contractions */
  GBS_FP32 = 1,   /* complex FP32 tensors and contractions; FP64 Gaussian SVD and singular values */
  GBS_BF16X3 = 2  /* FP32 tensors; bond contractions by split-BF16x3 compensated products */
} gbs_precision;

/* Build options.  d: photon cutoff (p <= d-1 per mode, Sec. II.C.1);
 * chi: bond dimension D (Sec. II.C, Eq. Am_definition); dstar: frozen-mode
 * tolerance D* > 1 (Sec. II.A; modes with symplectic eigenvalue below it are
 * treated as unentangled); trunc_rel: singular values below
 * trunc_rel * sigma_max are dropped by the truncation sweep (0 selects the
 * default, 1e-12 for FP64 and 1e-8 for FP32 builds); flags: GBS_KEEP_RAW keeps
 * the PCO tensors for gbs_mps_export; GBS_DENSE_SAMPLER makes the FP32
 * sampler use whole bonds instead of photon-parity sectors (the sectors need
 * the parity structure a zero-mean state has, and are checked on the built
 * tensors; the dense layout is also taken when that check fails).
 * eps_target > 0 picks the bond dimension per cut (Sec. II.C.2, D(eps)):
 * each cut keeps the fewest lowest-energy states whose discarded weight
 * eps_m = 1 - (1/Z) sum_kept exp(-E) is at most eps_target, and at most chi
 * of them; the truncation sweep then acts on those bonds as usual.
 * chi_build > chi (full builds): the kept bases and PCO tensors are built at
 * chi_build states per cut (D_build; eps_target then caps at chi_build) and
 * the truncation sweep recompresses every bond to at most chi singular
 * directions, a global truncation in place of the local analytic one
 * (Sec. II.C.1); 0 or <= chi: D_build = chi.  chi_build <= 4096 and
 * chi_build * d <= 8192; single-site builds do not use it.
 * Gaussian SVD: when every site's first block fits one workgroup
 * (2 (M - 1) <= 600), each site's Gaussian data is computed on its own, all
 * sites at once (Sec. III.A): site m starts at cut m - 1 straight from Gamma
 * and takes one chain step to cut m; the two neighbours of a cut then agree
 * on its Bogoliubov modes up to a phase per mode, which is read off their
 * b-mode maps and put into Q^m.  A build with a bond mode weaker than
 * Lambda = 1e-3 (D - 1 < 2e-6, whose phase the two sides cannot align to
 * FP64 accuracy) reruns as the chain, as does one whose two sides of a cut
 * count different modes.  GBS_CHAIN_GSVD forces the sequential chain (cut
 * after cut, Sec. II.B), which larger M always take; gsvd_mode in
 * gbs_mps_info_t tells which ran. */
#define GBS_KEEP_RAW 1u
#define GBS_DENSE_SAMPLER 2u
#define GBS_CHAIN_GSVD 4u
/* GBS_KEPT_HEAP: enumerate every kept basis with the sequential best-first
 * heap.  Bases of D >= 256 states are otherwise enumerated in parallel
 * (threshold search on the entanglement energy, then a sort by the same
 * key), which gives the heap's basis and order exactly; the flag is there
 * to compare the two. */
#define GBS_KEPT_HEAP 8u
typedef struct {
  int32_t d;
  int32_t chi;
  double dstar;
  int32_t prec;      /* gbs_precision */
  uint32_t flags;
  double trunc_rel;
  double eps_target;  /* > 0: D(eps) per cut, see below; 0: chi states at every cut */
  int32_t chi_build;  /* > chi: kept states per cut before the recompression to chi */
} gbs_build_opts;

/* Build the MPS of the pure state with covariance `gamma`.
 *   gamma : device, 2M x 2M FP64, row-major, quadratures ordered
 *           (x_1..x_M, p_1..p_M), vacuum = identity/2 (Sec. II.A, Eq. GammaMat;
 *           App. A, Gamma = M M^T / 2).  Read during the call only.
 *   opt   : host pointer to options.
 *   out   : host pointer receiving the handle (NULL on failure).
 * Validates Gamma (symmetric, positive definite, pure), runs the Gaussian SVD
 * chain (Sec. II.B.2), the kept-basis selection (Sec. II.C.1), the PCO
 * tensor construction (Sec. II.C.2) and the truncation sweep, and leaves a
 * right-canonical, unit-norm MPS whose vacuum amplitude is real > 0.
 * Synchronises `stream` internally (buffer sizes depend on the spectra).
 * A cut with more than 299 entangled mode pairs (2 (n_e + 1) > 600, the
 * widest Williamson step one workgroup takes) fails with GBS_E_INVAL. */
int gbs_mps_build(const double* gamma, int32_t M, const gbs_build_opts* opt, void* stream, gbs_mps* out);

/* The tensor of one site alone, at bond dimension chi <= 16384: the shape of
 * the paper's own benchmark, a central tensor at large D (Sec. III.A).  Runs
 * the Gaussian SVD of cuts site-1 and site alone: the chain starts at cut
 * site-1 straight from Gamma's block on modes 1..site-1, which stand in for
 * the bond modes of the cut before (from cut 300 when site > 301, the
 * widest block one workgroup takes), so each tensor is built on its own.
 * Past the middle (M - site < site - 1) the site is built as site
 * M + 1 - site of the mode-reversed state and its bonds are transposed, so
 * the first block is never wider than the middle one.
 * Then the kept bases of the two cuts and the PCO build of that tensor (Eq.
 * Am_definition, Sec. II.C.2), in FP64, with no truncation sweep or
 * normalisation.  The tensor's bond bases are those of this build: they
 * equal a full build's up to a phase per bond mode and photon (for a site
 * past the middle the Schmidt weights Lambda_q, which the reversed chain
 * puts on the other bond, are moved back: element (alpha, p, beta) times
 * prod Lambda_{site-1}^alpha / prod Lambda_site^beta).  The handle holds the
 * raw tensor (gbs_mps_export GBS_EXPORT_RAW at `site`, kept[site-1] x d x
 * kept[site]), its pair matrix (GBS_EXPORT_Q at `site`, modes in the order
 * left bond, a_site, right bond), the Gaussian data and kept bases of the
 * two cuts; exports of other sites fail with GBS_E_INVAL;
 * amplitude, sample and overlap calls on it fail with GBS_E_INVAL.
 *   gamma, M, opt, stream, out : as gbs_mps_build (opt->prec and
 *   opt->trunc_rel are not used; the chi * d limit of full builds does not
 *   apply, d <= 64; a kept state may occupy at most 12 distinct modes,
 *   GBS_E_INVAL otherwise);  site : 1..M (GBS_E_INVAL otherwise).
 * The tensor takes kept[site-1] * d * kept[site] * 16 bytes of device
 * memory (16 GB at chi = 10^4, d = 10). */
int gbs_mps_build_site(const double* gamma, int32_t M, const gbs_build_opts* opt, int32_t site, void* stream,
                       gbs_mps* out);

/* Amplitudes <n|psi> of the normalised MPS for B occupation patterns.
 *   patterns : device, B x M int32, 0 <= n < d.
 *   out      : device, B x 2 FP64 (re, im).
 * Synchronises `stream` to report invalid patterns (GBS_E_INVAL; their
 * outputs are NaN). */
int gbs_mps_amplitude(gbs_mps h, const int32_t* patterns, int64_t B, double* out, void* stream);

/* Draw `shots` photon-number samples by sequential conditional sampling on
 * the right-canonical MPS (the "standard MPS sampling" the paper defers to,
 * Sec. I).  At site m shot s draws one uniform u from Philox-4x32-10 keyed by
 * `seed` (low word, high word), counter (s low word, s high word, m, 0),
 * first output word, top 24 bits / 2^24; it takes the first photon number p
 * = 0, 1, ... whose cumulative conditional probability exceeds u.  The left
 * vector enters each site with unit norm and the tensors are right-
 * canonical, so the cumulative sum reaches 1 up to rounding; a u above the
 * rounded total takes the last p of positive probability.  Results do not
 * depend on batching.
 *   out : device, shots x M int32.  Asynchronous on `stream`. */
int gbs_mps_sample(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, void* stream);

/* gbs_mps_sample for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, samples and errors as gbs_mps_sample (bit-identical
 * output), but the sweep's buffers (left vectors, parities, running
 * sums, shot partitions) come from one static device array of
 * GBS_SAMPLE_NOALLOC_SCRATCH_BYTES that each GPU holds for the life of the
 * process, so the call makes no hipMalloc, hipFree or allocating library
 * call.  The shots go through in sweeps of the largest multiple of 128 shots
 * whose buffers fit the array (about 80 000 at a 256-wide bond, whole 10^6
 * sweeps never); a handle whose 128-shot sweep does not fit is rejected with
 * GBS_E_NOMEM.  Every call on one GPU uses that GPU's one array: calls that
 * overlap on the same GPU (other streams or host threads) race and must be
 * serialised by the caller.  The array keeps the last call's contents; each
 * call writes every buffer before reading it.  Asynchronous on `stream`. */
#define GBS_SAMPLE_NOALLOC_SCRATCH_BYTES (256ll << 20)
int gbs_mps_sample_noalloc(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, void* stream);

/* GPU time of the launches of one sampling call (HIP events on its stream). */
typedef struct {
  int32_t first_launches;  /* first-pass launches: outcome 0 for every shot, one per site */
  int32_t rest_launches;   /* launches for the shots a first pass left undecided */
  double first_ms;         /* summed time of the first-pass launches */
  double rest_ms;          /* summed time of the other launches */
  double total_ms;         /* the whole call, first launch to last */
} gbs_sample_timing_t;

/* gbs_mps_sample with HIP events recorded on `stream` around each launch of
 * the MFMA sampling sweep (FP32 and BF16x3 handles), for measurement: same
 * samples, plus the launch counts and times in `t` (host).  Synchronises
 * `stream` before returning.  Handles sampled by the vector sweep (FP64)
 * report zero launches and only total_ms.  Errors as gbs_mps_sample; a NULL
 * `t` is GBS_E_INVAL. */
int gbs_mps_sample_timed(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, void* stream,
                         gbs_sample_timing_t* t);

/* Overlap <psi1|psi2> of two MPS over the same M and d, by an FP64 transfer
 * contraction on the GPU (E <- sum_p A1[p]^dag E A2[p]).  The wavefunction
 * fidelity used to compare builds (Sec. III.A) is
 * |<psi1|psi2>|^2 / (<psi1|psi1> <psi2|psi2>), three calls of this function.
 *   out : host, 2 FP64 (re, im).  Synchronises `stream`. */
int gbs_mps_overlap(gbs_mps h1, gbs_mps h2, double* out, void* stream);

/* The same transfer contraction in a chosen arithmetic: GBS_FP64, GBS_FP32
 * (tensors rounded to FP32, FP32 matrix cores) or GBS_BF16X3 (FP32 tensors,
 * split-BF16x3 products on the BF16 matrix cores).  Used to compare the cost
 * and error of bond contractions by precision.  out: host, 2 FP64. */
int gbs_mps_overlap_prec(gbs_mps h1, gbs_mps h2, int32_t prec, double* out, void* stream);

/* Scalar information about a handle (host struct). */
typedef struct {
  int32_t M, d, chi, prec;
  int32_t max_bond;        /* largest bond dimension after truncation */
  int32_t max_ne;          /* largest number of entangled mode pairs at a cut */
  double eps_max;          /* max over cuts of the discarded weight eps_m (Sec. III.A) */
  double norm_raw;         /* norm of the MPS before normalisation */
  int64_t bytes;           /* device bytes held by the handle */
  int64_t pco_updates;     /* tensor elements produced by the PCO level gather */
  double t_gsvd_ms, t_kept_ms, t_pco_ms, t_svd_ms;  /* build phase times */
  int32_t eig_sweeps;      /* sweeps of the bond eigensolver in the truncation step */
  int32_t sampler_layout;  /* FP32 sampling operand: 0 none (FP64 builds, or a bond the
                              MFMA sampler cannot take), 1 dense, 2 photon-parity sectors */
  int32_t gsvd_mode;       /* 0: sequential Gaussian SVD chain; 1: every site's Gaussian data on its
                              own, bond modes aligned between neighbours (Sec. III.A) */
  int64_t pco_terms;       /* source terms the PCO level gather summed (pairs of occupied modes
                              over all elements: the sparse update count of Sec. II.C.2) */
  double t_pco_kernel_ms;  /* device time of the PCO level launches (HIP events, back to back) */
} gbs_mps_info_t;

/* Fill `info`; optional host arrays (may be NULL):
 *   bond  : M+1 int32, bond dimensions after truncation (bond[0] = bond[M] = 1);
 *   ne    : M+1 int32, entangled pairs n_e^m per cut (ne[0] = ne[M] = 0);
 *   eps   : M+1 FP64, discarded weight per cut (Sec. III.A);
 *   entropy: M+1 FP64, entanglement entropy per cut (Sec. II.A). */
int gbs_mps_info(gbs_mps h, gbs_mps_info_t* info, int32_t* bond, int32_t* ne, double* eps, double* entropy);

/* Copy diagnostic data to host memory (tests).  what:
 *   GBS_EXPORT_TENSOR : canonical tensor of site m (1-based), complex FP64,
 *                       bond[m-1] x d x bond[m];
 *   GBS_EXPORT_RAW    : PCO tensor of site m before truncation, complex FP64,
 *                       kept[m-1] x d x kept[m] (needs GBS_KEEP_RAW);
 *   GBS_EXPORT_Q      : pair matrix Q^m of site m, complex FP64, n x n with
 *                       n = ne[m-1] + 1 + ne[m];
 *   GBS_EXPORT_BASIS  : kept basis of cut m (0..M), int32 kept[m] x ne[m];
 *   GBS_EXPORT_LAMBDA : Lambda_q of cut m (1..M-1), FP64, ne[m] values;
 *   GBS_EXPORT_SVALS  : singular values of bond m after truncation, FP64;
 *   GBS_EXPORT_SECTORS: sizes of the two photon-parity sectors of every bond,
 *                       int32 (M+1) x 2 (m is ignored; zeros unless
 *                       sampler_layout is 2).
 * `dst` is a host buffer of `cap` bytes; the number of bytes written is
 * returned through *written (host, may be NULL). */
enum { GBS_EXPORT_TENSOR = 0, GBS_EXPORT_RAW = 1, GBS_EXPORT_Q = 2, GBS_EXPORT_BASIS = 3, GBS_EXPORT_LAMBDA = 4,
       GBS_EXPORT_SVALS = 5, GBS_EXPORT_SECTORS = 6 };
int gbs_mps_export(gbs_mps h, int32_t m, int32_t what, void* dst, int64_t cap, int64_t* written);

/* Selected elements of the tensor of site m (tests of tensors too large to
 * export whole, e.g. a 16 GB single-site tensor).  what: GBS_EXPORT_TENSOR
 * (canonical tensor, bond[m-1] x d x bond[m]) or GBS_EXPORT_RAW (PCO tensor,
 * kept[m-1] x d x kept[m]).  idx: host, n x 3 int64 (alpha, p, beta);
 * out: host, n x 2 FP64 (re, im).  GBS_E_INVAL for an index out of range. */
int gbs_mps_export_elements(gbs_mps h, int32_t m, int32_t what, const int64_t* idx, int64_t n, double* out);

/* Release every device buffer of the handle. NULL is ignored. */
void gbs_mps_free(gbs_mps h);

/* Upper estimate of the device bytes that one gbs_mps_build with these
 * options, followed by one gbs_mps_sample of `shots`, holds at its peak
 * (buffers sized from M, d and chi alone).  Returns -1 for invalid options.
 * Used for admission control by the server below. */
int64_t gbs_mps_footprint(int32_t M, const gbs_build_opts* opt, int64_t shots);

/* ---- Mixed -> pure filtration (Sec. III, Eq. decompose; App. C) ---------
 * A measured covariance Gamma_th describes a mixed state; the conversion
 * needs a pure one.  Gamma_th = Gamma_p + W with Gamma_p = S S^T / 2 pure
 * (S symplectic) and W >= 0 classical noise; the wanted split has the
 * fewest squeezed photons.  Following App. C: start at S = 1 and descend the
 * loss L(S) = -lambda_min(Gamma_th - S S^T / 2) (Eq. loss) along the
 * Riemannian gradient on Sp(2N) (the unit-norm element of the Lie algebra
 * that maximises the directional derivative, for the Frobenius norm), with
 * the exponential map as retraction, until L <= eps.  The step is the Newton
 * step of the loss along the gradient, capped at alpha_max (the paper leaves
 * the step size open).  FP64 throughout. */
#define GBS_FILTER_MODES_MAX 288
typedef struct {
  double eps;        /* stop when L <= eps; 0 selects 1e-12 */
  double alpha_max;  /* largest step along the unit gradient; 0 selects 0.5 */
  int32_t max_iter;  /* step budget; 0 selects 100000 */
} gbs_filter_opts;

typedef struct {
  int32_t iterations;  /* retraction steps taken */
  int32_t converged;   /* 1 when L <= eps was reached within max_iter */
  double loss;         /* L at the returned S */
  double n_eff;        /* mean photon number of Gamma_p, tr(Gamma_p)/2 - N/2 (vacuum = 1/2) */
  double ms;           /* wall time of the call */
} gbs_filter_info_t;

/* Pure part of a mixed Gaussian state.
 *   gamma_th : device, 2N x 2N FP64, xxpp, vacuum = identity/2, symmetric
 *              (GBS_E_NOT_PD otherwise); read only.
 *   N        : modes, 1..GBS_FILTER_MODES_MAX.
 *   opt      : host.
 *   gamma_p  : device, 2N x 2N FP64 output, S S^T / 2 (a valid input of
 *              gbs_mps_build).
 *   S_out    : device, 2N x 2N FP64 output (may be NULL): the symplectic S.
 *   info     : host output.
 * Synchronises `stream` (the host checks the loss between batches of
 * steps).  A state that does not reach L <= eps within max_iter returns
 * GBS_OK with info->converged = 0 and the last S. */
int gbs_filter_pure(const double* gamma_th, int32_t N, const gbs_filter_opts* opt, double* gamma_p, double* S_out,
                    gbs_filter_info_t* info, void* stream);

/* ---- Serving: build and sample requests on one GPU ----------------------
 * The consumer the paper names for its MPS is sampling (Sec. I).  A server
 * takes three kinds of request from many callers:
 *   GBS_REQ_BUILD_SAMPLE : convert a state, draw `shots` samples, free the MPS;
 *   GBS_REQ_BUILD        : convert a state and keep its MPS resident on the
 *                          device (drawing `shots` samples too when > 0); the
 *                          request's id names the resident MPS;
 *   GBS_REQ_SAMPLE       : draw `shots` samples from a resident MPS (`handle`).
 * Builds run the Gaussian SVD as the sequential chain (GBS_CHAIN_GSVD is
 * set on every build request): concurrent builds share the device, so total
 * work matters more than one build's latency.
 * Builds queue in FIFO order.  `slots` worker threads, each with its own HIP
 * stream, start the head of the build queue as soon as one is free and the
 * head's footprint (gbs_mps_footprint) fits `budget_bytes` beside everything
 * admitted, resident MPS included.  Samples are drawn by one batched sweep
 * (its own thread and stream): every request in it advances one site per
 * step, all requests in the same launches, each through its own descriptor
 * (site tensors, current site, buffers, seed, output); the sweep enqueues
 * up to 16 steps per round trip to the host, and requests join at the start
 * of a round as memory allows and leave after their last site.  MPS without the
 * FP32 sampler operand (FP64 builds) and requests above 2^20 shots are
 * sampled on their own.  A request's samples are identical whether it runs
 * alone or in a mix: the build is deterministic and the random numbers are
 * keyed by (seed, shot, site), so every shot's arithmetic depends only on its
 * own MPS, seed and shot number. */
typedef struct gbs_server_s* gbs_server;

enum { GBS_REQ_BUILD_SAMPLE = 0, GBS_REQ_BUILD = 1, GBS_REQ_SAMPLE = 2 };

typedef struct {
  const double* gamma; /* builds: device, 2M x 2M FP64 as for gbs_mps_build; caller keeps it valid until done */
  int32_t M;
  gbs_build_opts opt;
  int64_t shots;       /* >= 0 (>= 1 for GBS_REQ_SAMPLE) */
  uint64_t seed;
  int32_t* out;        /* device, shots x M int32; written when the request is done */
  int32_t kind;        /* GBS_REQ_* */
  int64_t handle;      /* GBS_REQ_SAMPLE: id of the GBS_REQ_BUILD request whose MPS to sample */
} gbs_request;

typedef struct {
  int32_t status;      /* GBS_OK or the build / sample error code */
  int32_t max_bond;
  double eps_max;
  double queue_ms;     /* submit -> start of service */
  double build_ms;     /* gbs_mps_build (0 for sample requests) */
  double sample_ms;    /* sampling, up to samples ready on the device */
  double latency_ms;   /* submit -> samples ready */
  int64_t handle;      /* GBS_REQ_BUILD: id of the resident MPS (the request's id); else 0 */
} gbs_result;

typedef struct {
  int64_t submitted, completed, failed;
  double p50_ms, p99_ms, mean_ms, max_ms; /* latency of completed requests, nearest-rank percentiles */
  double wall_s;                          /* first submit -> last completion */
  double throughput_rps;                  /* completed / wall_s */
  int64_t peak_bytes;                     /* largest admitted footprint sum */
  int64_t resident;                       /* MPS held resident now */
  int64_t sweep_steps;                    /* steps of the batched sampling sweep */
  double mean_batch;                      /* requests per sweep step, mean */
  int64_t max_batch;                      /* requests per sweep step, largest */
} gbs_server_stats_t;

/* Create a server on the current device.  slots in [1, 64]; budget_bytes:
 * device memory the admitted requests and resident MPS may hold together (a
 * build larger than the budget is rejected at submit with GBS_E_NOMEM);
 * max_queue: queued builds (or queued samples) beyond which submit returns
 * GBS_E_BUSY.  out: host.  Each build slot works on its own HIP stream;
 * slots run concurrently on the device only up to the process's hardware
 * queue count (the GPU_MAX_HW_QUEUES environment variable, read when HIP
 * starts), so a process serving many slots should set it to at least the
 * slot count plus one. */
int gbs_server_create(int32_t slots, int64_t budget_bytes, int32_t max_queue, gbs_server* out);
/* Queue a request (host struct, copied).  *id (host) receives its id.
 * GBS_E_INVAL for an unknown kind, a sample request naming no resident MPS
 * (or one being released), or missing pointers. */
int gbs_server_submit(gbs_server s, const gbs_request* req, int64_t* id);
/* Release a resident MPS: freed once the sample requests admitted or
 * queued on it are done; later sample requests naming it are rejected. */
int gbs_server_release(gbs_server s, int64_t handle);
/* *done (host) = 1 once the request's samples are ready. */
int gbs_server_poll(gbs_server s, int64_t id, int32_t* done);
/* Block until the request is done, fill *res (host, may be NULL), forget the
 * id, and return the request's status. */
int gbs_server_wait(gbs_server s, int64_t id, gbs_result* res);
/* Latency and throughput over the requests completed since the last reset. */
int gbs_server_stats(gbs_server s, gbs_server_stats_t* out);
int gbs_server_reset_stats(gbs_server s);
/* Finish every queued request, then stop the workers, free every resident
 * MPS and the server. */
void gbs_server_destroy(gbs_server s);

/* Thread-local message for the last failing call on this thread. */
const char* gbs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GBS_MPS_H */
