// MFMA sampling sweep launch interface.
//
// The sweep works on photon-parity sectors.  A Gaussian state with zero mean
// is an eigenstate of the total photon parity, so every bond index of its
// canonical MPS can carry a parity (0 or 1) with B[a, p, b] = 0 unless
// par(a) + p + par(b) is even.  A shot whose left vector lies in sector pi of
// bond m-1 then only touches the rows of sector pi and, for outcome p, the
// columns of sector pi ^ (p & 1) of bond m.  Left vectors are stored in
// sector-local indices.  With one sector per bond (pi = 0 for every shot and
// both column sets equal to the whole bond) the same code is the dense sweep.
//
// Outcomes are visited in the order 0, 1, 2, ... and grouped into passes:
// outcome 0 alone, then runs of consecutive outcomes whose column tiles
// together fit the kernel's accumulator budget, each pass one sweep over the
// K rows.  A shot stops at the first outcome whose cumulative probability
// passes its uniform, so most shots need only the first pass.
#pragma once
#include "gbs_common.h"

// K and N padded to multiples of 16 for the packed layout.
int sampler_pad(int n);
// Largest padded sector width and number of outcomes the kernel takes.
constexpr int kSamplerMaxSector = 256;
constexpr int kSamplerMaxOutcomes = 32;
// Accumulator budget: 16-column tiles of one pass.
constexpr int kSamplerMaxTiles = 32;

// Sector sizes of one site: nL[pi] rows of left sector pi, nR[s] columns of
// right sector s.  Dense layout: nL = {K, 0}, nR = {N, N}.
struct SamplerSite {
  int nL[2];
  int nR[2];
};

// Launch geometry of one site (host and device copies).  For left sector pi:
// nchunk[pi] K-chunks of 32 real rows, the last of each pass holding only
// its first 16 when half[pi] (rows are padded to 8 complex entries); right
// sector s is nt[s] tiles wide;
// pass q covers outcomes [j0[pi][q], j0[pi][q + 1]) with
// tiles[pi][q] tiles per chunk, its chunks starting at float base[pi][q] of
// the packed operand.  NT: accumulator tiles of the kernel instance.
struct SamplerGeom {
  int nchunk[2];
  int half[2];
  int nt[2];
  int npass[2];
  int NT;
  int j0[2][kSamplerMaxOutcomes + 1];
  int tiles[2][kSamplerMaxOutcomes];
  long base[2][kSamplerMaxOutcomes];
};
// Fill g for site s with d outcomes; returns the floats of the packed
// operand, or -1 when the site does not fit the kernel (d or a sector too
// large).
long sampler_geometry(const SamplerSite& s, int d, SamplerGeom* g);

// Bond parities from the site tensors, one site per call, left to right.
// mask_l (K ints) is the previous bond's result, mask_r (N ints, zeroed by the
// caller) receives bit (par(a) + p) & 1 for every nonzero B[a, p, b], with
// par(a) = 1 iff mask_l[a] == 2.  A column with mask 3 breaks the parity
// structure; mask 0 marks a zero column.
hipError_t launch_sector_mask(hipStream_t st, const cplx32* B, int K, int d, int N, const int32_t* mask_l,
                              int32_t* mask_r);

// Pack site tensor B (K x d x N, complex FP32) into the MFMA operand layout,
// sector by sector and pass by pass.  mapL / mapR list the bond indices of
// sector 0 followed by those of sector 1 (NULL: identity, for the dense
// layout).  gd: device copy of g.
hipError_t launch_pack(hipStream_t st, const cplx32* B, int K, int d, int N, const SamplerSite& s,
                       const SamplerGeom& g, const SamplerGeom* gd, const int32_t* mapL, const int32_t* mapR,
                       float* P);
// Shots per workgroup of the sampling kernel.
// One site's packing (the arguments of launch_pack) for a batched launch.
struct SamplerPackDesc {
  const cplx32* B;
  int K, d, N, pad;
  SamplerSite s;
  const SamplerGeom* g;     // device
  const int32_t* mapL;
  const int32_t* mapR;
  float* P;
};
// launch_pack for n sites in one launch: host and dev hold the same n
// descriptors (dev: a device copy the launch reads), geo_host their
// geometries (host copies, for the grid and the checks).
hipError_t launch_pack_batch(hipStream_t st, const SamplerPackDesc* host, const SamplerPackDesc* dev, int n,
                             const SamplerGeom* geo_host);
int sampler_shots_per_block();
// Left vectors of the first site (bond dimension k0, normally 1): row r of
// `l` (stride ldl2 floats) becomes e_0 over 2 pad(k0) floats.
hipError_t launch_sampler_init(hipStream_t st, float* l, long ldl2, int k0, int64_t n);

// Passes [qbeg, qend) of one conditional-sampling step at `site` for nshots
// shots (chunk-local rows of lin/lout, row stride ldl2 floats).  Rows of lin
// enter as they are; lout receives the row of each shot's outcome scaled to
// unit norm (zero if the outcome has weight zero).  perm == NULL: every shot is in
// sector 0 and workgroup b takes shots [128 b, 128 b + 128).  Otherwise
// perm / cnt come from launch_sampler_partition and the grid covers both
// sector groups.  par_out (may be NULL) receives the parity of each shot's
// new bond index.  A launch with qbeg = 0 starts every shot's cumulative
// probability at 0; if it stops before a sector's last pass, it writes key
// (127: decided, else 4 x the shot's left sector + a bucket 0..3 of how far
// its uniform lies past the running sum) and the running sum cum of each
// undecided shot, and a second launch with qbeg = 1 takes the undecided
// shots from the bucketed partition of key and continues from cum.
hipError_t launch_sample_mfma(hipStream_t st, const float* P, const SamplerGeom& g, const SamplerGeom* gd,
                              const float* lin, float* lout, long ldl2,
                              const int32_t* perm, const int32_t* cnt, int8_t* par_out, float* cum, int8_t* key,
                              int qbeg, int qend, int64_t shot0, int64_t nshots, int site, uint64_t seed, int32_t* out,
                              int M);

// Stable partition of shots by sector.  Without buckets the key is the
// sector in {0, 1}; with buckets it is 4 x sector + bucket (0..3) and each
// sector's shots are sorted by bucket (stable within a bucket).  Other keys
// are left out.  perm[0, c0) lists the sector-0 shots, perm[E, E + c1) the
// sector-1 shots, E = c0 rounded up to a multiple of 128; cnt = {c0, c1}.
// perm holds nshots + 128 ints; bcnt is a workspace of
// sampler_partition_ws(nshots) ints.
int64_t sampler_partition_ws(int64_t nshots);
hipError_t launch_sampler_partition(hipStream_t st, const int8_t* par, int64_t nshots, int32_t* bcnt,
                                    int32_t* perm, int32_t* cnt, bool buckets);

// One request of a batched sampling sweep at its current site (device copy
// read by the batched kernels).  The request's shots are numbered from 0
// (Philox counter and output row), its left-vector rows ping-pong between
// fb[0] / fb[1] (site m reads fb[(m - 1) & 1]), and par / perm / cnt / bcnt
// are its parity partition buffers (sized as
// for a single-request sweep of nshots).
struct SampleBatchDesc {
  const float* packed;      // packed operand of the handle
  const long* poff;         // device, M + 1 offsets into packed (floats), by site
  const SamplerGeom* geo;   // device, M + 1 site geometries
  float* fb[2];
  int8_t* par;
  int32_t* perm;
  int32_t* cnt;
  int32_t* bcnt;
  int32_t* out;             // nshots x M int32
  long ldl2;
  int64_t nshots;
  uint32_t k0, k1;          // seed (low, high word)
  int M;
  int site;                 // current site, 1..M
  int psplit;               // photon-parity sectors
  int pad;
};
// Accumulator tiles (8, 16, 24 or 32) a site's passes need.
int sampler_batch_nt(const SamplerGeom& g);
// One site step of nreq requests (desc: device array); max_blocks: the
// largest ceil(nshots / 128) + 1 among them; nt: the largest
// sampler_batch_nt of their current sites.
hipError_t launch_sample_batch(hipStream_t st, const SampleBatchDesc* desc, int nreq, int64_t max_blocks, int nt);
// The parity partitions of the same step (requests at their last site skip).
hipError_t launch_partition_batch(hipStream_t st, const SampleBatchDesc* desc, int nreq, int64_t max_shots);
