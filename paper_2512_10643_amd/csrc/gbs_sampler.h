// MFMA sampling sweep launch interface.
#pragma once
#include "gbs_common.h"

// K and N padded to multiples of 16 for the packed layout.
int sampler_pad(int n);
// Pack site tensor B (K x d x N, complex FP32) into the MFMA operand layout:
// d * (2 pad(K)) * (2 pad(N)) floats.
hipError_t launch_pack(hipStream_t st, const cplx32* B, int K, int d, int N, float* P);
// Shots per workgroup of the sampling kernel.
int sampler_shots_per_block();
// Left vectors of the first site (bond dimension k0, normally 1): row r of
// `l` (stride ldl2 floats) becomes e_0 over 2 pad(k0) floats.
hipError_t launch_sampler_init(hipStream_t st, float* l, long ldl2, int k0, int64_t n);
// One conditional-sampling step at `site` for nshots shots (chunk-local rows
// of lin/lout, row stride ldl2 floats, 2 pad(K) <= ldl2 and 2 pad(N) <= ldl2;
// pad(N) <= 256).  Rows of lin are scaled by sin (NULL: 1); lout receives the
// unnormalised selected rows and sout their inverse norms.
hipError_t launch_sample_mfma(hipStream_t st, const float* P, int K, int d, int N, const float* lin,
                              const float* sin, float* lout, float* sout, long ldl2, int64_t shot0, int64_t nshots,
                              int site, uint64_t seed, int32_t* out, int M);
