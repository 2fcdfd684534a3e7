// MFMA sampling sweep launch interface.
#pragma once
#include "gbs_common.h"

// K and N padded to multiples of 16 for the packed layout.
int sampler_pad(int n);
// Pack site tensor B (K x d x N, complex FP32) into the MFMA operand layout:
// d * (2 pad(K)) * (2 pad(N)) floats.
hipError_t launch_pack(hipStream_t st, const cplx32* B, int K, int d, int N, float* P);
// One conditional-sampling step at `site` for nshots shots (chunk-local rows
// of lin/lout, row stride ldl2 floats); requires pad(N) <= 256.
hipError_t launch_sample_mfma(hipStream_t st, const float* P, int K, int d, int N, const float* lin, float* lout,
                              long ldl2, int64_t shot0, int64_t nshots, int site, uint64_t seed, int32_t* out,
                              int M);
