// MPS-level kernel launch interfaces.
#pragma once
#include "gbs_common.h"

template <typename CD, typename CS>
hipError_t convert(hipStream_t st, CD* dst, const CS* src, long n);
template <typename CD>
hipError_t scaled_copy(hipStream_t st, CD* dst, long ld_dst, const cplx64* src, long ld_src, int rows, int cols,
                       const double* colscale, int invert, int conj_transpose);
// x[i][p][j] *= sqrt(wcol[j]) / sqrt(wrow[i])  (NULL -> 1)
template <typename C>
hipError_t gauge_scale(hipStream_t st, C* x, int rows, int d, int cols, const double* wrow, const double* wcol);
// Scales site 1 (n1 elements) so that the state has unit norm and a real
// positive vacuum amplitude.  vac: <0..0|psi> before scaling (device);
// nrm2_in: the squared norm (device scalar), or NULL to take it from site 1
// alone (exact when sites 2..M are right-canonical).
template <typename C>
hipError_t normalize_mps(hipStream_t st, C* site1, int n1, const cplx64* vac, const double* nrm2_in,
                         double* out_norm);
template <typename C>
hipError_t launch_amplitude(hipStream_t st, C* const* sites, const int* bond, int M, int d, const int32_t* pat,
                            int64_t B, double* out, int* bad, int maxbond);
template <typename C>
hipError_t launch_fill_first(hipStream_t st, C* l, long ldl, int64_t n);
template <typename C>
hipError_t launch_sample_site(hipStream_t st, const C* Bm, int rl, int d, int rr, const C* lin, C* lout, long ldl,
                              int64_t shot0, int64_t nshots, int site, uint64_t seed, int32_t* out, int M);
