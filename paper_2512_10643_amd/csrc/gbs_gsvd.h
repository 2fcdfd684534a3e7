// Validation and Gaussian-SVD launch interfaces.
#pragma once
#include "gbs_common.h"

#define GBS_GSVD_N2_MAX 600      // 2 * (n_e^{m-1} + 1) handled by one workgroup
#define GBS_GSVD_LDS_N2 176      // packed symmetric working matrix kept in LDS up to this size

struct GsvdArgs {
  int M;
  double dstar;
  const double* gamma;   // 2M x 2M, row-major
  int* ne;               // ne[0..M]
  int* err;
  double* dsym;          // (M+1) x ld_dsym: symplectic eigenvalues per cut
  double* lam;           // (M+1) x ld_dsym: Lambda per cut (all L modes)
  long ld_dsym;
  const double* drr_in;  // r-r block of the residual, ld_drr
  double* drr_out;
  long ld_drr;
  const double* cr_in;   // r - a cross block, rows = r quadratures, cols indexed as Gamma's
  double* cr_out;
  long ld_cr;
  cplx64* Q;             // per-site pair matrices
  long q_stride, ld_q;
  // workspace
  double *ws_G, *ws_L, *ws_A, *ws_B, *ws_E, *ws_O, *ws_S, *ws_vec, *ws_W, *ws_pack, *ws_w, *ws_glr;
  int* ws_ord;
  double* ws_tri;        // inverse-iteration scratch: 4 N2 doubles per thread, N2 / 2 threads
  long ld_ws, ld_glr;
  cplx64 *ws_U, *ws_V, *ws_aug;
  long ld_u;
  int q_first;           // Q^j is formed beside cut j + 1 only for j >= q_first
};

hipError_t launch_validate(hipStream_t st, const double* gamma, int M, double* scal, double* wsM, int* err);
// Cut m: Williamson step of cut m (with, beside it, Q^{m-1} of the previous
// cut) and the pairing and residual of cut m.
hipError_t launch_gsvd_cut(hipStream_t st, const GsvdArgs& a, int m, int n2max);
// Q^M of the last site, after the last cut.
hipError_t launch_gsvd_last_q(hipStream_t st, const GsvdArgs& a);
// Q^m of site m alone, after cut m (its S is the last one formed).
hipError_t launch_gsvd_q(hipStream_t st, const GsvdArgs& a, int m);
// Start the chain at cut k straight from Gamma: the modes a_1..a_{k-1} stand
// in for r_{k-1}, so drr_in and cr_in receive Gamma's rows of their
// quadratures and ne[k-1] = k - 1.  Needs 2 k <= n2max (the leading dimension
// and row count of drr_in, the row count of cr_in).
hipError_t launch_gsvd_restart(hipStream_t st, const GsvdArgs& a, int k);
// out = Gamma with the modes numbered M..1 (xxpp order kept), 2M x 2M.
hipError_t launch_reverse_modes(hipStream_t st, const double* gamma, int M, double* out);
// out[b][p][a] = in[a][p][b] for an A x d x B complex FP64 tensor.
hipError_t launch_transpose_bonds(hipStream_t st, const cplx64* in, long A, int d, long B, cplx64* out);
