// Validation and Gaussian-SVD launch interfaces.
#pragma once
#include "gbs_common.h"

#define GBS_GSVD_N2_MAX 600      // 2 * (n_e^{m-1} + 1) handled by one workgroup
#define GBS_GSVD_LDS_N2 176      // packed symmetric working matrix kept in LDS up to this size
#define GBS_GSVD_INDEP_LAMBDA_MIN 1e-3  // weakest bond mode (Lambda) a full build aligns site by site

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
  int q_slot0;           // Q^j is stored in slot j - 1 - q_slot0 of Q (stride q_stride)
};

// Alignment of the bond modes of cut m between site m (its chain step) and
// site m + 1 (its start from Gamma at cut m).
struct GsvdAlign {
  const double* t0;   // site m's start map at cut m-1: active rows (x then p), 2 (m-1) columns; NULL when m = 1
  long ldt0;
  const int* ne_e;    // site m's ne (ne_e[m-1]: r_{m-1} modes, ne_e[m]: l_m modes)
  const double* t1;   // site m's step map at cut m: active rows, 2 (ne_e[m-1] + 1) columns
  long ldt1;
  const double* tr;   // site m+1's start map at cut m: active rows, 2 m columns
  long ldtr;
  const int* ne_r;    // site m+1's ne (ne_r[m] must equal ne_e[m])
  cplx64* Q;          // Q^m, row stride ld_q
  long ld_q;
  int m;
  int pad;
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
// Every site's Gaussian data on its own: element e (site m) runs cut
// cut0[e] = m - 1 from Gamma (args0; 0 for site 1) and then cut1[e] = m
// (args1: the same workspaces, residual buffers swapped), forming Q^m (for
// the last site, the residual's own pair matrix).  keep_dst[e] / keep_ld[e]
// receive the b-mode map rows of the first cut.  Then the bond modes of
// every cut are aligned (al, nalign cuts).
hipError_t launch_gsvd_independent(hipStream_t st, const GsvdArgs* args0, const GsvdArgs* args1, const int* cut0,
                                   const int* cut1, int nel, double* const* keep_dst, const long* keep_ld,
                                   const GsvdAlign* al, int nalign, int* err);
// Entangled pairs and Lambda of every cut m = 1..M-1 from site m's second
// cut (args: the second-cut arguments of the sites) into ne_out[m] and row
// m of lam_out (leading dimension ld_out).
// Copy Q^m (n_m x n_m at leading dimension ld_q in slot m - 1 - slot0 of a
// strided buffer) to dst + dst_off[i] (leading dimension n_m), for the
// sites site[0..nsites).
hipError_t launch_q_compact(hipStream_t st, const cplx64* src, long q_stride, long ld_q, int slot0, const int* site,
                            const int* n, const long* dst_off, int nsites, cplx64* dst);
hipError_t launch_gsvd_gather_cuts(hipStream_t st, const GsvdArgs* args, int M, int* ne_out, double* lam_out,
                                   long ld_out);
// out = Gamma with the modes numbered M..1 (xxpp order kept), 2M x 2M.
hipError_t launch_reverse_modes(hipStream_t st, const double* gamma, int M, double* out);
// out[b][p][a] = in[a][p][b] for an A x d x B complex FP64 tensor.
hipError_t launch_transpose_bonds(hipStream_t st, const cplx64* in, long A, int d, long B, cplx64* out);
