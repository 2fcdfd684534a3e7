// Kept-basis and index-map launch interface.
#pragma once
#include "gbs_common.h"

struct CutDesc {
  int ne;          // active virtual modes at this cut
  int chi;         // requested basis size (1 when ne == 0)
  long off_state;  // offset into per-state arrays
  long off_occ;    // offset into occupation / lowering tables (chi * ne)
  int eslot;       // slot of the parallel enumeration's workspace (-1: none)
  int pad;
};

struct KeptArgs {
  const CutDesc* cuts;   // index 0..M
  const double* lam;     // Lambda per cut, row m, leading dimension ld_lam
  long ld_lam;
  double* E;
  int *parent, *pmode, *ntot, *nocc;
  unsigned long long* hash;
  short* occ;            // chi x ne per cut
  int* low;              // ne x chi per cut
  int4* olist;           // chi x GBS_K_MAX per cut: (mode, count, low index, 0)
  int* chi_out;          // kept count per cut
  int* err;
  char* gws;             // NULL: heap and sort buffer in LDS; else cut m's at gws + m * gws_stride
  long gws_stride;
  double eps_target;     // > 0: stop once the discarded weight is at most this (D(eps))
  // parallel enumeration (cuts with chi >= kKeptParallelMin): cut m's
  // workspace at ews + cuts[m].eslot * ews_stride; enum_done[m] = 1 once its
  // basis is written (0: the heap enumerates it)
  char* ews;
  long ews_stride;
  int ews_ne;            // largest ne the workspace was sized for
  int* enum_done;
};

// Bytes of the heap / sort workspace of one cut with `chi` states, and the
// largest that the kernel keeps in LDS.
size_t kept_workspace_bytes(int chi);
constexpr size_t kKeptLdsMax = 144 * 1024;

hipError_t launch_kept(hipStream_t st, const KeptArgs& a, int ncuts, int chi);

// Parallel enumeration of large bases, exactly the heap's order: cuts with
// chi >= kKeptParallelMin, one workgroup each.  kept_enum_bytes: workspace
// of one cut (chi states, ne modes).
constexpr int kKeptParallelMin = 256;
constexpr int kKeptEnumNeMax = 300;   // modes the parallel enumeration takes
size_t kept_enum_bytes(int chi, int ne);
hipError_t launch_kept_enum(hipStream_t st, const KeptArgs& a, int ncuts);
