// PCO level-gather launch interface.
#pragma once
#include "gbs_common.h"

struct SiteDesc {
  int nl, nr, d, chiL, chiR;   // incoming / outgoing active modes, cutoff, basis sizes
  long off_state_l, off_state_r;  // per-state array offsets of cuts m-1 and m
  long off_occ_l, off_occ_r;      // lowering-table offsets of cuts m-1 and m
  long off_q;                     // Q^m offset (elements)
  long off_t;                     // tensor offset (elements)
};

struct LevelBlock {
  int site;        // 0-based site index
  int p;           // physical occupation
  int a_off, a_cnt;  // slice of the left basis sorted by photon number
  int b_off, b_cnt;  // slice of the right basis sorted by photon number
  long elem_start; // first element index of this block within the level
};

struct PcoArgs {
  const SiteDesc* sites;
  const int* perm;       // per cut: states sorted by total photon number (offset off_state)
  const int4* olist;     // occupied lists (mode, count, low index, 0)
  const int* nocc;
  const int* low;        // lowering tables
  const cplx64* Q;
  long ld_q;
  cplx64* T;             // tensors, FP64
  unsigned long long* terms;  // optional: total number of source terms summed (NULL: not counted)
};

hipError_t launch_pco_init(hipStream_t st, const PcoArgs& a, int nsites);
hipError_t launch_pco_level(hipStream_t st, const PcoArgs& a, const LevelBlock* blocks, int nblocks, long nelem,
                            int k);
