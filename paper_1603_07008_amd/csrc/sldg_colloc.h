// Transverse Gauss-node collocated sweep (sldg_colloc.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sldg_internal.h"

namespace sldg {

struct ColArgs {
  const double* in_lo;
  const void* in_hi;
  double* out_lo;
  void* out_hi;
  const int32_t* pmap;     // per mode id: >= 0 plane in hi, < 0 plane -1-v in lo
  const int32_t* s_tab;    // per (transverse cell, node) entry: s mod N_d
  const double* ab_tab;    // A then B per entry, component-major (stride ab_cs)
  int64_t ab_cs;
  int64_t cells;
  int32_t ndim, d, t;      // swept and transverse dimensions
  int64_t Pd, Nd, Pt, Nt;  // strides (cells) and extents of d and t
  FastDiv fPd, fNd, fPt, fNt;
  int32_t n_lo;            // planes in lo
  int32_t wide;            // 0: at most the cell mean in FP64 (plane index m - n_lo)
  int32_t msd, mst;        // mode-id strides of j_d and j_t
  int32_t ngroups;         // spectator groups (o^(ndim-2))
  double P[4][4];          // P_j(y_q) at the Gauss nodes (ascending)
  double back[4][4];       // (2j+1)/2 w_q P_j(y_q)
};

hipError_t launch_colloc(int k, int tier, const ColArgs& a, hipStream_t st);

}  // namespace sldg
