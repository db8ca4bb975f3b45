// Instantiation unit of the sweep kernels for one degree k and one storage
// tier, selected when compiling (-DSLDG_K=1..3 -DSLDG_TIER=0..3): the build
// compiles this file once per pair, so the template-heavy sweep kernels
// compile in parallel.  Holds the launchers of the single-grid sweeps and of
// the batched sweep classes; the dispatch over (k, tier) is in
// sldg_kernels.hip.
#include "sldg_sweep.h"
#include "sldg_fused.h"
#include "sldg_staged.h"

#if !defined(SLDG_K) || !defined(SLDG_TIER)
#error "compile with -DSLDG_K=<degree> -DSLDG_TIER=<tier>"
#endif

namespace sldg {

template <int K, int TIER, int L, int NDMAX>
static void launch_strided(int nt, dim3 grid, dim3 block, hipStream_t st, const SweepArgs& a) {
  if constexpr (TIER >= 2) {
    if (nt == 2) {
      sweep_strided_kernel<K, TIER, L, NDMAX, 2><<<grid, block, 0, st>>>(a);
      return;
    }
  }
  if (nt) sweep_strided_kernel<K, TIER, L, NDMAX, 1><<<grid, block, 0, st>>>(a);
  else sweep_strided_kernel<K, TIER, L, NDMAX, 0><<<grid, block, 0, st>>>(a);
}

// Staged strided sweep (sldg_staged.h).  The host stages only grids whose
// columns come in runs of 64 (P % 64 == 0), where every store of a wave
// covers whole lines: the non-temporal hint on 4-byte values (FP32) and on
// 2-byte values too (16-bit tiers), as the direct kernel takes it there.
template <int K, int TIER>
static bool launch_staged(dim3 grid, hipStream_t st, const SweepArgs& a) {
  constexpr int NT = TIER == 1 ? 1 : 2;
  constexpr int SZ = (int)sizeof(typename Tier<TIER>::T);
  const dim3 block(256);
  switch (a.chunk * 8 + a.colwaves) {
    case 4 * 8 + 1:
      sweep_staged_kernel<K, TIER, 4, 1, NT><<<grid, block, staged_lds_bytes(K, SZ, 4, 1), st>>>(a);
      return true;
    case 4 * 8 + 2:
      sweep_staged_kernel<K, TIER, 4, 2, NT><<<grid, block, staged_lds_bytes(K, SZ, 4, 2), st>>>(a);
      return true;
    case 8 * 8 + 1:
      sweep_staged_kernel<K, TIER, 8, 1, NT><<<grid, block, staged_lds_bytes(K, SZ, 8, 1), st>>>(a);
      return true;
    case 8 * 8 + 2:
      sweep_staged_kernel<K, TIER, 8, 2, NT><<<grid, block, staged_lds_bytes(K, SZ, 8, 2), st>>>(a);
      return true;
    case 4 * 8 + 4:
      sweep_staged_kernel<K, TIER, 4, 4, NT><<<grid, block, staged_lds_bytes(K, SZ, 4, 4), st>>>(a);
      return true;
    case 8 * 8 + 4:
      sweep_staged_kernel<K, TIER, 8, 4, NT><<<grid, block, staged_lds_bytes(K, SZ, 8, 4), st>>>(a);
      return true;
    default:
      return false;
  }
}

template <int K, int TIER, int NDMAX>
static hipError_t launch_sweep_ktn(int dim, const SweepArgs& a, hipStream_t st) {
  int form;
  dim3 grid, block;
  if (!sweep_grid(dim, a, form, grid, block)) return hipErrorInvalidConfiguration;
  if (form == 0) {
    sweep_contig_window_kernel<K, TIER, NDMAX><<<grid, block, 0, st>>>(a);
  } else if (form == 1) {
    sweep_contig_group_kernel<K, TIER, NDMAX><<<grid, block, 0, st>>>(a);
  } else if (form == 3) {
    // the lanes' cells are consecutive: whole lines per wave
    sweep_lane_kernel<K, TIER, NDMAX, 2><<<grid, block, 0, st>>>(a);
  } else {
    // ntmask: bit 0, 1, 2 for 2-, 4-, 8-byte values.  The narrow planes'
    // value size decides; on the 16-bit tiers, the FP64 mean may take the
    // hint (mode 1) where the 2-byte planes may not (mode 2)
    if constexpr (TIER >= 1 && NDMAX == 1) {
      if (a.stage && block.x == 256 && launch_staged<K, TIER>(grid, st, a)) return hipGetLastError();
    }
    int nt;
    if (TIER == 0) nt = (a.ntmask & 4) ? 1 : 0;
    else if (TIER == 1) nt = (a.ntmask & 2) ? 1 : 0;
    else nt = (a.ntmask & 1) ? 2 : (a.ntmask & 4) ? 1 : 0;
    switch (a.chunk) {
      case 1: launch_strided<K, TIER, 1, NDMAX>(nt, grid, block, st, a); break;
      case 2: launch_strided<K, TIER, 2, NDMAX>(nt, grid, block, st, a); break;
      case 4: launch_strided<K, TIER, 4, NDMAX>(nt, grid, block, st, a); break;
      case 8: launch_strided<K, TIER, 8, NDMAX>(nt, grid, block, st, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <int K, int TIER>
static hipError_t launch_sweep_kt(int dim, const SweepArgs& a, hipStream_t st) {
  return a.wide_fp64 ? launch_sweep_ktn<K, TIER, K + 1>(dim, a, st)
                     : launch_sweep_ktn<K, TIER, 1>(dim, a, st);
}


template <int K, int TIER>
hipError_t launch_sweep_inst(int dim, const SweepArgs& a, hipStream_t st) {
  return launch_sweep_kt<K, TIER>(dim, a, st);
}

template <int K, int TIER, int KIND>
static hipError_t launch_class_ktk(int rows, const SweepArgs* args, const BatchItem* items,
                                   int32_t nitems, int32_t xcd, hipStream_t st) {
  if constexpr (KIND == 1) {
    if (rows == 1) batch_class_kernel<K, TIER, 3, 1><<<nitems, 256, 0, st>>>(args, items, xcd);
    else batch_class_kernel<K, TIER, 1, 1><<<nitems, 256, 0, st>>>(args, items, xcd);
  } else if constexpr (KIND != 2) {
    batch_class_kernel<K, TIER, KIND, 1><<<nitems, 256, 0, st>>>(args, items, xcd);
  } else {
    switch (rows) {
      case 0: batch_class_kernel<K, TIER, 3, 1><<<nitems, 256, 0, st>>>(args, items, xcd); break;
      case 2: batch_class_kernel<K, TIER, 2, 2><<<nitems, 256, 0, st>>>(args, items, xcd); break;
      case 4: batch_class_kernel<K, TIER, 2, 4><<<nitems, 256, 0, st>>>(args, items, xcd); break;
      case 8: batch_class_kernel<K, TIER, 2, 8><<<nitems, 256, 0, st>>>(args, items, xcd); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <int K, int TIER>
static hipError_t launch_class_kt(int kind, int rows, const SweepArgs* args,
                                  const BatchItem* items, int32_t nitems, int32_t xcd,
                                  hipStream_t st) {
  switch (kind) {
    case 0: return launch_class_ktk<K, TIER, 0>(rows, args, items, nitems, xcd, st);
    case 1: return launch_class_ktk<K, TIER, 1>(rows, args, items, nitems, xcd, st);
    case 2: return launch_class_ktk<K, TIER, 2>(rows, args, items, nitems, xcd, st);
    default: return hipErrorInvalidValue;
  }
}


template <int K, int TIER>
hipError_t launch_class_inst(int kind, int rows, const SweepArgs* args, const BatchItem* items,
                             int32_t nitems, int32_t xcd, hipStream_t st) {
  return launch_class_kt<K, TIER>(kind, rows, args, items, nitems, xcd, st);
}

template <int K, int TIER>
hipError_t launch_xy_inst(const XYArgs& a, int64_t lds_bytes, int32_t nblocks, hipStream_t st) {
  sweep_xy_kernel<K, TIER><<<nblocks, 256, (size_t)lds_bytes, st>>>(a);
  return hipGetLastError();
}

template hipError_t launch_sweep_inst<SLDG_K, SLDG_TIER>(int, const SweepArgs&, hipStream_t);
template hipError_t launch_xy_inst<SLDG_K, SLDG_TIER>(const XYArgs&, int64_t, int32_t, hipStream_t);
template hipError_t launch_class_inst<SLDG_K, SLDG_TIER>(int, int, const SweepArgs*,
                                                         const BatchItem*, int32_t, int32_t,
                                                         hipStream_t);

}  // namespace sldg
