// Transverse Gauss-node collocated sweep (C ABI sldg_advect_dim_collocated).
//
// The sweep along d (L. Einkemmer, arXiv 1603.07008, section II-A, update
// rule) with a displacement that varies across the transverse cells of one
// dimension t: the state is taken at the o Gauss-Legendre nodes y_q of the
// transverse cell (modal -> nodal in j_t), every node line is swept with its
// own displacement, and the result is projected back onto the Legendre modes
// in t with the Gauss weights (eq. (cj) with the o-point rule).  Every mode
// index other than j_d and j_t is a spectator.
//
// One thread per output cell and spectator group; for each node it gathers
// the two source cells of that node's shift, and keeps them for the next
// node when the integer shift is the same.  Arithmetic in FP64; the narrow
// modes are rounded to nearest even on store.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sldg_colloc.h"

namespace sldg {

template <class T>
__device__ __forceinline__ double c_widen(T v) {
  if constexpr (sizeof(T) == 2) return (double)(float)v;
  else return (double)v;
}

// FP64 -> storage type with one rounding to nearest even.  16-bit types go
// through FP32 rounded to odd (truncate, then set the last bit when inexact),
// which keeps the final RNE step correctly rounded (24 > 11 + 1 bits).
template <class T>
__device__ __forceinline__ T c_narrow(double v) {
  if constexpr (sizeof(T) == 2) {
    float f = (float)v;
    if (isfinite(f) && (double)f != v) {
      uint32_t b = __float_as_uint(f);
      if (fabs((double)f) > fabs(v)) b -= 1;
      f = __uint_as_float(b | 1u);
    } else if (!isfinite(f) && isfinite(v)) {
      f = v > 0 ? 3.4028234663852886e38f : -3.4028234663852886e38f;
    }
    return (T)f;
  } else {
    return (T)v;
  }
}

// Where the o x o modes (j_d, j_t) of a spectator group are stored.
// LO = 0: all in hi, at plane v.  LO = 1: mode (0, 0) is plane 0 of lo, the
// rest in hi (one FP64 mode and the group that holds it).  LO = 2: any mix,
// v < 0 meaning plane -1-v of lo.
template <int LO, class T>
__device__ __forceinline__ double c_load(const ColArgs& a, const T* hin, int32_t v, bool first,
                                         int64_t x) {
  if ((LO == 1 && first) || (LO == 2 && v < 0))
    return a.in_lo[(LO == 1 ? 0 : (int64_t)(-1 - v)) * a.cells + x];
  return c_widen(hin[(int64_t)v * a.cells + x]);
}

// Stores: consecutive lanes write consecutive cells, so a wave writes whole
// lines and 4- and 8-byte values carry the non-temporal hint (outputs are not
// read again by the sweep); 2-byte values stay plain.
template <int LO, class T>
__device__ __forceinline__ void c_store(const ColArgs& a, T* hout, int32_t v, bool first,
                                        int64_t x, double r) {
  if ((LO == 1 && first) || (LO == 2 && v < 0)) {
    __builtin_nontemporal_store(r, a.out_lo + (LO == 1 ? 0 : (int64_t)(-1 - v)) * a.cells + x);
  } else {
    T* p = hout + (int64_t)v * a.cells + x;
    if constexpr (sizeof(T) >= 4) __builtin_nontemporal_store(c_narrow<T>(r), p);
    else *p = c_narrow<T>(r);
  }
}

// The sweep of one output cell c of one spectator group, whose modes are
// stored at pl[j_d][j_t] (in the form LO).
template <int K, class T, int LO>
__device__ __forceinline__ void colloc_cell(const ColArgs& a, const int32_t (&pl)[K + 1][K + 1],
                                            int64_t c, int32_t id, int32_t it) {
  constexpr int O = K + 1;
  const T* hin = static_cast<const T*>(a.in_hi);
  T* hout = static_cast<T*>(a.out_hi);
  double res[O][O];
#pragma unroll
  for (int jd = 0; jd < O; ++jd)
#pragma unroll
    for (int jt = 0; jt < O; ++jt) res[jd][jt] = 0.0;
  // the o^2 modes of the two source cells, loaded again only when a node's
  // integer shift differs from the previous node's (the node loop stays
  // rolled: one node's tables live at a time)
  double va[O][O], vb[O][O];
  int32_t s_prev = -1;
#pragma unroll 1
  for (int q = 0; q < O; ++q) {
    const int32_t s = a.s_tab[(int64_t)it * O + q];
    if (s != s_prev) {
      s_prev = s;
      int32_t ia = id - s;
      if (ia < 0) ia += (int32_t)a.Nd;
      int32_t ib = ia - 1;
      if (ib < 0) ib += (int32_t)a.Nd;
      const int64_t ca = c + (int64_t)(ia - id) * a.Pd, cb = c + (int64_t)(ib - id) * a.Pd;
#pragma unroll
      for (int jd = 0; jd < O; ++jd)
#pragma unroll
        for (int jt = 0; jt < O; ++jt) {
          va[jd][jt] = c_load<LO>(a, hin, pl[jd][jt], jd + jt == 0, ca);
          vb[jd][jt] = c_load<LO>(a, hin, pl[jd][jt], jd + jt == 0, cb);
        }
    }
    double x[O], y[O];                                  // node values at the two sources
#pragma unroll
    for (int jd = 0; jd < O; ++jd) {
      double xa = 0.0, yb = 0.0;
#pragma unroll
      for (int jt = 0; jt < O; ++jt) {
        xa = fma(a.P[jt][q], va[jd][jt], xa);
        yb = fma(a.P[jt][q], vb[jd][jt], yb);
      }
      x[jd] = xa;
      y[jd] = yb;
    }
    const double* ab = a.ab_tab + (int64_t)it * O + q;  // entry (transverse cell, node)
#pragma unroll
    for (int j = 0; j < O; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < O; ++l) acc = fma(ab[(j * O + l) * a.ab_cs], x[l], acc);
#pragma unroll
      for (int l = 0; l < O; ++l) acc = fma(ab[(O * O + j * O + l) * a.ab_cs], y[l], acc);
#pragma unroll
      for (int jt = 0; jt < O; ++jt) res[j][jt] = fma(a.back[jt][q], acc, res[j][jt]);
    }
  }
#pragma unroll
  for (int jd = 0; jd < O; ++jd)
#pragma unroll
    for (int jt = 0; jt < O; ++jt) c_store<LO>(a, hout, pl[jd][jt], jd + jt == 0, c, res[jd][jt]);
}

// UNI: every wave lies in one transverse cell (the transverse stride is a
// multiple of 64 cells), so the shifts and weights are scalar loads.
// WIDE: more than the cell mean is FP64 (plane map from the table).
template <int K, class T, bool UNI, bool WIDE>
__global__ __launch_bounds__(256) void sweep_colloc_kernel(ColArgs a) {
  constexpr int O = K + 1;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.cells) return;
  // mode base of the spectator group blockIdx.y (dims other than d and t)
  int32_t base = 0;
  {
    int32_t r = (int32_t)blockIdx.y, ostride = 1;
    for (int e = 0; e < a.ndim; ++e) {
      if (e != a.d && e != a.t) {
        base += (r % O) * ostride;
        r /= O;
      }
      ostride *= O;
    }
  }
  const int32_t id = (int32_t)a.fNd.mod(a.fPd.div((uint32_t)c));
  int32_t it = (int32_t)a.fNt.mod(a.fPt.div((uint32_t)c));
  if (UNI) it = __builtin_amdgcn_readfirstlane(it);
  int32_t pl[O][O];
#pragma unroll
  for (int jd = 0; jd < O; ++jd)
#pragma unroll
    for (int jt = 0; jt < O; ++jt) {
      const int32_t m = __builtin_amdgcn_readfirstlane(base + jd * a.msd + jt * a.mst);
      pl[jd][jt] = WIDE ? __builtin_amdgcn_readfirstlane(a.pmap[m]) : m - a.n_lo;
    }
  if (WIDE) colloc_cell<K, T, 2>(a, pl, c, id, it);
  else if (a.n_lo == 1 && base == 0) colloc_cell<K, T, 1>(a, pl, c, id, it);
  else colloc_cell<K, T, 0>(a, pl, c, id, it);
}

template <int K, class T>
static void launch_colloc_t(const ColArgs& a, dim3 grid, hipStream_t st) {
  const bool uni = a.Pt % 64 == 0;
  if (a.wide) {
    if (uni) sweep_colloc_kernel<K, T, true, true><<<grid, 256, 0, st>>>(a);
    else sweep_colloc_kernel<K, T, false, true><<<grid, 256, 0, st>>>(a);
  } else {
    if (uni) sweep_colloc_kernel<K, T, true, false><<<grid, 256, 0, st>>>(a);
    else sweep_colloc_kernel<K, T, false, false><<<grid, 256, 0, st>>>(a);
  }
}

template <int K>
static hipError_t launch_colloc_k(int tier, const ColArgs& a, hipStream_t st) {
  dim3 grid((unsigned)((a.cells + 255) / 256), (unsigned)a.ngroups);
  switch (tier) {
    case 0: launch_colloc_t<K, double>(a, grid, st); break;
    case 1: launch_colloc_t<K, float>(a, grid, st); break;
    case 2: launch_colloc_t<K, __bf16>(a, grid, st); break;
    case 3: launch_colloc_t<K, _Float16>(a, grid, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_colloc(int k, int tier, const ColArgs& a, hipStream_t st) {
  if (a.cells <= 0) return hipSuccess;
  if ((a.cells + 255) / 256 > 0x7fffffff || a.ngroups > 65535) return hipErrorInvalidConfiguration;
  switch (k) {
    case 1: return launch_colloc_k<1>(tier, a, st);
    case 2: return launch_colloc_k<2>(tier, a, st);
    case 3: return launch_colloc_k<3>(tier, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sldg
