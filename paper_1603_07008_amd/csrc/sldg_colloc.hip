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
// the two source cells of that node's shift, so nodes with equal integer
// shifts re-read cells already in the cache.  Arithmetic in FP64; the
// narrow modes are rounded to nearest even on store.
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

template <int K, class T>
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
  const int64_t id = (c / a.Pd) % a.Nd;
  const int64_t it = (c / a.Pt) % a.Nt;
  const T* hin = static_cast<const T*>(a.in_hi);
  T* hout = static_cast<T*>(a.out_hi);
  // where mode (j_d, j_t) of the group is stored
  int32_t pl[O][O];
#pragma unroll
  for (int jd = 0; jd < O; ++jd)
#pragma unroll
    for (int jt = 0; jt < O; ++jt) pl[jd][jt] = a.pmap[base + jd * a.msd + jt * a.mst];
  double res[O][O];
#pragma unroll
  for (int jd = 0; jd < O; ++jd)
#pragma unroll
    for (int jt = 0; jt < O; ++jt) res[jd][jt] = 0.0;
  for (int q = 0; q < O; ++q) {
    const int64_t te = it * O + q;                      // table entry (transverse cell, node)
    const int64_t s = a.s_tab[te];
    int64_t ia = id - s;
    if (ia < 0) ia += a.Nd;
    int64_t ib = ia - 1;
    if (ib < 0) ib += a.Nd;
    const int64_t ca = c + (ia - id) * a.Pd, cb = c + (ib - id) * a.Pd;
    double x[O], y[O];                                  // node values at the two sources
#pragma unroll
    for (int jd = 0; jd < O; ++jd) {
      double xa = 0.0, yb = 0.0;
#pragma unroll
      for (int jt = 0; jt < O; ++jt) {
        const int32_t v = pl[jd][jt];
        double va, vb;
        if (v < 0) {
          va = a.in_lo[(int64_t)(-1 - v) * a.cells + ca];
          vb = a.in_lo[(int64_t)(-1 - v) * a.cells + cb];
        } else {
          va = c_widen(hin[(int64_t)v * a.cells + ca]);
          vb = c_widen(hin[(int64_t)v * a.cells + cb]);
        }
        xa = fma(a.P[jt][q], va, xa);
        yb = fma(a.P[jt][q], vb, yb);
      }
      x[jd] = xa;
      y[jd] = yb;
    }
    const double* ab = a.ab_tab + te;
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
    for (int jt = 0; jt < O; ++jt) {
      const int32_t v = pl[jd][jt];
      if (v < 0) a.out_lo[(int64_t)(-1 - v) * a.cells + c] = res[jd][jt];
      else hout[(int64_t)v * a.cells + c] = c_narrow<T>(res[jd][jt]);
    }
}

template <int K>
static hipError_t launch_colloc_k(int tier, const ColArgs& a, hipStream_t st) {
  dim3 grid((unsigned)((a.cells + 255) / 256), (unsigned)a.ngroups);
  switch (tier) {
    case 0: sweep_colloc_kernel<K, double><<<grid, 256, 0, st>>>(a); break;
    case 1: sweep_colloc_kernel<K, float><<<grid, 256, 0, st>>>(a); break;
    case 2: sweep_colloc_kernel<K, __bf16><<<grid, 256, 0, st>>>(a); break;
    case 3: sweep_colloc_kernel<K, _Float16><<<grid, 256, 0, st>>>(a); break;
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
