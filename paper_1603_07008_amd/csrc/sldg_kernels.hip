// HIP kernels of libsldg for gfx950 (MI355X) beside the sweeps themselves:
// the per-line tables of the sLdG projection sweep (L. Einkemmer, arXiv
// 1603.07008, section II-A, update rule), the dispatch of the sweep
// launches over (degree, storage tier), the scaled FP16 bookkeeping, the
// reference copies and the compensated mass reduction.  The sweep kernels
// are in sldg_sweep.h, instantiated by sldg_sweep_inst.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "ab_poly.h"
#include "sldg_internal.h"
#include "sldg_sweep.h"

namespace sldg {

// ---------------------------------------------------------------------------
// Per-line tables (section II-A: s and the matrices A, B for each line)
// ---------------------------------------------------------------------------

// Compensated Horner scheme (S. Graillat, P. Langlois, N. Louvet, "Compensated
// Horner scheme", 2005): Horner's rule with the rounding error of every
// product (FMA-based TwoProduct) and sum (TwoSum) carried in a second
// accumulator.  The result is as accurate as Horner in twice the working
// precision, then rounded, so the matrix entries come out within an ulp of the
// exact values even where the integer coefficients (up to ~500 for k = 3)
// cancel heavily; at dyadic alpha (0, 1/2, ...) every step is exact.
template <int K>
__device__ __forceinline__ double horner_comp(const double (&c)[2 * K + 2], double x) {
#pragma clang fp contract(off)
  double r = c[2 * K + 1];
  double err = 0.0;
#pragma unroll
  for (int p = 2 * K; p >= 0; --p) {
    const double prod = r * x;
    const double pe = fma(r, x, -prod);       // exact error of the product
    const double sum = prod + c[p];
    const double bb = sum - prod;
    const double se = (prod - (sum - bb)) + (c[p] - bb);   // exact error of the sum
    err = fma(err, x, pe + se);
    r = sum;
  }
  return r + err;
}

// Table layout: entry t, component e (A row-major, then B row-major) at
// ab_out[e * cs + t * ts]: (cs, ts) = (1, 2(k+1)^2) is entry-major (the public
// layout), (n, 1) component-major (used by the sweeps, so that lanes reading
// the matrices of consecutive lines touch consecutive addresses).
//
// ADJ: the table of the transposed sweep.  The forward sweep of one line,
// out[i] = A in[i-s] + B in[i-s-1], has the transpose
// g_in[m] = A^T g[m+s] + B^T g[m+s+1], which is again a forward-form sweep
// with shift s' = -s-1 and matrices (A', B') = (B^T, A^T).  It is built from
// the same (snapped, exact-mass-row) A and B, so it is the exact transpose of
// the forward map.
template <int K, bool ADJ>
__device__ __forceinline__ void line_table_entry(int64_t t, double sg, int64_t period,
                                                 int32_t* __restrict__ s_out,
                                                 double* __restrict__ ab_out, int64_t cs,
                                                 int64_t ts) {
  constexpr int O = K + 1;
  double fs = floor(sg);
  double alpha = sg - fs;
  const double beta0 = 1.0 - alpha;
  alpha = 1.0 - beta0;             // alpha + beta == 1 exactly (Sterbenz)
  double beta = beta0;
  if (alpha >= 1.0) {              // fractional part rounded up to 1
    fs += 1.0;
    alpha = 0.0;
    beta = 1.0;
  }
  int32_t s = 0;
  if (isfinite(sg)) {
    double r = fmod(ADJ ? -fs - 1.0 : fs, (double)period);   // exact
    if (r < 0) r += (double)period;
    s = (int32_t)r;
  } else {
    alpha = __builtin_nan("");
    beta = alpha;
  }
  s_out[t] = s;
  double A[O][O], B[O][O];
#pragma unroll
  for (int j = 0; j < O; ++j) {
#pragma unroll
    for (int l = 0; l < O; ++l) {
      A[j][l] = horner_comp<K>(AbPoly<K>::A[j][l], alpha);
      B[j][l] = horner_comp<K>(AbPoly<K>::B[j][l], alpha);
    }
  }
  // Mass row made exact: int P_l over a cell vanishes for l >= 1, so the two
  // contributions of a source cell to the cell means must cancel exactly.
  A[0][0] = beta;
  B[0][0] = alpha;
#pragma unroll
  for (int l = 1; l < O; ++l) B[0][l] = -A[0][l];
  double* base = ab_out + t * ts;
#pragma unroll
  for (int j = 0; j < O; ++j)
#pragma unroll
    for (int l = 0; l < O; ++l) {
      base[(j * O + l) * cs] = ADJ ? B[l][j] : A[j][l];
      base[(O * O + j * O + l) * cs] = ADJ ? A[l][j] : B[j][l];
    }
}

template <int K, bool ADJ>
__global__ __launch_bounds__(256) void line_tables_kernel(int64_t n, int64_t period,
                                                          const double* __restrict__ sigma,
                                                          int32_t* __restrict__ s_out,
                                                          double* __restrict__ ab_out,
                                                          int64_t cs, int64_t ts) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  line_table_entry<K, ADJ>(t, sigma[t], period, s_out, ab_out, cs, ts);
}

// The tables of several sweeps (forward, component-major) in one launch:
// entry t of the flat range belongs to sweep q with first[q] <= t <
// first[q + 1]; sweep q's table is the one line_tables_kernel writes, at
// s_out + first[q] and ab_out + 2 (k+1)^2 first[q].
template <int K>
__global__ __launch_bounds__(256) void line_tables_set_kernel(TableSet set,
                                                              int32_t* __restrict__ s_out,
                                                              double* __restrict__ ab_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= set.first[set.count]) return;
  int q = 0;
  while (q + 1 < set.count && t >= set.first[q + 1]) ++q;
  const int64_t f = set.first[q], n = set.first[q + 1] - f;
  line_table_entry<K, false>(t - f, set.sigma[q][t - f], set.period[q], s_out + f,
                             ab_out + 2LL * (K + 1) * (K + 1) * f, n, 1);
}

hipError_t launch_line_tables(int k, int64_t n, int64_t period, const double* sigma,
                              int32_t* s_out, double* ab_out, bool component_major,
                              bool adjoint, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t e = 2LL * (k + 1) * (k + 1);
  const int64_t cs = component_major ? n : 1, ts = component_major ? 1 : e;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define SLDG_TABLES(KK, AA) line_tables_kernel<KK, AA><<<grid, block, 0, st>>>(n, period, sigma, s_out, ab_out, cs, ts)
  switch (k * 2 + (adjoint ? 1 : 0)) {
    case 2: SLDG_TABLES(1, false); break;
    case 3: SLDG_TABLES(1, true); break;
    case 4: SLDG_TABLES(2, false); break;
    case 5: SLDG_TABLES(2, true); break;
    case 6: SLDG_TABLES(3, false); break;
    case 7: SLDG_TABLES(3, true); break;
    default: return hipErrorInvalidValue;
  }
#undef SLDG_TABLES
  return hipGetLastError();
}

hipError_t launch_line_tables_set(int k, const TableSet& set, int32_t* s_out, double* ab_out,
                                  hipStream_t st) {
  const int64_t n = set.first[set.count];
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (k) {
    case 1: line_tables_set_kernel<1><<<grid, block, 0, st>>>(set, s_out, ab_out); break;
    case 2: line_tables_set_kernel<2><<<grid, block, 0, st>>>(set, s_out, ab_out); break;
    case 3: line_tables_set_kernel<3><<<grid, block, 0, st>>>(set, s_out, ab_out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool contig_window_ok(const SweepArgs& a) {
  const uintptr_t align = (uintptr_t)a.in_lo | (uintptr_t)a.in_hi | (uintptr_t)a.out_lo |
                          (uintptr_t)a.out_hi;
  return a.N % 4 == 0 && (align & 15) == 0;
}

int sweep_form(int dim, const SweepArgs& a) {
  int form;
  dim3 grid, block;
  if (!sweep_grid(dim, a, form, grid, block)) return -1;
  return form == 2 && a.stage && block.x == 256 ? 4 : form;
}

int64_t sweep_slots(int dim, const SweepArgs& a) {
  int form;
  dim3 grid, block;
  if (!sweep_grid(dim, a, form, grid, block)) return -1;
  if (form != 2) return (int64_t)grid.x * (block.x / 64);
  return (int64_t)grid.x * grid.z * (block.x / 64);
}

hipError_t launch_sweep(int k, int tier, int dim, const SweepArgs& a, hipStream_t st) {
#define SLDG_SWEEP_CALL(KK, TT) launch_sweep_inst<KK, TT>(dim, a, st)
  switch (k) {
    case 1:
      switch (tier) {
        case 0: return SLDG_SWEEP_CALL(1, 0);
        case 1: return SLDG_SWEEP_CALL(1, 1);
        case 2: return SLDG_SWEEP_CALL(1, 2);
        case 3: return SLDG_SWEEP_CALL(1, 3);
      }
      break;
    case 2:
      switch (tier) {
        case 0: return SLDG_SWEEP_CALL(2, 0);
        case 1: return SLDG_SWEEP_CALL(2, 1);
        case 2: return SLDG_SWEEP_CALL(2, 2);
        case 3: return SLDG_SWEEP_CALL(2, 3);
      }
      break;
    case 3:
      switch (tier) {
        case 0: return SLDG_SWEEP_CALL(3, 0);
        case 1: return SLDG_SWEEP_CALL(3, 1);
        case 2: return SLDG_SWEEP_CALL(3, 2);
        case 3: return SLDG_SWEEP_CALL(3, 3);
      }
      break;
  }
#undef SLDG_SWEEP_CALL
  return hipErrorInvalidValue;
}

hipError_t launch_xy(int k, int tier, const XYArgs& a, int64_t lds_bytes, int32_t nblocks,
                     hipStream_t st) {
#define SLDG_XY_CALL(KK, TT) launch_xy_inst<KK, TT>(a, lds_bytes, nblocks, st)
  switch (k) {
    case 1:
      switch (tier) {
        case 0: return SLDG_XY_CALL(1, 0);
        case 1: return SLDG_XY_CALL(1, 1);
        case 2: return SLDG_XY_CALL(1, 2);
        case 3: return SLDG_XY_CALL(1, 3);
      }
      break;
    case 2:
      switch (tier) {
        case 0: return SLDG_XY_CALL(2, 0);
        case 1: return SLDG_XY_CALL(2, 1);
        case 2: return SLDG_XY_CALL(2, 2);
        case 3: return SLDG_XY_CALL(2, 3);
      }
      break;
    case 3:
      switch (tier) {
        case 0: return SLDG_XY_CALL(3, 0);
        case 1: return SLDG_XY_CALL(3, 1);
        case 2: return SLDG_XY_CALL(3, 2);
        case 3: return SLDG_XY_CALL(3, 3);
      }
      break;
  }
#undef SLDG_XY_CALL
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Batched sweep: many independent problems (own grid, degree and tables).
// The work list of a sweep holds one item per workgroup-sized tile of one
// problem, grouped by class (tile kind and degree).  Each class is one
// launch of a kernel compiled for that kind and degree alone (one workgroup
// per item, XCD-aware order), so no kernel carries the registers of the
// other code paths; the classes of a split step are captured together in one
// HIP graph.  Kinds: 0 dimension-0 window form (256 groups of 4 cells),
// 1 dimension-0 group form (256 groups of 4 interleaved cells), 2 strided
// (64 columns x 4 row chunks); kinds 1 and 2 run in the lane form (256
// consecutive cells, kernel kind 3) when their class's rows are 1 and 0.  A
// run of spectator tuples is part of the item.
// ---------------------------------------------------------------------------

hipError_t launch_batch_class(int tier, int k, int kind, int rows, const SweepArgs* args,
                              const BatchItem* items, int32_t nitems, int32_t xcd,
                              hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
#define SLDG_CLASS_CALL(KK, TT) launch_class_inst<KK, TT>(kind, rows, args, items, nitems, xcd, st)
  switch (k) {
    case 1:
      switch (tier) {
        case 0: return SLDG_CLASS_CALL(1, 0);
        case 1: return SLDG_CLASS_CALL(1, 1);
        case 2: return SLDG_CLASS_CALL(1, 2);
        case 3: return SLDG_CLASS_CALL(1, 3);
      }
      break;
    case 2:
      switch (tier) {
        case 0: return SLDG_CLASS_CALL(2, 0);
        case 1: return SLDG_CLASS_CALL(2, 1);
        case 2: return SLDG_CLASS_CALL(2, 2);
        case 3: return SLDG_CLASS_CALL(2, 3);
      }
      break;
    case 3:
      switch (tier) {
        case 0: return SLDG_CLASS_CALL(3, 0);
        case 1: return SLDG_CLASS_CALL(3, 1);
        case 2: return SLDG_CLASS_CALL(3, 2);
        case 3: return SLDG_CLASS_CALL(3, 3);
      }
      break;
  }
#undef SLDG_CLASS_CALL
  return hipErrorInvalidValue;
}


// ---------------------------------------------------------------------------
// Scaled FP16 storage: exponent prediction, absmax decision, overflow redo,
// import from and export to FP64.
// ---------------------------------------------------------------------------

constexpr int kFp16Top = 15;             // 2^15 <= 65504 < 2^16
constexpr int kScaleEmin = -100, kScaleEmax = 100;
constexpr int kRepairHeadroom = 1;

// Exponent e with 2^(14 - h) <= amax 2^e < 2^(15 - h), clamped; `keep` when
// amax is 0 or not finite.
__device__ __forceinline__ int32_t storage_exponent(float amax, int headroom, int32_t keep) {
  if (!(amax > 0.0f) || !isfinite(amax)) return keep;
  int x;
  (void)frexpf(amax, &x);                // amax = f 2^x, 0.5 <= f < 1
  return min(max(kFp16Top - headroom - x, kScaleEmin), kScaleEmax);
}

__global__ __launch_bounds__(256) void scale_predict_kernel(int64_t n_hi,
                                                            const int32_t* __restrict__ in_exp,
                                                            const float* __restrict__ in_amax,
                                                            int32_t* __restrict__ out_exp,
                                                            int headroom,
                                                            float* __restrict__ part,
                                                            int64_t npart,
                                                            int32_t* __restrict__ nredo) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (i0 == 0) *nredo = 0;
  for (int64_t p = i0; p < n_hi; p += stride)
    out_exp[p] = storage_exponent(in_amax[p], headroom, in_exp[p]);
  for (int64_t i = i0; i < npart; i += stride) part[i] = 0.0f;
}

hipError_t launch_scale_predict(int64_t n_hi, const int32_t* in_exp, const float* in_amax,
                                int32_t* out_exp, int headroom, float* part, int64_t npart,
                                int32_t* nredo, hipStream_t st) {
  const int64_t need = std::max(n_hi, npart);
  const unsigned blocks = (unsigned)std::min<int64_t>(2048, std::max<int64_t>(1, (need + 255) / 256));
  scale_predict_kernel<<<blocks, 256, 0, st>>>(n_hi, in_exp, in_amax, out_exp, headroom, part,
                                               npart, nredo);
  return hipGetLastError();
}

__device__ __forceinline__ float block_max(float v, float* sh) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = 0.0f;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmaxf(r, sh[w]);
  return r;
}

// One workgroup of 1024 threads per plane; four independent maxima per
// thread keep several loads in flight (fmaxf ignores NaN operands, and the
// maximum does not depend on the order).
constexpr int kDecideThreads = 1024;

__global__ __launch_bounds__(kDecideThreads) void scale_decide_kernel(
    const float* __restrict__ part, int32_t nslot, int32_t* __restrict__ out_exp,
    float* __restrict__ out_amax, int32_t* __restrict__ redo, int32_t* __restrict__ nredo) {
  __shared__ float sh[kDecideThreads / 64];
  const int64_t p = blockIdx.x;
  const float* q = part + p * nslot;
  const int32_t step = (int32_t)blockDim.x;
  float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f, m3 = 0.0f;
  int32_t i = threadIdx.x;
  for (; i + 3 * step < nslot; i += 4 * step) {
    m0 = fmaxf(m0, q[i]);
    m1 = fmaxf(m1, q[i + step]);
    m2 = fmaxf(m2, q[i + 2 * step]);
    m3 = fmaxf(m3, q[i + 3 * step]);
  }
  for (; i < nslot; i += step) m0 = fmaxf(m0, q[i]);
  float m = fmaxf(fmaxf(m0, m1), fmaxf(m2, m3));
  m = block_max(m, sh);
  if (threadIdx.x == 0) {
    const int32_t e = out_exp[p];
    int32_t fix = 0;
    if (isfinite(m) && ldexp((double)m, e) >= (double)(1 << kFp16Top)) {
      out_exp[p] = storage_exponent(m, kRepairHeadroom, e);
      fix = 1;
    }
    out_amax[p] = m;
    redo[p] = fix;
    if (fix) atomicAdd(nredo, 1);
  }
}

hipError_t launch_scale_decide(int64_t n_hi, const float* part, int32_t nslot, int32_t* out_exp,
                               float* out_amax, int32_t* redo, int32_t* nredo, hipStream_t st) {
  if (n_hi <= 0) return hipSuccess;
  scale_decide_kernel<<<(unsigned)n_hi, kDecideThreads, 0, st>>>(part, nslot, out_exp, out_amax,
                                                                 redo, nredo);
  return hipGetLastError();
}

// Recompute the flagged planes (outputs that overflowed their predicted
// exponent) with their final exponents: every workgroup lists the flagged
// planes in LDS, exits when there is none, and walks the cells of each with a
// grid stride.  The update is the same sequence of operations as in the sweep
// kernels (FP32 accumulation of the widened, unscaled inputs).
template <int K>
__global__ __launch_bounds__(256) void scale_redo_kernel(SweepArgs a, int32_t n_hi,
                                                         const int32_t* __restrict__ redo,
                                                         const int32_t* __restrict__ nredo,
                                                         const int32_t* __restrict__ hi_mode) {
  constexpr int O = K + 1;
  constexpr int kList = 4096;          // >= the most narrow planes of a plan (4^6 - 1)
  __shared__ int32_t list[kList];
  __shared__ int32_t count;
  // the decision kernel counted the flagged planes: usually none, and then
  // every workgroup leaves after one load
  if (__builtin_amdgcn_readfirstlane(*nredo) == 0) return;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  for (int32_t p = threadIdx.x; p < n_hi; p += blockDim.x)
    if (redo[p]) {
      const int32_t i = atomicAdd(&count, 1);
      if (i < kList) list[i] = p;
    }
  __syncthreads();
  const int32_t nfix = min(count, kList);
  if (nfix == 0) return;
  const _Float16* hin = reinterpret_cast<const _Float16*>(a.in_hi);
  _Float16* hout = reinterpret_cast<_Float16*>(a.out_hi);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int32_t ms = a.mstride;
  for (int32_t f = 0; f < nfix; ++f) {
    const int32_t p = list[f];
    const int32_t m = hi_mode[p];
    const int32_t j = (m / ms) % O;
    const int32_t m0 = m - j * ms;
    int32_t src[O];
    float fin[O];
#pragma unroll
    for (int l = 0; l < O; ++l) {
      src[l] = a.pmap[m0 + l * ms];
      fin[l] = src[l] >= 0 ? pow2f(-a.in_exp[src[l]]) : 1.0f;
    }
    const float fout = pow2f(a.out_exp[p]);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.cells; c += stride) {
      const int32_t ilow = (int32_t)(c % a.P);
      const int64_t rest = c / a.P;
      const int32_t id = (int32_t)(rest % a.N);
      const int32_t ihigh = (int32_t)(rest / a.N);
      const int32_t t = table_index(a.map, ilow, ihigh);
      const int32_t s = a.s_tab[t];
      int32_t ia = id - s;
      if (ia < 0) ia += a.N;
      int32_t ib = ia - 1;
      if (ib < 0) ib += a.N;
      const int64_t base = (int64_t)ihigh * a.P * a.N + ilow;
      const int64_t ca = base + (int64_t)ia * a.P, cb = base + (int64_t)ib * a.P;
      float x[O], y[O];
#pragma unroll
      for (int l = 0; l < O; ++l) {
        if (src[l] >= 0) {
          x[l] = (float)hin[(int64_t)src[l] * a.cells + ca] * fin[l];
          y[l] = (float)hin[(int64_t)src[l] * a.cells + cb] * fin[l];
        } else {
          x[l] = (float)a.in_lo[(int64_t)(-1 - src[l]) * a.cells + ca];
          y[l] = (float)a.in_lo[(int64_t)(-1 - src[l]) * a.cells + cb];
        }
      }
      float acc = 0.0f;
#pragma unroll
      for (int l = 0; l < O; ++l) acc = fma((float)a.ab_tab[(j * O + l) * a.ab_cs + t], x[l], acc);
#pragma unroll
      for (int l = 0; l < O; ++l)
        acc = fma((float)a.ab_tab[(O * O + j * O + l) * a.ab_cs + t], y[l], acc);
      hout[(int64_t)p * a.cells + c] = (_Float16)(acc * fout);
    }
  }
}

hipError_t launch_scale_redo(int k, int dim, const SweepArgs& a, int64_t n_hi,
                             const int32_t* redo, const int32_t* nredo, const int32_t* hi_mode, hipStream_t st) {
  (void)dim;
  if (n_hi <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (a.cells + 255) / 256));
  switch (k) {
    case 1: scale_redo_kernel<1><<<blocks, 256, 0, st>>>(a, (int32_t)n_hi, redo, nredo, hi_mode); break;
    case 2: scale_redo_kernel<2><<<blocks, 256, 0, st>>>(a, (int32_t)n_hi, redo, nredo, hi_mode); break;
    case 3: scale_redo_kernel<3><<<blocks, 256, 0, st>>>(a, (int32_t)n_hi, redo, nredo, hi_mode); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// FP64 -> FP16 with one rounding to nearest even: the value is first taken to
// FP32 by rounding to odd (truncate, then set the last bit when inexact),
// which keeps enough information for the final RNE step to FP16 (24 > 11 + 1
// significant bits) to be correctly rounded.
__device__ __forceinline__ _Float16 f64_to_f16_rne(double v) {
  float f = (float)v;                              // RNE
  if (isfinite(f) && (double)f != v) {
    uint32_t b = __float_as_uint(f);
    if (fabs((double)f) > fabs(v)) b -= 1;         // rounded away from zero: step back
    f = __uint_as_float(b | 1u);                   // inexact: odd last bit
  } else if (!isfinite(f) && isfinite(v)) {
    f = v > 0 ? 3.4028234663852886e38f : -3.4028234663852886e38f;   // beyond FP32: FP16 inf
  }
  return (_Float16)f;
}

// Absmax partials of an FP64 array [n_hi][cells]: grid (nslot, n_hi).
__global__ __launch_bounds__(256) void import_absmax_kernel(const double* __restrict__ src,
                                                            int64_t cells,
                                                            float* __restrict__ part) {
  __shared__ float sh[4];
  const int64_t p = blockIdx.y;
  double m = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells;
       c += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(src[p * cells + c]));
  // FP32 rounding is monotonic, so the max of rounded values is the rounded max
  const float r = block_max((float)m, sh);
  if (threadIdx.x == 0) part[p * gridDim.x + blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void import_exp_kernel(const float* __restrict__ part,
                                                         int32_t nslot, int headroom,
                                                         int32_t* __restrict__ exp,
                                                         float* __restrict__ amax) {
  __shared__ float sh[4];
  const int64_t p = blockIdx.x;
  float m = 0.0f;
  for (int32_t i = threadIdx.x; i < nslot; i += blockDim.x) m = fmaxf(m, part[p * nslot + i]);
  m = block_max(m, sh);
  if (threadIdx.x == 0) {
    exp[p] = storage_exponent(m, headroom, 0);
    amax[p] = m;
  }
}

__global__ __launch_bounds__(256) void import_convert_kernel(const double* __restrict__ src,
                                                             int64_t n, int64_t cells,
                                                             const int32_t* __restrict__ exp,
                                                             _Float16* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = f64_to_f16_rne(ldexp(src[i], exp[i / cells]));
}

hipError_t launch_scale_import(const double* src, int64_t n_hi, int64_t cells, int headroom,
                               float* part, int32_t nslot, void* dst, int32_t* exp, float* amax,
                               hipStream_t st) {
  if (n_hi <= 0) return hipSuccess;
  if (n_hi > 65535) return hipErrorInvalidConfiguration;
  import_absmax_kernel<<<dim3((unsigned)nslot, (unsigned)n_hi), 256, 0, st>>>(src, cells, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  import_exp_kernel<<<(unsigned)n_hi, 256, 0, st>>>(part, nslot, headroom, exp, amax);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = n_hi * cells;
  const unsigned blocks = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (n + 255) / 256));
  import_convert_kernel<<<blocks, 256, 0, st>>>(src, n, cells, exp,
                                                static_cast<_Float16*>(dst));
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void export_kernel(const _Float16* __restrict__ src, int64_t n,
                                                     int64_t cells,
                                                     const int32_t* __restrict__ exp,
                                                     double* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = ldexp((double)(float)src[i], -exp[i / cells]);
}

hipError_t launch_scale_export(const void* src, int64_t n_hi, int64_t cells, const int32_t* exp,
                               double* dst, hipStream_t st) {
  const int64_t n = n_hi * cells;
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (n + 255) / 256));
  export_kernel<<<blocks, 256, 0, st>>>(static_cast<const _Float16*>(src), n, cells, exp, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain copy (reference bandwidth): one 16-byte load and store per thread.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void copy16_kernel(const uint4* __restrict__ src,
                                                     uint4* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t st) {
  if (n16 <= 0) return hipSuccess;
  const int64_t blocks = (n16 + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  copy16_kernel<<<(unsigned)blocks, 256, 0, st>>>(static_cast<const uint4*>(src),
                                                  static_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mass: deterministic double-double (compensated) reduction of the FP64 mass
// array (section II-A: c_0 carries the mass).
// ---------------------------------------------------------------------------

struct DD { double hi, lo; };

__device__ __forceinline__ DD two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__device__ __forceinline__ DD dd_add(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi);
  const double e = s.lo + (a.lo + b.lo);
  const double hi = s.hi + e;                 // fast two-sum renormalisation
  return {hi, e - (hi - s.hi)};
}

__device__ __forceinline__ DD dd_add(DD a, double b) {
  DD s = two_sum(a.hi, b);
  const double e = s.lo + a.lo;
  const double hi = s.hi + e;
  return {hi, e - (hi - s.hi)};
}

constexpr int kMassThreads = 256;
constexpr int kMassMaxBlocks = 1024;

int mass_blocks(int64_t n) {
  int64_t b = (n + kMassThreads - 1) / kMassThreads;
  if (b > kMassMaxBlocks) b = kMassMaxBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

__device__ __forceinline__ DD block_reduce(DD v, DD* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kMassThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = dd_add(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(kMassThreads) void mass_partial_kernel(const double* __restrict__ m,
                                                                    int64_t n,
                                                                    double* __restrict__ part) {
  __shared__ DD sh[kMassThreads];
  DD acc = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kMassThreads;
  for (int64_t i = (int64_t)blockIdx.x * kMassThreads + threadIdx.x; i < n; i += stride)
    acc = dd_add(acc, m[i]);
  DD r = block_reduce(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r.hi;
    part[2 * blockIdx.x + 1] = r.lo;
  }
}

__global__ __launch_bounds__(kMassThreads) void mass_final_kernel(const double* __restrict__ part,
                                                                  int nb, double* __restrict__ out) {
  __shared__ DD sh[kMassThreads];
  DD acc = {0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kMassThreads) acc = dd_add(acc, DD{part[2 * b], part[2 * b + 1]});
  DD r = block_reduce(acc, sh);
  if (threadIdx.x == 0) {
    out[0] = r.hi;
    out[1] = r.lo;
  }
}

hipError_t launch_mass(const double* mass, int64_t n, double* partial, int nblocks,
                       double* result, hipStream_t st) {
  mass_partial_kernel<<<nblocks, kMassThreads, 0, st>>>(mass, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mass_final_kernel<<<1, kMassThreads, 0, st>>>(partial, nblocks, result);
  return hipGetLastError();
}

}  // namespace sldg
