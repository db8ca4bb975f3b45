// HIP kernels of libsldg for gfx950 (MI355X): the sLdG projection sweep
// (L. Einkemmer, arXiv 1603.07008, section II-A, update rule)
//     out[i] = A(alpha) in[i - s] + B(alpha) in[i - s - 1]
// along one dimension of a periodic tensor grid, on split storage (FP64 cell
// mean + narrower higher modes), plus the per-line table kernel and the
// compensated mass reduction.
//
// The sweep is a batched (k+1)x(k+1) contraction with 1-3 flop per byte moved,
// far below the machine balance, so it is HBM-bound: the kernels are built
// around coalesced plane reads (split mode-major storage keeps every mode plane
// contiguous along dimension 0) and each coefficient is read once and written
// once per sweep.  No matrix cores: the contraction is too small and too
// memory-bound for MFMA to matter.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ab_poly.h"
#include "sldg_internal.h"

namespace sldg {

// ---------------------------------------------------------------------------
// Storage tiers (section II-A: c_0 in FP64, the higher modes narrower)
// ---------------------------------------------------------------------------

template <int TIER> struct Tier;
template <> struct Tier<0> { using T = double;   using Acc = double; };
template <> struct Tier<1> { using T = float;    using Acc = double; };
template <> struct Tier<2> { using T = __bf16;   using Acc = float;  };
template <> struct Tier<3> { using T = _Float16; using Acc = float;  };

// Exact widening of a stored value to FP64 / FP32.
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return (double)v; }
__device__ __forceinline__ double widen(__bf16 v) { return (double)(float)v; }
__device__ __forceinline__ double widen(_Float16 v) { return (double)(float)v; }

// Round-to-nearest-even narrowing on store (hardware conversions on gfx950).
template <class T, class A> __device__ __forceinline__ T narrow(A v) { return (T)v; }

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

template <int K>
__global__ __launch_bounds__(256) void line_tables_kernel(int64_t n, int64_t period,
                                                          const double* __restrict__ sigma,
                                                          int32_t* __restrict__ s_out,
                                                          double* __restrict__ ab_out) {
  constexpr int O = K + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double sg = sigma[t];
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
  bool ok = isfinite(sg);
  if (ok) {
    double r = fmod(fs, (double)period);   // exact
    if (r < 0) r += (double)period;
    s = (int32_t)r;
  } else {
    alpha = __builtin_nan("");
    beta = alpha;
  }
  s_out[t] = s;
  double* A = ab_out + t * 2 * O * O;
  double* B = A + O * O;
#pragma unroll
  for (int j = 0; j < O; ++j) {
#pragma unroll
    for (int l = 0; l < O; ++l) {
      A[j * O + l] = horner_comp<K>(AbPoly<K>::A[j][l], alpha);
      B[j * O + l] = horner_comp<K>(AbPoly<K>::B[j][l], alpha);
    }
  }
  // Mass row made exact: int P_l over a cell vanishes for l >= 1, so the two
  // contributions of a source cell to the cell means must cancel exactly.
  A[0] = beta;
  B[0] = alpha;
#pragma unroll
  for (int l = 1; l < O; ++l) B[l] = -A[l];
}

hipError_t launch_line_tables(int k, int64_t n, int64_t period, const double* sigma,
                              int32_t* s_out, double* ab_out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (k) {
    case 1: line_tables_kernel<1><<<grid, block, 0, st>>>(n, period, sigma, s_out, ab_out); break;
    case 2: line_tables_kernel<2><<<grid, block, 0, st>>>(n, period, sigma, s_out, ab_out); break;
    case 3: line_tables_kernel<3><<<grid, block, 0, st>>>(n, period, sigma, s_out, ab_out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Line-table index
// ---------------------------------------------------------------------------

__device__ __forceinline__ int32_t table_index(const LineMap& m, int32_t lo, int32_t hi) {
  int32_t t = 0;
  for (int e = 0; e < m.nlo; ++e) t += ((lo / m.lo_div[e]) % m.lo_mod[e]) * m.lo_str[e];
  for (int e = 0; e < m.nhi; ++e) t += ((hi / m.hi_div[e]) % m.hi_mod[e]) * m.hi_str[e];
  return t;
}

// ---------------------------------------------------------------------------
// The per-cell update for one spectator tuple: o outputs from the o modes of
// the two source cells.  MASS: the tuple contains the cell mean (mode 0); its
// output is computed in FP64 from the exactly widened inputs.
// ---------------------------------------------------------------------------

template <int K, int TIER, bool MASS>
struct Cell {
  static constexpr int O = K + 1;
  using T = typename Tier<TIER>::T;
  using Acc = typename Tier<TIER>::Acc;

  const T* in[O];      // planes of the input modes j_dim = 0..k (in[0] unused if MASS)
  T* out[O];
  const double* in_mass;
  double* out_mass;
  double Ad[O][O], Bd[O][O];   // FP64 matrices (mass row and FP64 arithmetic)
  Acc Aa[O][O], Ba[O][O];      // matrices in the arithmetic type

  __device__ __forceinline__ void load_matrices(const double* ab) {
#pragma unroll
    for (int j = 0; j < O; ++j)
#pragma unroll
      for (int l = 0; l < O; ++l) {
        Ad[j][l] = ab[j * O + l];
        Bd[j][l] = ab[O * O + j * O + l];
        Aa[j][l] = (Acc)Ad[j][l];
        Ba[j][l] = (Acc)Bd[j][l];
      }
  }

  // Load the o modes of cell c as exact FP64 values.
  __device__ __forceinline__ void load(int64_t c, double (&v)[O]) const {
#pragma unroll
    for (int l = 0; l < O; ++l) {
      if (MASS && l == 0) v[l] = in_mass[c];
      else v[l] = widen(in[l][c]);
    }
  }

  __device__ __forceinline__ void update_store(int64_t c, const double (&x)[O],
                                               const double (&y)[O]) const {
#pragma unroll
    for (int j = 0; j < O; ++j) {
      if (MASS && j == 0) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < O; ++l) acc = fma(Ad[0][l], x[l], acc);
#pragma unroll
        for (int l = 0; l < O; ++l) acc = fma(Bd[0][l], y[l], acc);
        out_mass[c] = acc;
      } else {
        Acc acc = 0;
#pragma unroll
        for (int l = 0; l < O; ++l) acc = fma(Aa[j][l], (Acc)x[l], acc);
#pragma unroll
        for (int l = 0; l < O; ++l) acc = fma(Ba[j][l], (Acc)y[l], acc);
        out[j][c] = narrow<T>(acc);
      }
    }
  }

  __device__ __forceinline__ void bind(const SweepArgs& a, int64_t m0, int32_t mstride) {
    const T* hin = reinterpret_cast<const T*>(a.in_hi);
    T* hout = reinterpret_cast<T*>(a.out_hi);
#pragma unroll
    for (int l = 0; l < O; ++l) {
      const int64_t m = m0 + (int64_t)l * mstride;
      const int64_t off = (m - 1) * a.cells;      // mode m >= 1 lives at plane m-1
      in[l] = (MASS && l == 0) ? nullptr : hin + off;
      out[l] = (MASS && l == 0) ? nullptr : hout + off;
    }
    in_mass = a.in_mass;
    out_mass = a.out_mass;
  }
};

// ---------------------------------------------------------------------------
// Sweep along dimension 0 (contiguous).  One wave per (line, spectator tuple):
// the line's s, A and B are wave-uniform (scalar registers), lanes walk the
// line's cells, so every plane access of a wave is one contiguous run with a
// periodic wrap.  The second source cell of lane L is the first one of lane
// L-1, so the reuse is served by the vector L1.
// ---------------------------------------------------------------------------

template <int K, int TIER, bool MASS>
__device__ __forceinline__ void contig_line(const SweepArgs& a, int64_t line, int32_t sp,
                                            int lane) {
  constexpr int O = K + 1;
  Cell<K, TIER, MASS> cell;
  const int32_t t = __builtin_amdgcn_readfirstlane(table_index(a.map, 0, (int32_t)line));
  const int32_t s = __builtin_amdgcn_readfirstlane(a.s_tab[t]);
  cell.load_matrices(a.ab_tab + (int64_t)t * 2 * O * O);
  cell.bind(a, (int64_t)sp * O, 1);
  const int32_t N = a.N;
  const int64_t base = line * (int64_t)N;
  for (int32_t i = lane; i < N; i += 64) {
    int32_t ia = i - s;
    if (ia < 0) ia += N;
    int32_t ib = ia - 1;
    if (ib < 0) ib += N;
    double x[O], y[O];
    cell.load(base + ia, x);
    cell.load(base + ib, y);
    cell.update_store(base + i, x, y);
  }
}

template <int K, int TIER>
__global__ __launch_bounds__(256) void sweep_contig_kernel(SweepArgs a) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t nlines = (int64_t)a.Q;
  const int64_t item = (int64_t)blockIdx.x * 4 + wave;
  if (item >= nlines * a.nspec) return;
  const int32_t sp = (int32_t)(item / nlines);
  const int64_t line = item - (int64_t)sp * nlines;
  if (sp == 0) contig_line<K, TIER, true>(a, line, sp, lane);
  else contig_line<K, TIER, false>(a, line, sp, lane);
}

// ---------------------------------------------------------------------------
// Sweep along a dimension d > 0 (strided).  Lanes take consecutive cells of
// the flattened lower dimensions (contiguous in memory); each thread streams
// along its line through a chunk of rows keeping the previous source row in
// registers, so every input row of the chunk is read once.  The displacement
// (and so s, A, B) may differ from lane to lane.
// ---------------------------------------------------------------------------

template <int K, int TIER, bool MASS>
__device__ __forceinline__ void strided_run(const SweepArgs& a, int32_t ilow, int32_t chunk,
                                            int32_t ihigh, int32_t sp) {
  constexpr int O = K + 1;
  Cell<K, TIER, MASS> cell;
  const int32_t t = table_index(a.map, ilow, ihigh);
  const int32_t s = a.s_tab[t];
  cell.load_matrices(a.ab_tab + (int64_t)t * 2 * O * O);
  const int32_t ms = a.mstride;
  const int64_t m0 = (int64_t)(sp % ms) + (int64_t)(sp / ms) * ms * O;
  cell.bind(a, m0, ms);
  const int32_t N = a.N, P = a.P;
  const int64_t base = (int64_t)ihigh * P * N + ilow;
  const int32_t r0 = chunk * a.chunk;
  const int32_t r1 = min(N, r0 + a.chunk);
  int32_t iy = r0 - s - 1;
  if (iy < 0) iy += N;
  if (iy < 0) iy += N;
  double y[O];
  cell.load(base + (int64_t)iy * P, y);
  int32_t ix = iy + 1;
  if (ix == N) ix = 0;
  for (int32_t i = r0; i < r1; ++i) {
    double x[O];
    cell.load(base + (int64_t)ix * P, x);
    cell.update_store(base + (int64_t)i * P, x, y);
#pragma unroll
    for (int l = 0; l < O; ++l) y[l] = x[l];
    if (++ix == N) ix = 0;
  }
}

template <int K, int TIER>
__global__ __launch_bounds__(256) void sweep_strided_kernel(SweepArgs a) {
  const int32_t sp = blockIdx.y;
  const int64_t per = (int64_t)a.P * a.nchunk * a.Q;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= per) return;
  const int32_t ilow = (int32_t)(tid % a.P);
  const int64_t r = tid / a.P;
  const int32_t chunk = (int32_t)(r % a.nchunk);
  const int32_t ihigh = (int32_t)(r / a.nchunk);
  if (sp == 0) strided_run<K, TIER, true>(a, ilow, chunk, ihigh, sp);
  else strided_run<K, TIER, false>(a, ilow, chunk, ihigh, sp);
}

template <int K, int TIER>
static hipError_t launch_sweep_kt(int dim, const SweepArgs& a, hipStream_t st) {
  if (dim == 0) {
    const int64_t items = (int64_t)a.Q * a.nspec;
    dim3 grid((unsigned)((items + 3) / 4)), block(256);
    sweep_contig_kernel<K, TIER><<<grid, block, 0, st>>>(a);
  } else {
    const int64_t per = (int64_t)a.P * a.nchunk * a.Q;
    dim3 grid((unsigned)((per + 255) / 256), (unsigned)a.nspec), block(256);
    sweep_strided_kernel<K, TIER><<<grid, block, 0, st>>>(a);
  }
  return hipGetLastError();
}

template <int K>
static hipError_t launch_sweep_k(int tier, int dim, const SweepArgs& a, hipStream_t st) {
  switch (tier) {
    case 0: return launch_sweep_kt<K, 0>(dim, a, st);
    case 1: return launch_sweep_kt<K, 1>(dim, a, st);
    case 2: return launch_sweep_kt<K, 2>(dim, a, st);
    case 3: return launch_sweep_kt<K, 3>(dim, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sweep(int k, int tier, int dim, const SweepArgs& a, hipStream_t st) {
  switch (k) {
    case 1: return launch_sweep_k<1>(tier, dim, a, st);
    case 2: return launch_sweep_k<2>(tier, dim, a, st);
    case 3: return launch_sweep_k<3>(tier, dim, a, st);
    default: return hipErrorInvalidValue;
  }
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
