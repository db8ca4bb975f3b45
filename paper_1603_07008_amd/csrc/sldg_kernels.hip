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
// Raw storage of one cell's o modes (along the swept dimension) and the
// arithmetic on it.  Values stay in their storage type in registers and are
// widened exactly when used.
// ---------------------------------------------------------------------------

template <int K, int TIER, bool MASS>
struct Raw {
  static constexpr int O = K + 1;
  using T = typename Tier<TIER>::T;
  double m;   // mode j = 0 when MASS
  T h[O];     // modes (h[0] unused when MASS)
};

template <int K, int TIER, bool MASS>
struct Mat {
  static constexpr int O = K + 1;
  using T = typename Tier<TIER>::T;
  using Acc = typename Tier<TIER>::Acc;
  double Ad[O], Bd[O];         // mass row in FP64 (used when MASS)
  Acc Aa[O][O], Ba[O][O];      // all rows in the arithmetic type

  __device__ __forceinline__ void load(const double* ab) {
#pragma unroll
    for (int j = 0; j < O; ++j)
#pragma unroll
      for (int l = 0; l < O; ++l) {
        Aa[j][l] = (Acc)ab[j * O + l];
        Ba[j][l] = (Acc)ab[O * O + j * O + l];
      }
#pragma unroll
    for (int l = 0; l < O; ++l) {
      Ad[l] = ab[l];
      Bd[l] = ab[O * O + l];
    }
  }

  __device__ __forceinline__ static double wide(const Raw<K, TIER, MASS>& r, int l) {
    return (MASS && l == 0) ? r.m : widen(r.h[l]);
  }
  __device__ __forceinline__ static Acc acc_of(const Raw<K, TIER, MASS>& r, int l) {
    if (MASS && l == 0) return (Acc)r.m;
    if constexpr (sizeof(Acc) == 8) return widen(r.h[l]);
    else return (Acc)r.h[l];
  }

  // Output mode j of the update from the two source cells x (cell i-s) and
  // y (cell i-s-1).  The mass row of a MASS tuple is FP64 throughout.
  __device__ __forceinline__ double mass_out(const Raw<K, TIER, MASS>& x,
                                             const Raw<K, TIER, MASS>& y) const {
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < O; ++l) acc = fma(Ad[l], wide(x, l), acc);
#pragma unroll
    for (int l = 0; l < O; ++l) acc = fma(Bd[l], wide(y, l), acc);
    return acc;
  }
  __device__ __forceinline__ T hi_out(int j, const Raw<K, TIER, MASS>& x,
                                      const Raw<K, TIER, MASS>& y) const {
    Acc acc = 0;
#pragma unroll
    for (int l = 0; l < O; ++l) acc = fma(Aa[j][l], acc_of(x, l), acc);
#pragma unroll
    for (int l = 0; l < O; ++l) acc = fma(Ba[j][l], acc_of(y, l), acc);
    return narrow<T>(acc);
  }
};

// Plane pointers of one spectator tuple: mode m0 + l*mstride for l = 0..k.
template <int K, int TIER, bool MASS>
struct Planes {
  static constexpr int O = K + 1;
  using T = typename Tier<TIER>::T;
  const T* in[O];
  T* out[O];
  const double* in_mass;
  double* out_mass;

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
  __device__ __forceinline__ void load(int64_t c, Raw<K, TIER, MASS>& r) const {
    if (MASS) r.m = in_mass[c];
#pragma unroll
    for (int l = (MASS ? 1 : 0); l < O; ++l) r.h[l] = in[l][c];
  }
  __device__ __forceinline__ void store(int64_t c, const Mat<K, TIER, MASS>& M,
                                        const Raw<K, TIER, MASS>& x,
                                        const Raw<K, TIER, MASS>& y) const {
    if (MASS) out_mass[c] = M.mass_out(x, y);
#pragma unroll
    for (int j = (MASS ? 1 : 0); j < O; ++j) out[j][c] = M.hi_out(j, x, y);
  }
};

// ---------------------------------------------------------------------------
// Sweep along dimension 0, generic form (any N_0).  One wave per (line,
// spectator tuple):
// the line's s, A and B are wave-uniform (scalar registers), lanes walk the
// line's cells, so every plane access of a wave is one contiguous run with a
// periodic wrap.  The second source cell of lane L is the first one of lane
// L-1, so the reuse is served by the vector L1.
// ---------------------------------------------------------------------------

template <int K, int TIER, bool MASS>
__device__ __forceinline__ void contig_line(const SweepArgs& a, int64_t line, int32_t sp,
                                            int lane) {
  constexpr int O = K + 1;
  Mat<K, TIER, MASS> M;
  Planes<K, TIER, MASS> pl;
  const int32_t t = __builtin_amdgcn_readfirstlane(table_index(a.map, 0, (int32_t)line));
  const int32_t s = __builtin_amdgcn_readfirstlane(a.s_tab[t]);
  M.load(a.ab_tab + (int64_t)t * 2 * O * O);
  pl.bind(a, (int64_t)sp * O, 1);
  const int32_t N = a.N;
  const int64_t base = line * (int64_t)N;
  for (int32_t i = lane; i < N; i += 64) {
    int32_t ia = i - s;
    if (ia < 0) ia += N;
    int32_t ib = ia - 1;
    if (ib < 0) ib += N;
    Raw<K, TIER, MASS> x, y;
    pl.load(base + ia, x);
    pl.load(base + ib, y);
    pl.store(base + i, M, x, y);
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
// along its line through a chunk of rows, keeping the previous source row in
// registers so every input row of the chunk is read once.  Rows are loaded U
// at a time and the loads of the next U rows are issued before the current
// ones are computed and stored, so a wave keeps 2U rows of o planes in flight
// (the sweep is latency-bound otherwise: one row per wave is far too little
// to cover HBM latency).  The displacement (and so s, A, B) may differ from
// lane to lane.
// ---------------------------------------------------------------------------

template <int K, int TIER, bool MASS, int U>
__device__ __forceinline__ void strided_run(const SweepArgs& a, int32_t ilow, int32_t chunk,
                                            int32_t ihigh, int32_t sp) {
  constexpr int O = K + 1;
  using R = Raw<K, TIER, MASS>;
  Mat<K, TIER, MASS> M;
  Planes<K, TIER, MASS> pl;
  const int32_t t = table_index(a.map, ilow, ihigh);
  const int32_t s = a.s_tab[t];
  M.load(a.ab_tab + (int64_t)t * 2 * O * O);
  const int32_t ms = a.mstride;
  const int64_t m0 = (int64_t)(sp % ms) + (int64_t)(sp / ms) * ms * O;
  pl.bind(a, m0, ms);
  const int32_t N = a.N, P = a.P;
  const int64_t base = (int64_t)ihigh * P * N + ilow;
  const int32_t r0 = chunk * a.chunk;
  const int32_t n = min(N, r0 + a.chunk) - r0;
  int32_t iy = r0 - s - 1;
  if (iy < 0) iy += N;
  R y;
  pl.load(base + (int64_t)iy * P, y);
  int32_t ix = iy + 1;             // next source row to load (cell i - s)
  if (ix == N) ix = 0;
  R xa[U], xb[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (u < n) {
      pl.load(base + (int64_t)ix * P, xa[u]);
      if (++ix == N) ix = 0;
    }
  }
  for (int32_t g = 0; g < n; g += U) {
    const int32_t cnt = min(U, n - g);
    const int32_t nxt = n - g - U;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (u < nxt) {
        pl.load(base + (int64_t)ix * P, xb[u]);
        if (++ix == N) ix = 0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (u < cnt) {
        pl.store(base + (int64_t)(r0 + g + u) * P, M, xa[u], y);
        y = xa[u];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xa[u] = xb[u];
  }
}

template <int K, int TIER>
__global__ __launch_bounds__(256) void sweep_strided_kernel(SweepArgs a) {
  constexpr int U = 4;
  const int32_t sp = blockIdx.y;
  const int64_t per = (int64_t)a.P * a.nchunk * a.Q;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= per) return;
  const int32_t ilow = (int32_t)(tid % a.P);
  const int64_t r = tid / a.P;
  const int32_t chunk = (int32_t)(r % a.nchunk);
  const int32_t ihigh = (int32_t)(r / a.nchunk);
  if (sp == 0) strided_run<K, TIER, true, U>(a, ilow, chunk, ihigh, sp);
  else strided_run<K, TIER, false, U>(a, ilow, chunk, ihigh, sp);
}

// ---------------------------------------------------------------------------
// Sweep along dimension 0 with an LDS tile.  A block takes `tile_lines`
// consecutive lines of one spectator tuple: a contiguous segment of each of
// the o planes, copied to LDS with 16-byte loads (the whole line is resident,
// so the periodic wrap and the upwind neighbour cost no extra HBM access),
// together with the lines' s, A and B.  Each thread then produces V = 4
// consecutive output cells of one line from a window of V+1 source cells
// read from LDS, and writes them with one vector store per plane.
// Requires N_0 % 8 == 0 (16-byte alignment of every line in every plane).
// ---------------------------------------------------------------------------

constexpr int kTileV = 4;

template <class T> struct Vec4;
template <> struct Vec4<double> { using type = double4; };
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<__bf16> { using type = uint2; };
template <> struct Vec4<_Float16> { using type = uint2; };

template <class T>
__device__ __forceinline__ void store4(T* dst, const T (&v)[4]) {
  if constexpr (sizeof(T) == 8) {
    double2* d = reinterpret_cast<double2*>(dst);
    d[0] = make_double2(v[0], v[1]);
    d[1] = make_double2(v[2], v[3]);
  } else if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    uint16_t b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) b[u] = __builtin_bit_cast(uint16_t, v[u]);
    *reinterpret_cast<uint2*>(dst) = make_uint2((uint32_t)b[0] | ((uint32_t)b[1] << 16),
                                                (uint32_t)b[2] | ((uint32_t)b[3] << 16));
  }
}

// Copy `bytes` (a multiple of 16) from global to LDS with 16-byte accesses.
__device__ __forceinline__ void copy_to_lds(void* lds, const void* src, int32_t bytes) {
  const uint4* s4 = reinterpret_cast<const uint4*>(src);
  uint4* d4 = reinterpret_cast<uint4*>(lds);
  const int32_t n = bytes >> 4;
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) d4[i] = s4[i];
}

template <int K, int TIER, bool MASS>
__device__ __forceinline__ void contig_tile(const SweepArgs& a, int32_t tile_lines,
                                            unsigned char* smem) {
  constexpr int O = K + 1;
  constexpr int V = kTileV;
  using T = typename Tier<TIER>::T;
  using Acc = typename Tier<TIER>::Acc;
  using R = Raw<K, TIER, MASS>;
  const int32_t sp = blockIdx.y;
  const int32_t N = a.N;
  const int64_t line0 = (int64_t)blockIdx.x * tile_lines;
  const int32_t nl = (int32_t)min((int64_t)tile_lines, (int64_t)a.Q - line0);
  const int32_t tc = nl * N;                      // cells in this tile
  const int32_t cap = tile_lines * N;             // cells per plane slot
  // LDS layout: A/B per line | s per line | plane 0 (8-byte slots) | planes 1..k
  double* ab_l = reinterpret_cast<double*>(smem);
  int32_t* s_l = reinterpret_cast<int32_t*>(ab_l + tile_lines * 2 * O * O);
  unsigned char* pbase = smem + tile_lines * (2 * O * O * 8 + 4);
  pbase += (16 - ((uintptr_t)pbase & 15)) & 15;
  double* p0d = reinterpret_cast<double*>(pbase);
  T* p0t = reinterpret_cast<T*>(pbase);
  T* ph[O];
#pragma unroll
  for (int l = 1; l < O; ++l)
    ph[l] = reinterpret_cast<T*>(pbase + (size_t)cap * 8 + (size_t)(l - 1) * cap * sizeof(T));
  ph[0] = p0t;

  Planes<K, TIER, MASS> pl;
  pl.bind(a, (int64_t)sp * O, 1);
  const int64_t cell0 = line0 * N;
  // per-line tables
  for (int32_t q = threadIdx.x; q < nl * 2 * O * O; q += blockDim.x) {
    const int32_t li = q / (2 * O * O);
    const int32_t e = q - li * (2 * O * O);
    const int32_t t = table_index(a.map, 0, (int32_t)(line0 + li));
    ab_l[q] = a.ab_tab[(int64_t)t * 2 * O * O + e];
    if (e == 0) s_l[li] = a.s_tab[t];
  }
  // plane segments
  if (MASS) copy_to_lds(p0d, pl.in_mass + cell0, tc * 8);
#pragma unroll
  for (int l = (MASS ? 1 : 0); l < O; ++l)
    copy_to_lds(ph[l], pl.in[l] + cell0, tc * (int32_t)sizeof(T));
  __syncthreads();

  const int32_t ng = tc / V;
  for (int32_t g = threadIdx.x; g < ng; g += blockDim.x) {
    const int32_t c = g * V;
    const int32_t li = c / N;
    const int32_t i0 = c - li * N;
    const int32_t s = s_l[li];
    Mat<K, TIER, MASS> M;
    M.load(ab_l + li * 2 * O * O);
    // window of source cells i0-s-1 .. i0-s+V-1 (periodic in the line)
    R w[V + 1];
    int32_t idx = i0 - s - 1;
    if (idx < 0) idx += N;
    const int32_t lb = li * N;
#pragma unroll
    for (int u = 0; u <= V; ++u) {
      if (MASS) w[u].m = p0d[lb + idx];
#pragma unroll
      for (int l = (MASS ? 1 : 0); l < O; ++l) w[u].h[l] = ph[l][lb + idx];
      if (++idx == N) idx = 0;
    }
    const int64_t gc = cell0 + c;
    if (MASS) {
      double o4[V];
#pragma unroll
      for (int u = 0; u < V; ++u) o4[u] = M.mass_out(w[u + 1], w[u]);
      store4<double>(pl.out_mass + gc, o4);
    }
#pragma unroll
    for (int j = (MASS ? 1 : 0); j < O; ++j) {
      T o4[V];
#pragma unroll
      for (int u = 0; u < V; ++u) o4[u] = M.hi_out(j, w[u + 1], w[u]);
      store4<T>(pl.out[j] + gc, o4);
    }
  }
}

template <int K, int TIER>
__global__ __launch_bounds__(256) void sweep_contig_tiled_kernel(SweepArgs a, int32_t tile_lines) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (blockIdx.y == 0) contig_tile<K, TIER, true>(a, tile_lines, smem);
  else contig_tile<K, TIER, false>(a, tile_lines, smem);
}

template <int K, int TIER>
static hipError_t launch_sweep_kt(int dim, const SweepArgs& a, hipStream_t st) {
  using T = typename Tier<TIER>::T;
  constexpr int O = K + 1;
  if (dim == 0) {
    const int64_t lds_per_cell = 8 + (int64_t)(O - 1) * sizeof(T);
    const int64_t tile_cells = sizeof(T) == 8 ? 1024 : 2048;
    const uintptr_t align = (uintptr_t)a.in_mass | (uintptr_t)a.in_hi | (uintptr_t)a.out_mass |
                            (uintptr_t)a.out_hi;
    if (a.N % 8 == 0 && a.N <= tile_cells && (align & 15) == 0) {
      const int32_t tl = (int32_t)(tile_cells / a.N);
      const size_t lds = (size_t)tl * (2 * O * O * 8 + 4) + 16 + (size_t)tl * a.N * lds_per_cell;
      dim3 grid((unsigned)((a.Q + tl - 1) / tl), (unsigned)a.nspec), block(256);
      sweep_contig_tiled_kernel<K, TIER><<<grid, block, lds, st>>>(a, tl);
    } else {
      const int64_t items = (int64_t)a.Q * a.nspec;
      dim3 grid((unsigned)((items + 3) / 4)), block(256);
      sweep_contig_kernel<K, TIER><<<grid, block, 0, st>>>(a);
    }
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
