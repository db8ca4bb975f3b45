// Fused pair of projection sweeps (L. Einkemmer, arXiv 1603.07008, section
// II-A update rule): the sweep along dimension 0 followed by the sweep along
// dimension 1, in one pass over the state.  The split step of section II
// applies these two sweeps one after the other (x1 then x2); between them the
// unfused path writes the whole state to HBM and reads it back.  Here a
// workgroup holds one tile of the (x0, x1) slab in LDS for one group of
// spectator modes and applies both sweeps to it:
//   tile      the o^2 modes (j0, j1) of one spectator group (j2, j3, ...), for
//             every cell of dimension 0 and R + 1 consecutive rows of
//             dimension 1, of one slab (a fixed cell of the dimensions >= 2)
//   phase 1   the tile is read from HBM (each row a contiguous run of cells)
//   phase 2   the dimension-0 sweep, in place in LDS, every value rounded to
//             the storage format as the unfused sweep stores it
//   phase 3   the dimension-1 sweep from the LDS tile, stored to HBM: output
//             rows r0 .. r0+R-1 read tile rows t and t+1, because the tile
//             starts at row r0 - s1 - 1
// Each coefficient is read once (plus one halo row per tile) and written once
// for two sweeps.  Both displacements must be uniform over a slab (neither
// depends on dimension 0 or 1), so a workgroup needs one line table per
// sweep.  The arithmetic of every output is the unfused kernels' own (the same
// Mat / Rows64 evaluation order and the same rounding), so results are
// bitwise those of two separate sweeps.
#pragma once

#include "sldg_sweep.h"

namespace sldg {

struct XYArgs {
  const double* in_lo;     // FP64 plane of mode 0 (n_lo == 1), or unused
  const void* in_hi;       // the other modes, storage type of the tier
  double* out_lo;
  void* out_hi;
  int32_t n_lo;            // 1: mode 0 stored in FP64; 0: every mode narrow
  int64_t cells;           // cells of the grid (plane length)
  int32_t N0, N1;          // extents of dimensions 0 and 1 (N0 % 4 == 0)
  int32_t Q;               // slabs: product of the extents of dimensions >= 2
  int32_t R;               // output rows of dimension 1 per tile
  int32_t nrc;             // row chunks per slab: ceil(N1 / R)
  int32_t tstride;         // LDS elements per plane of a tile (>= (R + 1) N0, % 8 == 0)
  int32_t xcd;             // XCD-aware tile order: run length G (0 off)
  float one;               // 1.0f: the FP16 tier's unit output scale (see tuple4)
  FastDiv fnb;             // division by N0 / 4 (4-cell blocks per row)
  FastDiv fnrc;            // division by nrc
  FastDiv fQ;              // division by Q
  // line tables of the dimension-0 and dimension-1 sweeps: entry t holds s
  // mod N at s_tab[t] and A, B component e at ab[e * cs + t]
  const int32_t* s0;
  const double* ab0;
  int64_t cs0;
  LineMap map0;
  const int32_t* s1;
  const double* ab1;
  int64_t cs1;
  LineMap map1;
};

// A 4-cell block of LDS as the storage type.
template <class T>
__device__ __forceinline__ Blk4<T> lds_blk4(const T* p) {
  return unpack4<T>(fetch4<T>(p));
}

template <class T>
__device__ __forceinline__ void lds_put4(T* p, const T (&v)[4]) {
  if constexpr (sizeof(T) == 8) {
    nt_d2* d = reinterpret_cast<nt_d2*>(p);
    d[0] = nt_d2{v[0], v[1]};
    d[1] = nt_d2{v[2], v[3]};
  } else if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<nt_f4*>(p) = nt_f4{v[0], v[1], v[2], v[3]};
  } else {
    uint16_t b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) b[u] = __builtin_bit_cast(uint16_t, v[u]);
    *reinterpret_cast<nt_u2*>(p) = nt_u2{(uint32_t)b[0] | ((uint32_t)b[1] << 16),
                                         (uint32_t)b[2] | ((uint32_t)b[3] << 16)};
  }
}

// Output modes of one tuple (the swept index varying) for 4 cells, from the
// source values x (cell i - s, through A) and y (cell i - s - 1, through B)
// of each cell: the FP64 row (ND == 1) and the narrow rows, rounded to the
// storage type exactly as the unfused kernels round them on store.  The FP16
// tier stores acc * 2^e there (the plane's storage scale, a run-time value);
// with the unit scale `one` (1.0f, a run-time value too) the same two
// roundings happen here: the FP32 accumulation, then FP32 -> FP16.  Without
// the multiply the compiler may merge the last FMA and the conversion into
// one mixed-precision instruction that rounds only once.
template <int K, int TIER, int ND>
__device__ __forceinline__ void tuple4(const Mat<K, TIER>& M, const Rows64<K, 1>& R64,
                                       const Raw<K, TIER, ND> (&x)[4],
                                       const Raw<K, TIER, ND> (&y)[4],
                                       typename Tier<TIER>::T (&out)[K + 1][4],
                                       double (&out64)[4], float one) {
  using T = typename Tier<TIER>::T;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
#pragma unroll
    for (int j = 0; j < K + 1; ++j) {
      if (j < ND) {
        Rows64<K, ND> r;
#pragma unroll
        for (int l = 0; l < K + 1; ++l) {
          r.A[0][l] = R64.A[0][l];
          r.B[0][l] = R64.B[0][l];
        }
        out64[v] = Mat<K, TIER>::template out64<ND>(r, 0, x[v], y[v]);
      } else {
        if constexpr (TIER == 3) out[j][v] = (T)(M.template out_acc<ND>(j, x[v], y[v]) * one);
        else out[j][v] = narrow<T>(M.template out_acc<ND>(j, x[v], y[v]));
      }
    }
  }
}

// A source value as the unfused kernels hold it: the FP16 tier widens and
// multiplies by the input plane's scale (here the run-time unit `one`).
template <int K, int TIER, int ND>
__device__ __forceinline__ void raw_set(Raw<K, TIER, ND>& r, int l, typename Tier<TIER>::T v,
                                        double d, float one) {
  if (l < ND) r.d[l] = d;
  else r.h[l] = to_reg<TIER>(v, one);
}

constexpr int kXYMaxItems = 4;     // phase-2 items per thread (host checks)

// The 5-cell window at a compile-time offset D of the first of two
// consecutive 4-cell blocks.
template <class T, int D>
__device__ __forceinline__ void window5_at(const Blk4<T>& b0, const Blk4<T>& b1, T (&w)[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) w[v] = D + v < 4 ? b0.v[D + v] : b1.v[D + v - 4];
}

// The items tid, tid + 256, ... of a flat index space (q, r, b), b fastest
// (extents nq x nr x nb): the start is split with float reciprocals (exact
// for these small integers: tid < 256 and the quotient's fractional part is
// at least 1/(2 nr nb)), then every step adds 256 items without division.
struct Walk {
  int32_t q, r, b;
  int32_t dq, dr, db, nr, nb;
  __device__ __forceinline__ void init(int32_t tid, int32_t nr_, int32_t nb_) {
    nr = nr_;
    nb = nb_;
    const int32_t ne = nr * nb;
    q = (int32_t)(((float)tid + 0.5f) * (1.0f / (float)ne));
    const int32_t e = tid - q * ne;
    r = (int32_t)(((float)e + 0.5f) * (1.0f / (float)nb));
    b = e - r * nb;
    dq = 256 / ne;
    const int32_t de = 256 - dq * ne;
    dr = de / nb;
    db = de - dr * nb;
  }
  __device__ __forceinline__ void next() {
    q += dq;
    r += dr;
    b += db;
    if (b >= nb) {
      b -= nb;
      ++r;
    }
    if (r >= nr) {
      r -= nr;
      ++q;
    }
  }
};

// A 64-bit offset j * stride for a small per-lane j (0 <= j < O), by selects.
template <int O>
__device__ __forceinline__ int64_t small_mul(int32_t j, int64_t stride) {
  int64_t r = 0;
#pragma unroll
  for (int v = 1; v < O; ++v) r = j == v ? (int64_t)v * stride : r;
  return r;
}

template <int K, int TIER>
__global__ __launch_bounds__(256) void sweep_xy_kernel(XYArgs a) {
  constexpr int O = K + 1, O2 = O * O;
  using T = typename Tier<TIER>::T;
  extern __shared__ __align__(16) unsigned char xy_smem[];
  T* tile = reinterpret_cast<T*>(xy_smem);                                      // [O2][tstride]
  double* tile64 = reinterpret_cast<double*>(xy_smem + (size_t)O2 * a.tstride * sizeof(T));

  uint32_t w = blockIdx.x;
  if (a.xcd) w = xcd_tile(w, gridDim.x, a.xcd);
  const uint32_t rest = a.fnrc.div(w);
  const int32_t rc = (int32_t)(w - rest * (uint32_t)a.nrc);
  const uint32_t gq = a.fQ.div(rest);
  const int32_t slab = (int32_t)(rest - gq * (uint32_t)a.Q);
  const int32_t g = (int32_t)gq;
  const int32_t N0 = a.N0, N1 = a.N1, nb = N0 >> 2;
  const int32_t r0 = rc * a.R;
  const int32_t n = min(a.R, N1 - r0);
  const int32_t rows = n + 1;
  const bool has64 = g == 0 && a.n_lo == 1;

  // the two sweeps' line tables (uniform over the workgroup)
  const int32_t t0 = table_index(a.map0, 0, N1 * slab);
  const int32_t t1 = table_index(a.map1, 0, slab);
  const int32_t sh0 = a.s0[t0], sh1 = a.s1[t1];
  // the dimension-0 sweep's matrices now, the dimension-1 sweep's after the
  // tile is built (fewer scalar registers live at once)
  Mat<K, TIER> M0;
  M0.load(a.ab0 + t0, a.cs0);
  Rows64<K, 1> R0;
  R0.load(M0.ab, M0.cs);

  const T* hin = reinterpret_cast<const T*>(a.in_hi);
  T* hout = reinterpret_cast<T*>(a.out_hi);
  const int64_t slab_off = (int64_t)slab * N1 * N0;
  const int32_t top = r0 - sh1 - 1;            // row of dimension 1 at tile row 0 (mod N1)

  // phase 1: the tile's rows of every mode of the group into LDS
  for (int32_t e4 = (int32_t)threadIdx.x; e4 < rows * nb; e4 += 256) {
    const int32_t u = (int32_t)a.fnb.div((uint32_t)e4);
    const int32_t b = e4 - u * nb;
    int32_t gr = top + u;
    if (gr < 0) gr += N1;
    if (gr >= N1) gr -= N1;
    const int64_t off = slab_off + (int64_t)gr * N0 + 4 * b;
    Raw4<T> v[O2];
#pragma unroll
    for (int l = 0; l < O2; ++l) {
      const int32_t m = g * O2 + l;
      if (!(has64 && l == 0)) v[l] = fetch4<T>(hin + (int64_t)(m - a.n_lo) * a.cells + off);
    }
    Raw4<double> v64;
    if (has64) v64 = fetch4<double>(a.in_lo + off);
#pragma unroll
    for (int l = 0; l < O2; ++l) {
      if (!(has64 && l == 0)) {
        auto* d = reinterpret_cast<typename Raw4<T>::V*>(tile + (int64_t)l * a.tstride + e4 * 4);
#pragma unroll
        for (int q = 0; q < Raw4<T>::W; ++q) d[q] = v[l].v[q];
      }
    }
    if (has64) {
      auto* d = reinterpret_cast<nt_d2*>(tile64 + e4 * 4);
      d[0] = v64.v[0];
      d[1] = v64.v[1];
    }
  }
  __syncthreads();

  // phase 2: the dimension-0 sweep of every tile row, in place.  Item (j1,
  // e4): the 4 cells of block e4 of the tile, the tuple of modes (j0, j1),
  // j0 = 0..k.  The sources of output cells i0..i0+3 are the 5 cells from
  // c = i0 - s0 - 1 (periodic in the row), inside the aligned blocks at
  // c & ~3 and the next one.
  // The window's offset in its first block, (i0 - s0 - 1) mod 4, is the
  // same for every item (i0 and N0 are multiples of 4, s0 is uniform over
  // the slab): phase 2 is compiled for each of the 4 offsets and takes the
  // window by fixed indices instead of per-lane selects.
  T res[kXYMaxItems][O][4];
  double res64[kXYMaxItems][4];
  const int32_t nitem = O * rows * nb;
  auto phase2 = [&](auto dc) {
    constexpr int D = decltype(dc)::value;
#pragma unroll
    for (int it = 0; it < kXYMaxItems; ++it) {
      const int32_t item = (int32_t)threadIdx.x + 256 * it;
      if (item >= nitem) break;
      const int32_t j1 = item / (rows * nb);
      const int32_t e4 = item - j1 * (rows * nb);
      const int32_t u = (int32_t)a.fnb.div((uint32_t)e4);
      const int32_t i0 = 4 * (e4 - u * nb);
      int32_t c = i0 - sh0 - 1;
      if (c < 0) c += N0;
      const int32_t blk0 = c & ~3;
      int32_t blk1 = blk0 + 4;
      if (blk1 == N0) blk1 = 0;
      const int32_t rowoff = u * N0;
      T wv[O][5];
      double w64[5];
#pragma unroll
      for (int l0 = 0; l0 < O; ++l0) {
        const int32_t l = l0 + O * j1;
        const T* pl = tile + (int64_t)l * a.tstride + rowoff;
        const Blk4<T> b0 = lds_blk4<T>(pl + blk0), b1 = lds_blk4<T>(pl + blk1);
        window5_at<T, D>(b0, b1, wv[l0]);
      }
      const bool nd1 = has64 && j1 == 0;
      if (nd1) {
        const Blk4<double> b0 = lds_blk4<double>(tile64 + rowoff + blk0);
        const Blk4<double> b1 = lds_blk4<double>(tile64 + rowoff + blk1);
        window5_at<double, D>(b0, b1, w64);
      }
      auto run = [&](auto ndc) {
        constexpr int ND = decltype(ndc)::value;
        Raw<K, TIER, ND> x[4], y[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int l0 = 0; l0 < O; ++l0) {
            raw_set<K, TIER, ND>(x[v], l0, wv[l0][v + 1], ND ? w64[v + 1] : 0.0, a.one);
            raw_set<K, TIER, ND>(y[v], l0, wv[l0][v], ND ? w64[v] : 0.0, a.one);
          }
        tuple4<K, TIER, ND>(M0, R0, x, y, res[it], res64[it], a.one);
      };
      if (nd1) run(std::integral_constant<int, 1>{});
      else run(std::integral_constant<int, 0>{});
    }
  };
  switch (__builtin_amdgcn_readfirstlane((-sh0 - 1) & 3)) {
    case 0: phase2(std::integral_constant<int, 0>{}); break;
    case 1: phase2(std::integral_constant<int, 1>{}); break;
    case 2: phase2(std::integral_constant<int, 2>{}); break;
    default: phase2(std::integral_constant<int, 3>{}); break;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kXYMaxItems; ++it) {
    const int32_t item = (int32_t)threadIdx.x + 256 * it;
    if (item >= nitem) break;
    const int32_t j1 = item / (rows * nb);
    const int32_t e4 = item - j1 * (rows * nb);
    const int32_t poff = 4 * e4;
    const bool nd1 = has64 && j1 == 0;
#pragma unroll
    for (int j0 = 0; j0 < O; ++j0) {
      if (nd1 && j0 == 0) {
        nt_d2* dd = reinterpret_cast<nt_d2*>(tile64 + poff);
        dd[0] = nt_d2{res64[it][0], res64[it][1]};
        dd[1] = nt_d2{res64[it][2], res64[it][3]};
      } else {
        lds_put4<T>(tile + (int64_t)(j0 + O * j1) * a.tstride + poff, res[it][j0]);
      }
    }
  }
  __syncthreads();

  Mat<K, TIER> M1;
  M1.load(a.ab1 + t1, a.cs1);
  Rows64<K, 1> R1;
  R1.load(M1.ab, M1.cs);

  // phase 3: the dimension-1 sweep from the tile, to HBM.  Items (j0, t, b):
  // output row t of the chunk, cells 4b .. 4b+3, the tuple of modes (j0, j1),
  // j1 = 0..k, from tile rows t + 1 (cell i - s1) and t (cell i - s1 - 1).
  {
    const int64_t cells = a.cells;
    T* hout_g = hout + ((int64_t)g * O2 - a.n_lo) * cells;      // mode g O2 + l at l * cells
    Walk w;
    w.init((int32_t)threadIdx.x, n, nb);
    for (; w.q < O; w.next()) {
      const int32_t j0 = w.q, t = w.r, i0 = 4 * w.b;
      const bool nd1 = has64 && j0 == 0;
      const int32_t eoff = (int32_t)__umul24((uint32_t)t, (uint32_t)N0) + i0;
      const T* tcol = tile + (int32_t)__umul24((uint32_t)j0, (uint32_t)a.tstride) + eoff;
      Blk4<T> xb[O], yb[O];
#pragma unroll
      for (int l1 = 0; l1 < O; ++l1) {
        yb[l1] = lds_blk4<T>(tcol + O * l1 * a.tstride);
        xb[l1] = lds_blk4<T>(tcol + O * l1 * a.tstride + N0);
      }
      Blk4<double> x64, y64;
      if (nd1) {
        y64 = lds_blk4<double>(tile64 + eoff);
        x64 = lds_blk4<double>(tile64 + eoff + N0);
      }
      T out[O][4];
      double out64[4];
      auto run = [&](auto ndc) {
        constexpr int ND = decltype(ndc)::value;
        Raw<K, TIER, ND> x[4], y[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int l1 = 0; l1 < O; ++l1) {
            raw_set<K, TIER, ND>(x[v], l1, xb[l1].v[v], ND ? x64.v[v] : 0.0, a.one);
            raw_set<K, TIER, ND>(y[v], l1, yb[l1].v[v], ND ? y64.v[v] : 0.0, a.one);
          }
        tuple4<K, TIER, ND>(M1, R1, x, y, out, out64, a.one);
      };
      if (nd1) run(std::integral_constant<int, 1>{});
      else run(std::integral_constant<int, 0>{});
      const int64_t off = slab_off + (int32_t)__umul24((uint32_t)(r0 + t), (uint32_t)N0) + i0;
      const int64_t poff = off + small_mul<O>(j0, cells);
#pragma unroll
      for (int j1 = 0; j1 < O; ++j1) {
        if (nd1 && j1 == 0) {
          const double v4[4] = {out64[0], out64[1], out64[2], out64[3]};
          store4<double>(a.out_lo + off, v4);
        } else {
          store4<T>(hout_g + poff + (int64_t)(O * j1) * cells, out[j1]);
        }
      }
    }
  }
}

// LDS bytes of a tile of R output rows (the launcher's dynamic shared memory).
inline int64_t xy_tile_stride(int32_t N0, int32_t R) {
  return ((int64_t)(R + 1) * N0 + 7) / 8 * 8;
}
inline int64_t xy_lds_bytes(int k, int tier_bytes, int32_t N0, int32_t R) {
  const int64_t o2 = (int64_t)(k + 1) * (k + 1);
  return o2 * xy_tile_stride(N0, R) * tier_bytes + xy_tile_stride(N0, R) * 8;
}

}  // namespace sldg
