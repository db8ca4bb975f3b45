// Device code of the sLdG projection sweep kernels (L. Einkemmer, arXiv
// 1603.07008, section II-A, update rule)
//     out[i] = A(alpha) in[i - s] + B(alpha) in[i - s - 1]
// along one dimension of a periodic tensor grid, on split storage (FP64 cell
// mean + narrower higher modes).  Templates only: sldg_sweep_inst.hip
// instantiates them once per (degree, storage tier), and sldg_kernels.hip
// uses the shared helpers (table index, scaling) of its own kernels.
//
// The sweep is a batched (k+1)x(k+1) contraction with 1-3 flop per byte moved,
// far below the machine balance, so it is HBM-bound: the kernels are built
// around coalesced plane reads (split mode-major storage keeps every mode plane
// contiguous along dimension 0) and each coefficient is read once and written
// once per sweep.  No matrix cores: the contraction is too small and too
// memory-bound for MFMA to matter.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "sldg_internal.h"

namespace sldg {

// Stores of the sweeps' outputs.  Every output coefficient is written once
// per sweep and not read again by it, so stores whose wave writes whole
// 128-byte lines carry the non-temporal hint, which raises the HBM rate of
// this pattern: the window form's 8 or 16 bytes per lane, and one value per
// lane (kernels instantiated with NT > 0) where the host found the wave's
// cells to cover whole lines (SweepArgs::ntmask).  Stores that leave partial
// lines (the group form's interleaved cells, strided rows of 48 FP32 or BF16
// cells) stay plain: there the hint measured slower.  The choice is made
// at compile time: a run-time branch between the two stores is merged by the
// compiler into one plain store.  Loads stay plain (the hint evicts the
// neighbouring cells that the next lanes and rows read again).
template <class T>
__device__ __forceinline__ void st_stream(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// NT: 0 plain; 1 the hint on 4- and 8-byte values; 2 on 2-byte values too
// (the 16-bit tiers where a wave's 64 values fill a whole line).
template <int NT, class T>
__device__ __forceinline__ void st_lane(T* p, T v) {
  if constexpr (NT >= 1 && sizeof(T) >= 4) {
    __builtin_nontemporal_store(v, p);
  } else if constexpr (NT >= 2 && sizeof(T) == 2) {
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), reinterpret_cast<uint16_t*>(p));
  } else {
    *p = v;
  }
}

typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef uint32_t nt_u2 __attribute__((ext_vector_type(2)));


// ---------------------------------------------------------------------------
// Storage tiers (section II-A: c_0 in FP64, the higher modes narrower)
// ---------------------------------------------------------------------------

// T: storage type of the narrow modes; Acc: arithmetic type of their update;
// R: register type of a loaded narrow value (the FP16 tier widens on load,
// where its per-mode storage scale is removed).
template <int TIER> struct Tier;
template <> struct Tier<0> { using T = double;   using Acc = double; using R = double; };
template <> struct Tier<1> { using T = float;    using Acc = double; using R = float;  };
template <> struct Tier<2> { using T = __bf16;   using Acc = float;  using R = __bf16; };
template <> struct Tier<3> { using T = _Float16; using Acc = float;  using R = float;  };

// Exact widening of a stored value to FP64 / FP32.
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return (double)v; }
__device__ __forceinline__ double widen(__bf16 v) { return (double)(float)v; }
__device__ __forceinline__ double widen(_Float16 v) { return (double)(float)v; }

// Round-to-nearest-even narrowing on store (hardware conversions on gfx950).
template <class T, class A> __device__ __forceinline__ T narrow(A v) { return (T)v; }

// ---------------------------------------------------------------------------
// Line-table index
// ---------------------------------------------------------------------------

__device__ __forceinline__ int32_t table_index(const LineMap& m, int32_t lo, int32_t hi) {
  int32_t t = 0;
  for (int e = 0; e < m.nlo; ++e)
    t += (int32_t)m.lo_mod[e].mod(m.lo_div[e].div((uint32_t)lo)) * m.lo_str[e];
  for (int e = 0; e < m.nhi; ++e)
    t += (int32_t)m.hi_mod[e].mod(m.hi_div[e].div((uint32_t)hi)) * m.hi_str[e];
  return t;
}

// ---------------------------------------------------------------------------
// Modes of one spectator tuple (modes m0 + l * mstride, l = 0..k, the swept
// index j_d varying) and where they are stored.  The modes of total degree
// below the plan's "number of FP64 modes" live in the FP64 array `lo`, the
// others in the storage type of the tier (array `hi`); within a tuple the FP64
// modes are the leading ones (the total degree grows with j_d).  ND, the
// number of leading FP64 modes, is a compile-time parameter of the per-tuple
// code (the paper's mixed-precision scheme keeps c_0 in FP64, section II-A;
// its experiments vary how many leading coefficients are FP64, section III-A).
// Values stay in their storage type in registers and are widened exactly when
// used.
// ---------------------------------------------------------------------------

struct TupleMap {
  int32_t idx[4];   // plane index in lo (l < nd) or hi (l >= nd)
  int32_t nd;       // leading FP64 modes of the tuple
};

// Planes of the modes m0 + l * ms, l < O.  With at most the cell mean in
// FP64 (NDMAX == 1: mode 0 in `lo` when n_lo == 1, mode m at hi plane
// m - n_lo) the map is arithmetic and needs no memory access: a load here,
// between the stores of one tuple and the loads of the next, would make the
// wave wait for those stores (one counter covers all vector memory
// operations).  Otherwise the plane map is read at a wave-uniform index.
template <int NDMAX>
__device__ __forceinline__ TupleMap tuple_map(const SweepArgs& a, int32_t m0, int32_t ms,
                                              int O) {
  TupleMap t;
  t.nd = 0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    if (l < O) {
      const int32_t m = __builtin_amdgcn_readfirstlane(m0 + l * ms);
      if constexpr (NDMAX == 1) {
        const bool lo = m < a.n_lo;
        t.idx[l] = lo ? m : m - a.n_lo;
        t.nd += lo ? 1 : 0;
      } else {
        const int32_t v = __builtin_amdgcn_readfirstlane(a.pmap[m]);
        t.idx[l] = v < 0 ? -1 - v : v;
        t.nd += v < 0 ? 1 : 0;
      }
    }
  }
  return t;
}

template <int K, int TIER, int ND>
struct Raw {
  static constexpr int O = K + 1;
  using R = typename Tier<TIER>::R;
  double d[O];   // modes l < ND
  R h[O];        // modes l >= ND
};

// Copy of the fields a tuple with ND leading FP64 modes uses (whole-struct
// copies of partly used register structs end up in scratch memory).
template <int K, int TIER, int ND>
__device__ __forceinline__ void copy_raw(Raw<K, TIER, ND>& dst, const Raw<K, TIER, ND>& src) {
#pragma unroll
  for (int l = 0; l < K + 1; ++l) {
    if (l < ND) dst.d[l] = src.d[l];
    else dst.h[l] = src.h[l];
  }
}

// FP64 rows j < ND of A and B (the rows of the modes stored in FP64, whose
// update is FP64 throughout).
template <int K, int ND>
struct Rows64 {
  static constexpr int O = K + 1;
  double A[ND > 0 ? ND : 1][O], B[ND > 0 ? ND : 1][O];
  __device__ __forceinline__ void load(const double* ab, int64_t cs) {
#pragma unroll
    for (int j = 0; j < ND; ++j)
#pragma unroll
      for (int l = 0; l < O; ++l) {
        A[j][l] = ab[(j * O + l) * cs];
        B[j][l] = ab[(O * O + j * O + l) * cs];
      }
  }
};

template <int K, int TIER>
struct Mat {
  static constexpr int O = K + 1;
  using T = typename Tier<TIER>::T;
  using Acc = typename Tier<TIER>::Acc;
  Acc Aa[O][O], Ba[O][O];      // all rows in the arithmetic type
  const double* ab;            // the table entry (component e at ab[e * cs])
  int64_t cs;

  __device__ __forceinline__ void load(const double* ab_, int64_t cs_) {
    ab = ab_;
    cs = cs_;
#pragma unroll
    for (int j = 0; j < O; ++j)
#pragma unroll
      for (int l = 0; l < O; ++l) {
        Aa[j][l] = (Acc)ab[(j * O + l) * cs];
        Ba[j][l] = (Acc)ab[(O * O + j * O + l) * cs];
      }
  }

  template <int ND>
  __device__ __forceinline__ static double wide(const Raw<K, TIER, ND>& r, int l) {
    return l < ND ? r.d[l] : widen(r.h[l]);
  }
  template <int ND>
  __device__ __forceinline__ static Acc acc_of(const Raw<K, TIER, ND>& r, int l) {
    if (l < ND) return (Acc)r.d[l];
    if constexpr (sizeof(Acc) == 8) return widen(r.h[l]);
    else return (Acc)r.h[l];
  }

  // Output mode j of the update from the two source cells x (cell i-s) and
  // y (cell i-s-1): FP64 for the FP64-stored modes, else in the arithmetic type.
  template <int ND>
  __device__ __forceinline__ static double out64(const Rows64<K, ND>& R, int j,
                                                 const Raw<K, TIER, ND>& x,
                                                 const Raw<K, TIER, ND>& y) {
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < O; ++l) acc = fma(R.A[j][l], wide(x, l), acc);
#pragma unroll
    for (int l = 0; l < O; ++l) acc = fma(R.B[j][l], wide(y, l), acc);
    return acc;
  }
  template <int ND>
  __device__ __forceinline__ Acc out_acc(int j, const Raw<K, TIER, ND>& x,
                                         const Raw<K, TIER, ND>& y) const {
    Acc acc = 0;
#pragma unroll
    for (int l = 0; l < O; ++l) acc = fma(Aa[j][l], acc_of(x, l), acc);
#pragma unroll
    for (int l = 0; l < O; ++l) acc = fma(Ba[j][l], acc_of(y, l), acc);
    return acc;
  }
};

// ---------------------------------------------------------------------------
// FP16 storage with per-mode power-of-two scaling.  A narrow plane p of an
// FP16 state may hold c * 2^e[p]: loads multiply by 2^-e of the input plane
// (exact), stores by 2^e of the output plane before the RNE conversion (exact
// scaling, so the stored value is the rounding of c onto FP16 with its
// exponent range moved by -e).  With scaling on, every wave also records the
// absolute maximum of each output plane it computed (before scaling) in a
// partial array [plane][slot], one slot per wave, from which a follow-up
// kernel takes the plane's absmax.  Unscaled FP16 runs the same code with
// factors 1.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float pow2f(int32_t e) { return __builtin_amdgcn_ldexpf(1.0f, e); }

// Maximum over the 64 lanes of a wave (every lane active), in registers:
// quad permutes (lane ^ 1, lane ^ 2) and row rotations (by 4, 8) give every
// lane the maximum of its row of 16; the four rows meet through readlane.
// The result is wave-uniform.  fmaxf ignores NaN operands, as in any order.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                               0xF, 0xF, true));
}

__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp_f<0xB1>(v));     // quad_perm [1, 0, 3, 2]
  v = fmaxf(v, dpp_f<0x4E>(v));     // quad_perm [2, 3, 0, 1]
  v = fmaxf(v, dpp_f<0x124>(v));    // row_ror 4
  v = fmaxf(v, dpp_f<0x128>(v));    // row_ror 8
  const int b = __builtin_bit_cast(int, v);
  const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 0));
  const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 16));
  const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 32));
  const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 48));
  return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}

// Stored value -> register value (the FP16 tier widens and unscales).
template <int TIER, class T>
__device__ __forceinline__ typename Tier<TIER>::R to_reg(T v, float fin) {
  if constexpr (TIER == 3) return (float)v * fin;
  else return v;
}

// Plane pointers of one spectator tuple.
template <int K, int TIER, int ND>
struct Planes {
  static constexpr int O = K + 1;
  using T = typename Tier<TIER>::T;
  const double* ind[O];
  double* outd[O];
  const T* inh[O];
  T* outh[O];
  float fin[O], fout[O];   // FP16 tier: 2^-e of the input planes, 2^e of the output planes
  int32_t hp[O];           // FP16 tier: hi plane of mode l (absmax partials)

  __device__ __forceinline__ void bind(const SweepArgs& a, const TupleMap& tm) {
    const T* hin = reinterpret_cast<const T*>(a.in_hi);
    T* hout = reinterpret_cast<T*>(a.out_hi);
#pragma unroll
    for (int l = 0; l < O; ++l) {
      const int64_t off = (int64_t)tm.idx[l] * a.cells;
      if (l < ND) {
        ind[l] = a.in_lo + off;
        outd[l] = a.out_lo + off;
      } else {
        inh[l] = hin + off;
        outh[l] = hout + off;
        if constexpr (TIER == 3) {
          hp[l] = tm.idx[l];
          if (a.in_exp) {
            fin[l] = pow2f(-a.in_exp[tm.idx[l]]);
            fout[l] = pow2f(a.out_exp[tm.idx[l]]);
          } else {
            fin[l] = 1.0f;
            fout[l] = 1.0f;
          }
        }
      }
    }
  }
  __device__ __forceinline__ void load(int64_t c, Raw<K, TIER, ND>& r) const {
#pragma unroll
    for (int l = 0; l < O; ++l) {
      if (l < ND) r.d[l] = ind[l][c];
      else r.h[l] = to_reg<TIER>(inh[l][c], fin[l]);
    }
  }
  __device__ __forceinline__ void copy_from(const Planes& o) {
#pragma unroll
    for (int l = 0; l < O; ++l) {
      if (l < ND) {
        ind[l] = o.ind[l];
        outd[l] = o.outd[l];
      } else {
        inh[l] = o.inh[l];
        outh[l] = o.outh[l];
        if constexpr (TIER == 3) {
          fin[l] = o.fin[l];
          fout[l] = o.fout[l];
          hp[l] = o.hp[l];
        }
      }
    }
  }
  // Narrow output j: the FP16 tier records |acc| in am[j] and stores acc * 2^e.
  __device__ __forceinline__ T put(int j, typename Tier<TIER>::Acc acc, float (&am)[O]) const {
    if constexpr (TIER == 3) {
      am[j] = fmaxf(am[j], fabsf(acc));
      return (T)(acc * fout[j]);
    } else {
      return narrow<T>(acc);
    }
  }
  template <int NT>
  __device__ __forceinline__ void store(int64_t c, const Mat<K, TIER>& M, const Rows64<K, ND>& R,
                                        const Raw<K, TIER, ND>& x, const Raw<K, TIER, ND>& y,
                                        float (&am)[O], bool active) const {
#pragma unroll
    for (int j = 0; j < O; ++j) {
      if (j < ND) {
        const double v = Mat<K, TIER>::out64(R, j, x, y);
        if (active) st_lane<NT>(outd[j] + c, v);
      } else {
        const T v = put(j, M.out_acc(j, x, y), am);
        if (active) st_lane<NT>(outh[j] + c, v);
      }
    }
  }
};

// End of one tuple of a wave in a scaled FP16 sweep: the wave's absmax of
// each narrow output plane goes to slot `slot` of that plane's partials.
// Every lane of the wave must be here (lanes beyond the grid work on a
// duplicate of a valid cell and do not store).
// One buffer store per tuple: lane j writes the maximum of the tuple's j-th
// narrow plane (wave-uniform values) and the other lanes an offset past the
// buffer, which writes nothing.  Without partials (unscaled FP16) the store
// goes to an empty buffer and touches no memory: the tuple loops then issue
// the same memory operations on every path, and the waits for the next
// tuple's loads do not wait for the stores issued after them (one counter
// covers loads and stores).  The host keeps the partials below 2^31 - 4 bytes.
template <int K, int TIER, int ND>
__device__ __forceinline__ void flush_amax(const SweepArgs& a, const Planes<K, TIER, ND>& pl,
                                           const float (&am)[K + 1], int32_t slot) {
  if constexpr (TIER == 3) {
    const bool on = a.amax_part != nullptr;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        a.amax_part, (short)0, on ? 0x7fffffff : 0, 0x00020000);
    const int32_t lane = (int32_t)(threadIdx.x & 63);
    float mv = 0.0f;
    int32_t off = 0x7fffffff;                  // past the buffer: no write
#pragma unroll
    for (int l = ND; l < K + 1; ++l) {
      const float m = on ? wave_max(am[l]) : 0.0f;
      if (lane == l - ND) {
        mv = m;
        off = (int32_t)(((int64_t)pl.hp[l] * a.nslot + slot) * 4);
      }
    }
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, mv), rs, off, 0, 0);
  }
}

template <int O>
__device__ __forceinline__ void zero_amax(float (&am)[O]) {
#pragma unroll
  for (int l = 0; l < O; ++l) am[l] = 0.0f;
}

// Dispatch on the number of leading FP64 modes of a tuple (0 .. NDMAX).
// Kernels are instantiated with NDMAX = 1 (the cell mean alone in FP64, or
// nothing) and with NDMAX = k+1 (any number of FP64 modes), so the common
// case does not carry the register cost of the all-FP64 tuple variants.
template <int NDMAX, class F>
__device__ __forceinline__ void dispatch_nd(int nd, F&& f) {
  if (nd == 0) {
    f(std::integral_constant<int, 0>{});
  } else if constexpr (NDMAX == 1) {
    f(std::integral_constant<int, 1>{});
  } else {
    if (nd == 1) f(std::integral_constant<int, 1>{});
    else if (nd == 2) f(std::integral_constant<int, (NDMAX >= 2 ? 2 : 1)>{});
    else if (nd == 3) f(std::integral_constant<int, (NDMAX >= 3 ? 3 : 1)>{});
    else f(std::integral_constant<int, (NDMAX >= 4 ? 4 : 1)>{});
  }
}

// ---------------------------------------------------------------------------
// Sweep along dimension 0, window form (N_0 % 4 == 0, 16-byte aligned
// buffers).  A thread produces 4 consecutive output cells i0..i0+3 of one line
// for one spectator tuple.  Their sources are the 5 cells i0-s-1 .. i0-s+3,
// which lie in two consecutive aligned 4-cell blocks of the line (periodic at
// block granularity since N_0 % 4 == 0); the thread loads both blocks with
// vector loads, picks the window with the in-block offset and writes its 4
// outputs with one vector store per plane.  Neighbouring threads load the same
// blocks, which the vector L1 serves: every coefficient crosses HBM once.
// A launch is one-shot (each thread a few loads, then stores, then exit),
// which on MI355X streams closer to peak than long-lived threads.  Where the
// window form does not apply, the group and lane forms below take the line.
// ---------------------------------------------------------------------------

template <class T>
struct Blk4 { T v[4]; };

// An aligned 4-cell block as loaded (vector words), unpacked only when used,
// so that a fetch does not make the wave wait for its data.
template <class T>
struct Raw4 {
  using V = typename std::conditional<
      sizeof(T) == 8, nt_d2,
      typename std::conditional<sizeof(T) == 4, nt_f4, nt_u2>::type>::type;
  static constexpr int W = sizeof(T) == 8 ? 2 : 1;
  V v[W];
};

template <class T>
__device__ __forceinline__ Raw4<T> fetch4(const T* p) {
  Raw4<T> r;
  const auto* q = reinterpret_cast<const typename Raw4<T>::V*>(p);
#pragma unroll
  for (int i = 0; i < Raw4<T>::W; ++i) r.v[i] = q[i];
  return r;
}

template <class T>
__device__ __forceinline__ Blk4<T> unpack4(const Raw4<T>& w) {
  Blk4<T> r;
  if constexpr (sizeof(T) == 8) {
    r.v[0] = w.v[0].x; r.v[1] = w.v[0].y; r.v[2] = w.v[1].x; r.v[3] = w.v[1].y;
  } else if constexpr (sizeof(T) == 4) {
    r.v[0] = w.v[0].x; r.v[1] = w.v[0].y; r.v[2] = w.v[0].z; r.v[3] = w.v[0].w;
  } else {
    const nt_u2 a = w.v[0];
    r.v[0] = __builtin_bit_cast(T, (uint16_t)(a.x & 0xffff));
    r.v[1] = __builtin_bit_cast(T, (uint16_t)(a.x >> 16));
    r.v[2] = __builtin_bit_cast(T, (uint16_t)(a.y & 0xffff));
    r.v[3] = __builtin_bit_cast(T, (uint16_t)(a.y >> 16));
  }
  return r;
}

template <class T>
__device__ __forceinline__ void store4(T* dst, const T (&v)[4]) {
  if constexpr (sizeof(T) == 8) {
    nt_d2* d = reinterpret_cast<nt_d2*>(dst);
    st_stream(d, nt_d2{v[0], v[1]});
    st_stream(d + 1, nt_d2{v[2], v[3]});
  } else if constexpr (sizeof(T) == 4) {
    st_stream(reinterpret_cast<nt_f4*>(dst), nt_f4{v[0], v[1], v[2], v[3]});
  } else {
    uint16_t b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) b[u] = __builtin_bit_cast(uint16_t, v[u]);
    st_stream(reinterpret_cast<nt_u2*>(dst), nt_u2{(uint32_t)b[0] | ((uint32_t)b[1] << 16),
                                                   (uint32_t)b[2] | ((uint32_t)b[3] << 16)});
  }
}

// The 5-cell window starting at offset d (0..3) of the 8 cells of blocks b0,
// b1, as two branch-free shifts (by d & 1, then by d & 2): 12 selects, no
// divergent control flow.
template <class T>
__device__ __forceinline__ void window5(const Blk4<T>& b0, const Blk4<T>& b1, int d, T (&w)[5]) {
  const bool s1 = (d & 1) != 0, s2 = (d & 2) != 0;
  const T u0 = s1 ? b0.v[1] : b0.v[0];
  const T u1 = s1 ? b0.v[2] : b0.v[1];
  const T u2 = s1 ? b0.v[3] : b0.v[2];
  const T u3 = s1 ? b1.v[0] : b0.v[3];
  const T u4 = s1 ? b1.v[1] : b1.v[0];
  const T u5 = s1 ? b1.v[2] : b1.v[1];
  const T u6 = s1 ? b1.v[3] : b1.v[2];
  w[0] = s2 ? u2 : u0;
  w[1] = s2 ? u3 : u1;
  w[2] = s2 ? u4 : u2;
  w[3] = s2 ? u5 : u3;
  w[4] = s2 ? u6 : u4;
}

template <int K, int TIER, int ND>
struct Win {               // the source cells of one tuple: the 5-cell window of the
  Raw<K, TIER, ND> w[8];   // window form, or (x_u, y_u) at (2u, 2u+1) in the group form
};

// Where the source cells of a thread's output cells lie.  Window form: two
// aligned 4-cell blocks of the line and the offset in the first.  Group
// form: the thread's outputs are cells i0 + u step (u < n, step =
// ceil(N_0 / 4)) of its line, interleaved with the other threads of the line
// so that a wave's lanes touch consecutive cells; x[u], y[u] are the line
// offsets of output u's sources i - s and i - s - 1.
template <bool GROUP> struct Geo;
template <> struct Geo<false> { int32_t blk0, blk1, d; };
template <> struct Geo<true> { int32_t x[4], y[4]; int32_t n, step; };

// The source cells of one tuple as loaded: two raw 4-cell blocks per plane
// (window form) or the two sources of each of 4 outputs per plane (group
// form, x_u at 2u and y_u at 2u+1).
template <int K, int TIER, int ND, bool GROUP>
struct Fetched {
  using T = typename Tier<TIER>::T;
  static constexpr int O = K + 1;
  static constexpr int NV = GROUP ? 8 : 2;
  typename std::conditional<GROUP, double, Raw4<double>>::type d[O][NV];   // l < ND
  typename std::conditional<GROUP, T, Raw4<T>>::type h[O][NV];             // l >= ND
};

template <int K, int TIER, int ND, bool GROUP>
__device__ __forceinline__ void contig_fetch(const Planes<K, TIER, ND>& pl, int64_t lb,
                                             const Geo<GROUP>& g, Fetched<K, TIER, ND, GROUP>& F) {
  constexpr int O = K + 1;
#pragma unroll
  for (int l = 0; l < O; ++l) {
    if constexpr (GROUP) {           // one load per source of each output
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (l < ND) {
          F.d[l][2 * u] = pl.ind[l][lb + g.x[u]];
          F.d[l][2 * u + 1] = pl.ind[l][lb + g.y[u]];
        } else {
          F.h[l][2 * u] = pl.inh[l][lb + g.x[u]];
          F.h[l][2 * u + 1] = pl.inh[l][lb + g.y[u]];
        }
      }
    } else if (l < ND) {
      F.d[l][0] = fetch4(pl.ind[l] + lb + 4 * g.blk0);
      F.d[l][1] = fetch4(pl.ind[l] + lb + 4 * g.blk1);
    } else {
      F.h[l][0] = fetch4(pl.inh[l] + lb + 4 * g.blk0);
      F.h[l][1] = fetch4(pl.inh[l] + lb + 4 * g.blk1);
    }
  }
}

template <int K, int TIER, int ND, bool GROUP>
__device__ __forceinline__ void copy_fetched(Fetched<K, TIER, ND, GROUP>& dst,
                                             const Fetched<K, TIER, ND, GROUP>& src) {
#pragma unroll
  for (int l = 0; l < K + 1; ++l)
#pragma unroll
    for (int u = 0; u < Fetched<K, TIER, ND, GROUP>::NV; ++u) {
      if (l < ND) dst.d[l][u] = src.d[l][u];
      else dst.h[l][u] = src.h[l][u];
    }
}

// The 5-cell window of each plane from the fetched cells.
template <int K, int TIER, int ND, bool GROUP>
__device__ __forceinline__ void contig_select(const Planes<K, TIER, ND>& pl, const Geo<GROUP>& g,
                                              const Fetched<K, TIER, ND, GROUP>& F,
                                              Win<K, TIER, ND>& W) {
  constexpr int O = K + 1;
  using T = typename Tier<TIER>::T;
#pragma unroll
  for (int l = 0; l < O; ++l) {
    if constexpr (GROUP) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (l < ND) W.w[u].d[l] = F.d[l][u];
        else W.w[u].h[l] = to_reg<TIER>(F.h[l][u], pl.fin[l]);
      }
    } else if (l < ND) {
      double m[5];
      window5<double>(unpack4(F.d[l][0]), unpack4(F.d[l][1]), g.d, m);
#pragma unroll
      for (int u = 0; u < 5; ++u) W.w[u].d[l] = m[u];
    } else {
      T h[5];
      window5<T>(unpack4(F.h[l][0]), unpack4(F.h[l][1]), g.d, h);
#pragma unroll
      for (int u = 0; u < 5; ++u) W.w[u].h[l] = to_reg<TIER>(h[u], pl.fin[l]);
    }
  }
}

template <int K, int TIER, int ND, bool GROUP>
__device__ __forceinline__ void contig_store(const SweepArgs& a, const Planes<K, TIER, ND>& pl,
                                             int64_t c, const Geo<GROUP>& g,
                                             const Mat<K, TIER>& M, const Rows64<K, ND>& R,
                                             const Win<K, TIER, ND>& W, int32_t slot,
                                             bool active) {
  constexpr int O = K + 1;
  using T = typename Tier<TIER>::T;
  float am[O];
  zero_amax(am);
#pragma unroll
  for (int j = 0; j < O; ++j) {
    if constexpr (GROUP) {           // one store per output cell; the line's last ones partial
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u < g.n) {
          const int64_t cu = c + (int64_t)u * g.step;
          if (j < ND) {
            const double v = Mat<K, TIER>::out64(R, j, W.w[2 * u], W.w[2 * u + 1]);
            if (active) pl.outd[j][cu] = v;
          } else {
            const T v = pl.put(j, M.out_acc(j, W.w[2 * u], W.w[2 * u + 1]), am);
            if (active) pl.outh[j][cu] = v;
          }
        }
      }
    } else if (j < ND) {
      double o4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) o4[u] = Mat<K, TIER>::out64(R, j, W.w[u + 1], W.w[u]);
      if (active) store4<double>(pl.outd[j] + c, o4);
    } else {
      T o4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) o4[u] = pl.put(j, M.out_acc(j, W.w[u + 1], W.w[u]), am);
      if (active) store4<T>(pl.outh[j] + c, o4);
    }
  }
  flush_amax<K, TIER, ND>(a, pl, am, slot);
}

template <int K, int TIER, int ND, bool GROUP>
__device__ __forceinline__ void contig_single(const SweepArgs& a, const TupleMap& tm,
                                              const Mat<K, TIER>& M, int64_t lb,
                                              const Geo<GROUP>& g, int64_t c, int32_t slot,
                                              bool active) {
  Planes<K, TIER, ND> pl;
  pl.bind(a, tm);
  Rows64<K, ND> R;
  R.load(M.ab, M.cs);
  Fetched<K, TIER, ND, GROUP> F;
  contig_fetch<K, TIER, ND, GROUP>(pl, lb, g, F);
  Win<K, TIER, ND> W;
  contig_select<K, TIER, ND, GROUP>(pl, g, F, W);
  contig_store<K, TIER, ND, GROUP>(a, pl, c, g, M, R, W, slot, active);
}

// One thread: 4 output cells of one line (consecutive in the window form,
// interleaved with the line's other threads in the group form), for the
// spectator tuples [q, qe) in turn (the line's s, A and B are loaded once; across a run
// of tuples without FP64 modes, the loads of the next tuple are issued before
// the current tuple is computed and stored).  When every lane of the wave
// works on lines that share one table entry (the common case: the
// displacement of a dimension-0 sweep rarely depends on dimension 1), the
// entry is read with scalar loads and the matrices live in scalar registers.
template <int K, int TIER, int NDMAX, bool GROUP>
__device__ __forceinline__ void contig_body(const SweepArgs& a, int32_t c, int32_t line,
                                            int32_t i0, int32_t t, int32_t q, int32_t qe,
                                            int32_t slot, bool active) {
  constexpr int O = K + 1;
  const int32_t N = a.N;
  const int32_t s = a.s_tab[t];
  int32_t w0 = i0 - s - 1;
  if (w0 < 0) w0 += N;
  Geo<GROUP> geo;
  if constexpr (GROUP) {
    // outputs i0 + u step; sources (i - s) and (i - s - 1) mod N, s in [0, N)
    const int32_t step = (N + 3) >> 2;
    geo.step = step;
    geo.n = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int32_t i = i0 + u * step;
      if (i < N) ++geo.n;
      else i = i0;                     // past the line: a valid duplicate, not stored
      int32_t x = i - s;
      if (x < 0) x += N;
      int32_t y = x - 1;
      if (y < 0) y += N;
      geo.x[u] = x;
      geo.y[u] = y;
    }
  } else {
    const int32_t nb = N >> 2;
    geo.blk0 = w0 >> 2;
    geo.d = w0 & 3;
    geo.blk1 = (geo.blk0 + 1 == nb) ? 0 : geo.blk0 + 1;
  }
  const int64_t lb = (int64_t)line * N;
  Mat<K, TIER> M;
  M.load(a.ab_tab + t, a.ab_cs);
  while (q < qe) {
    TupleMap tm = tuple_map<NDMAX>(a, q * O, 1, O);
    if (tm.nd != 0) {
      dispatch_nd<NDMAX>(tm.nd, [&](auto ndc) {
        contig_single<K, TIER, decltype(ndc)::value, GROUP>(a, tm, M, lb, geo, c, slot, active);
      });
      ++q;
      continue;
    }
    // a run of tuples without FP64 modes: the next tuple's loads are issued
    // before the current tuple is selected, computed and stored, and stay in
    // flight until its turn
    // Two register sets in turn (no copies: moving a register whose load is
    // in flight would wait for it).
    Planes<K, TIER, 0> pa, pb;
    Rows64<K, 0> R0;
    Fetched<K, TIER, 0, GROUP> fa, fb;
    pa.bind(a, tm);
    contig_fetch<K, TIER, 0, GROUP>(pa, lb, geo, fa);
    // binds and fetches tuple qn if it exists and has no FP64 mode
    auto next = [&](int32_t qn, Planes<K, TIER, 0>& p, Fetched<K, TIER, 0, GROUP>& f) {
      if (qn >= qe) return false;
      const TupleMap t1 = tuple_map<NDMAX>(a, qn * O, 1, O);
      if (t1.nd != 0) return false;
      p.bind(a, t1);
      contig_fetch<K, TIER, 0, GROUP>(p, lb, geo, f);
      return true;
    };
    auto process = [&](const Planes<K, TIER, 0>& p, const Fetched<K, TIER, 0, GROUP>& f) {
      Win<K, TIER, 0> W;
      contig_select<K, TIER, 0, GROUP>(p, geo, f, W);
      contig_store<K, TIER, 0, GROUP>(a, p, c, geo, M, R0, W, slot, active);
    };
    for (;;) {
      const bool mb = next(q + 1, pb, fb);
      process(pa, fa);
      ++q;
      if (!mb) break;
      const bool ma = next(q + 1, pa, fa);
      process(pb, fb);
      ++q;
      if (!ma) break;
    }
  }
}

// Group g (4 cells) of the dimension-0 sweep, tuples [q, qe).  In a scaled
// FP16 sweep, lanes past the last group redo the last group without storing
// it, so that whole waves reach the absmax reductions.
template <int K, int TIER, int NDMAX>
__device__ __forceinline__ void contig_group(const SweepArgs& a, int64_t g, int32_t q,
                                             int32_t qe, int32_t slot) {
  const int64_t groups = a.cells >> 2;
  bool active = true;
  if (g >= groups) {
    if constexpr (TIER != 3) {
      return;
    } else {
      if (!a.amax_part) return;
      g = groups - 1;
      active = false;
    }
  }
  const int32_t c = (int32_t)(g << 2);
  const int32_t line = (int32_t)a.fN.div((uint32_t)c);
  const int32_t i0 = c - line * a.N;
  const int32_t t = table_index(a.map, 0, line);
  const int32_t t0 = __builtin_amdgcn_readfirstlane(t);
  if (__all(t == t0)) contig_body<K, TIER, NDMAX, false>(a, c, line, i0, t0, q, qe, slot, active);
  else contig_body<K, TIER, NDMAX, false>(a, c, line, i0, t, q, qe, slot, active);
}

// Group gi of the dimension-0 sweep in the group form (any N_0, any
// alignment): cells g, g + ng, g + 2 ng, g + 3 ng (those below N_0) of line
// gi / ng, g = gi % ng, ng = ceil(N_0 / 4), so consecutive lanes of a line
// touch consecutive cells and the four cells share the line's table; tuples
// [q, qe).  Lanes past the last group act as in contig_group.
template <int K, int TIER, int NDMAX>
__device__ __forceinline__ void contig_group_any(const SweepArgs& a, int64_t gi, int32_t q,
                                                 int32_t qe, int32_t slot) {
  const int32_t ng = (a.N + 3) >> 2;
  const int64_t total = (int64_t)a.Q * ng;
  bool active = true;
  if (gi >= total) {
    if constexpr (TIER != 3) {
      return;
    } else {
      if (!a.amax_part) return;
      gi = total - 1;
      active = false;
    }
  }
  const int32_t line = (int32_t)a.fG.div((uint32_t)gi);
  const int32_t i0 = (int32_t)gi - line * ng;
  const int32_t c = line * a.N + i0;
  const int32_t t = table_index(a.map, 0, line);
  const int32_t t0 = __builtin_amdgcn_readfirstlane(t);
  if (__all(t == t0)) contig_body<K, TIER, NDMAX, true>(a, c, line, i0, t0, q, qe, slot, active);
  else contig_body<K, TIER, NDMAX, true>(a, c, line, i0, t, q, qe, slot, active);
}

// XCD-aware tile order.  Workgroups are dispatched round-robin over the 8
// XCDs (flat workgroup id w goes to XCD w % 8), each with its own L2, so
// tiles that share cache lines (neighbouring cells of a line, the halo rows
// of neighbouring row chunks) are fetched from HBM once per XCD that touches
// them.  With group size G > 0, the XCD's i-th workgroup (i = w / 8) takes
// tile ((i / G) * 8 + xcd) * G + i % G: runs of G consecutive tiles execute
// on one XCD one after the other, while the 8 XCDs still work on 8 adjacent
// runs (which keeps the HBM access stream local).  The tiles of the last,
// incomplete round keep the dispatch order.  G = -1 gives every XCD one
// contiguous eighth of the tiles; G = 0 keeps the dispatch order.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t w, uint32_t n, int32_t G) {
  if (G == 0) return w;
  const uint32_t xcd = w & 7, i = w >> 3;
  if (G < 0) {
    const uint32_t per = n >> 3, rem = n & 7;
    return xcd * per + min(xcd, rem) + i;
  }
  const uint32_t g = (uint32_t)G, round = 8 * g;
  if (w >= n / round * round) return w;
  return ((i / g) * 8 + xcd) * g + i % g;
}

// Tile of a strided-sweep workgroup: x column block, y tuple run, z row
// chunk group.  The tuple run is the slowest index.  Within a run, either the
// row chunk groups of a column block follow one another (nblk = 0), or the
// tiles go in memory order: the nblk column blocks of a slab (one value of the
// dimensions above the swept one) for one row chunk group, then the slab's
// next row chunk group, then the next slab, so that the tiles in flight cover
// one contiguous range of every plane.  XCD runs of length xcd are laid over
// either order; the hardware order (x fastest) is kept when both are off.
__device__ __forceinline__ void strided_tile(const SweepArgs& a, uint32_t& bx, uint32_t& by,
                                             uint32_t& bz) {
  bx = blockIdx.x;
  by = blockIdx.y;
  bz = blockIdx.z;
  if (!a.xcd && !a.nblk) return;
  const uint32_t gx = gridDim.x, gz = gridDim.z, xz = gx * gz;
  const uint32_t t = xcd_tile(blockIdx.x + gx * (blockIdx.y + gridDim.y * blockIdx.z),
                              xz * gridDim.y, a.xcd);
  by = t / xz;
  const uint32_t r = t - by * xz;
  if (a.nblk) {
    const uint32_t nb = (uint32_t)a.nblk;
    const uint32_t rest = r / nb;
    const uint32_t ih = rest / gz;
    bz = rest - ih * gz;
    bx = ih * nb + (r - rest * nb);
  } else {
    bx = r / gz;
    bz = r - bx * gz;
  }
}

template <int K, int TIER, int NDMAX>
__global__ __launch_bounds__(256) void sweep_contig_window_kernel(SweepArgs a) {
  uint32_t bx = blockIdx.x, by = blockIdx.y;
  if (a.xcd) {                 // tile order: x fastest, then y
    const uint32_t t = xcd_tile(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y, a.xcd);
    by = t / gridDim.x;
    bx = t - by * gridDim.x;
  }
  const int64_t g = (int64_t)bx * blockDim.x + threadIdx.x;
  const int32_t q = by * a.tuples;
  contig_group<K, TIER, NDMAX>(a, g, q, min(a.nspec, q + a.tuples),
                               (int32_t)(bx * (blockDim.x >> 6) + (threadIdx.x >> 6)));
}

template <int K, int TIER, int NDMAX>
__global__ __launch_bounds__(256) void sweep_contig_group_kernel(SweepArgs a) {
  uint32_t bx = blockIdx.x, by = blockIdx.y;
  if (a.xcd) {                 // tile order: x fastest, then y
    const uint32_t t = xcd_tile(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y, a.xcd);
    by = t / gridDim.x;
    bx = t - by * gridDim.x;
  }
  const int64_t gi = (int64_t)bx * blockDim.x + threadIdx.x;
  const int32_t q = by * a.tuples;
  contig_group_any<K, TIER, NDMAX>(a, gi, q, min(a.nspec, q + a.tuples),
                                   (int32_t)(bx * (blockDim.x >> 6) + (threadIdx.x >> 6)));
}

// ---------------------------------------------------------------------------
// Sweep along a dimension d > 0 (strided).  Lanes take consecutive cells of
// the flattened lower dimensions (contiguous in memory, coalesced in every
// plane).  A thread produces L consecutive rows i..i+L-1 along d, for a run of
// spectator tuples (blockIdx.y selects the run) in turn: its L+1 source rows
// per plane are loaded before any arithmetic, across tuples without FP64
// modes the loads of the next tuple are issued before the current tuple is
// computed, and the line's s, A and B (which may differ from lane to lane)
// are loaded once for all tuples.  Concurrent waves work on neighbouring
// cells of the same rows of the same planes, which keeps the HBM access
// stream local; the one extra source row per thread is the last row of the
// neighbouring chunk, loaded by a wave of the same workgroup.
// ---------------------------------------------------------------------------

// Source rows of a thread: L+1 rows from row i-s-1 of its own shift s, or
// with SP = 1 the L+2 rows from the wave's larger shift (see strided_cell).
template <int K, int TIER, int ND, int L, int SP = 0>
struct Rows {
  Raw<K, TIER, ND> v[L + 1 + SP];
};

template <int K, int TIER, int ND, int L, int SP>
__device__ __forceinline__ void strided_load(const Planes<K, TIER, ND>& pl, int64_t base,
                                             const int32_t (&roff)[L + 1 + SP],
                                             Rows<K, TIER, ND, L, SP>& R) {
  // all rows are loaded (row offsets wrap); only the stores are cut
#pragma unroll
  for (int u = 0; u <= L + SP; ++u) pl.load(base + roff[u], R.v[u]);
}

// dl ? x1 : x0, field by field (lanes one row below the wave's shift take
// their window one row further down)
template <int K, int TIER, int ND>
__device__ __forceinline__ Raw<K, TIER, ND> pick_row(bool dl, const Raw<K, TIER, ND>& x1,
                                                     const Raw<K, TIER, ND>& x0) {
  Raw<K, TIER, ND> r;
#pragma unroll
  for (int l = 0; l < K + 1; ++l) {
    if (l < ND) r.d[l] = dl ? x1.d[l] : x0.d[l];
    else r.h[l] = dl ? x1.h[l] : x0.h[l];
  }
  return r;
}

template <int K, int TIER, int ND, int L, int NT, int SP>
__device__ __forceinline__ void strided_store(const SweepArgs& a, const Planes<K, TIER, ND>& pl,
                                              int64_t base, int32_t r0, int32_t n,
                                              const Mat<K, TIER>& M, const Rows64<K, ND>& R64,
                                              const Rows<K, TIER, ND, L, SP>& R, bool dl,
                                              int32_t slot, bool active) {
  const int32_t P = a.P;
  float am[K + 1];
  zero_amax(am);
  auto row = [&](int u) {
    const int64_t c = base + (int64_t)(r0 + u) * P;
    if constexpr (SP == 0) {
      pl.template store<NT>(c, M, R64, R.v[u + 1], R.v[u], am, active);
    } else {
      const Raw<K, TIER, ND> x = pick_row<K, TIER, ND>(dl, R.v[u + 2], R.v[u + 1]);
      const Raw<K, TIER, ND> y = pick_row<K, TIER, ND>(dl, R.v[u + 1], R.v[u]);
      pl.template store<NT>(c, M, R64, x, y, am, active);
    }
  };
  if (n == L) {            // full chunk: no per-row predicate
#pragma unroll
    for (int u = 0; u < L; ++u) row(u);
  } else {                 // the last chunk of a line whose length L does not divide
#pragma unroll
    for (int u = 0; u < L; ++u)
      if (u < n) row(u);
  }
  flush_amax<K, TIER, ND>(a, pl, am, slot);
}

template <int K, int TIER, int ND, int L, int NT, int SP = 0>
__device__ __forceinline__ void strided_single(const SweepArgs& a, const TupleMap& tm,
                                               const Mat<K, TIER>& M, int64_t base,
                                               const int32_t (&roff)[L + 1 + SP], int32_t r0,
                                               int32_t n, bool dl, int32_t slot, bool active) {
  Planes<K, TIER, ND> pl;
  pl.bind(a, tm);
  Rows64<K, ND> R64;
  R64.load(M.ab, M.cs);
  Rows<K, TIER, ND, L, SP> R;
  strided_load<K, TIER, ND, L, SP>(pl, base, roff, R);
  strided_store<K, TIER, ND, L, NT, SP>(a, pl, base, r0, n, M, R64, R, dl, slot, active);
}

// One thread's column: table entry t, rows from i - s - 1 on.  SP = 0: s is
// the column's shift.  SP = 1: s is the larger of the wave's two shifts
// (modulo N) and dl says that the column's shift is one less.
template <int K, int TIER, int L, int NDMAX, int NT, int SP = 0>
__device__ __forceinline__ void strided_body(const SweepArgs& a, int32_t ilow, int32_t chunk,
                                             int32_t ihigh, int32_t t, int32_t s, bool dl,
                                             int32_t q, int32_t qe, int32_t slot, bool active) {
  constexpr int O = K + 1;
  const int32_t N = a.N, P = a.P, ms = a.mstride;
  const int64_t base = (int64_t)ihigh * P * N + ilow;
  const int32_t r0 = chunk * L;
  const int32_t n = min(L, N - r0);
  int32_t roff[L + 1 + SP];
  int32_t row = r0 - s - 1;
  if (row < 0) row += N;
#pragma unroll
  for (int u = 0; u <= L + SP; ++u) {
    roff[u] = row * P;
    if (++row == N) row = 0;
  }
  Mat<K, TIER> M;
  M.load(a.ab_tab + t, a.ab_cs);
  // mode base of tuple q, stepped without division: the low part (dims below
  // d) counts to ms, then the base jumps over the swept index's o-1 planes
  int32_t low = q % ms;
  int32_t m0 = low + (q / ms) * ms * O;
  auto advance = [&](int32_t& qq, int32_t& lw, int32_t& mm) {
    ++qq;
    ++mm;
    if (++lw == ms) {
      lw = 0;
      mm += ms * (O - 1);
    }
  };
  while (q < qe) {
    const TupleMap tm = tuple_map<NDMAX>(a, m0, ms, O);
    if (tm.nd != 0) {
      dispatch_nd<NDMAX>(tm.nd, [&](auto ndc) {
        strided_single<K, TIER, decltype(ndc)::value, L, NT, SP>(a, tm, M, base, roff, r0, n, dl,
                                                             slot, active);
      });
      advance(q, low, m0);
      continue;
    }
    // Two register sets in turn (no copies: moving a register whose load is
    // in flight would wait for it).
    Planes<K, TIER, 0> pa, pb;
    Rows64<K, 0> R64;
    Rows<K, TIER, 0, L, SP> ra, rb;
    pa.bind(a, tm);
    strided_load<K, TIER, 0, L, SP>(pa, base, roff, ra);
    // the tuple after (q, low, m0): binds and loads it if it exists and has no
    // FP64 mode; (q, low, m0) move on to it either way
    auto next = [&](Planes<K, TIER, 0>& p, Rows<K, TIER, 0, L, SP>& r) {
      advance(q, low, m0);
      if (q >= qe) return false;
      const TupleMap t1 = tuple_map<NDMAX>(a, m0, ms, O);
      if (t1.nd != 0) return false;
      p.bind(a, t1);
      strided_load<K, TIER, 0, L, SP>(p, base, roff, r);
      return true;
    };
    for (;;) {
      const bool mb = next(pb, rb);
      strided_store<K, TIER, 0, L, NT, SP>(a, pa, base, r0, n, M, R64, ra, dl, slot, active);
      if (!mb) break;
      const bool ma = next(pa, ra);
      strided_store<K, TIER, 0, L, NT, SP>(a, pb, base, r0, n, M, R64, rb, dl, slot, active);
      if (!ma) break;
    }
  }
}

// Column col, row chunk `chunk` of a strided sweep, tuples [q, qe).  The
// chunk is uniform across a wave; in a scaled FP16 sweep, lanes past the
// last column redo the last column without storing it, so that whole waves
// reach the absmax reductions.
template <int K, int TIER, int L, int NDMAX, int NT>
__device__ __forceinline__ void strided_cell(const SweepArgs& a, int32_t col, int32_t chunk,
                                             int32_t q, int32_t qe, int32_t slot) {
  if (chunk >= a.nchunk) return;
  const int32_t ncol = a.P * a.Q;
  bool active = true;
  if (col >= ncol) {
    if constexpr (TIER != 3) {
      return;
    } else {
      if (!a.amax_part) return;
      col = ncol - 1;
      active = false;
    }
  }
  const uint32_t ih = a.fP.div((uint32_t)col);
  const int32_t ilow = col - (int32_t)ih * a.P;
  const int32_t ihigh = (int32_t)ih;
  const int32_t t = table_index(a.map, ilow, ihigh);
  const int32_t t0 = __builtin_amdgcn_readfirstlane(t);
  if (__all(t == t0)) {
    strided_body<K, TIER, L, NDMAX, NT>(a, ilow, chunk, ihigh, t0, a.s_tab[t0], false, q, qe,
                                        slot, active);
    return;
  }
  // Shifts that differ across the wave put its lanes on different rows in
  // every load.  Where they take two values one apart (modulo N: a field
  // around zero gives N-1 and 0), the wave loads one more row, the same rows
  // in every lane, and each lane picks its window.  Equal shifts (entries
  // that differ in alpha only) and wider spreads take the general body.
  const int32_t s = a.s_tab[t];
  const int32_t s0 = __builtin_amdgcn_readfirstlane(s);
  const int32_t N = a.N;
  const int32_t up = s0 + 1 == N ? 0 : s0 + 1;
  const int32_t dn = s0 == 0 ? N - 1 : s0 - 1;
  const bool two_up = __all(s == s0 || s == up);
  const bool two = !__all(s == s0) && (two_up || __all(s == s0 || s == dn));
  if (two) {
    const int32_t shi = two_up ? up : s0;                // the larger of the two
    strided_body<K, TIER, L, NDMAX, NT, 1>(a, ilow, chunk, ihigh, t, shi, s != shi, q, qe, slot,
                                           active);
  } else {
    strided_body<K, TIER, L, NDMAX, NT>(a, ilow, chunk, ihigh, t, s, false, q, qe, slot, active);
  }
}

// Lane form of a sweep along any dimension: one output cell per lane,
// consecutive lanes on consecutive cells, tuples [q, qe).  Cell c is
// (ilow, row, ihigh) with c = (ihigh * N + row) * P + ilow, and the sweep of
// its column is the strided body with L = 1 and the cell's row as its row
// chunk: the sources c - s P and c - (s+1) P of a wave's lanes are contiguous
// (up to the periodic wrap), one access per plane and source, and every
// store of a wave writes 64 consecutive cells.  Along dimension 0 (P = 1) the
// column is the line itself.  Lanes past the last cell act as in
// contig_group.
template <int K, int TIER, int NDMAX, int NT>
__device__ __forceinline__ void lane_cell(const SweepArgs& a, int64_t c, int32_t q, int32_t qe,
                                          int32_t slot) {
  bool active = true;
  if (c >= a.cells) {
    if constexpr (TIER != 3) {
      return;
    } else {
      if (!a.amax_part) return;
      c = a.cells - 1;
      active = false;
    }
  }
  const uint32_t rest = a.fP.div((uint32_t)c);
  const int32_t ilow = (int32_t)c - (int32_t)rest * a.P;
  const uint32_t ih = a.fN.div(rest);
  const int32_t row = (int32_t)rest - (int32_t)ih * a.N;
  const int32_t ihigh = (int32_t)ih;
  const int32_t t = table_index(a.map, ilow, ihigh);
  const int32_t t0 = __builtin_amdgcn_readfirstlane(t);
  if (__all(t == t0))
    strided_body<K, TIER, 1, NDMAX, NT>(a, ilow, row, ihigh, t0, a.s_tab[t0], false, q, qe, slot,
                                        active);
  else
    strided_body<K, TIER, 1, NDMAX, NT>(a, ilow, row, ihigh, t, a.s_tab[t], false, q, qe, slot,
                                        active);
}

// Work decomposition: a wave takes 64 consecutive columns (column =
// ihigh * P + ilow, i.e. a cell of the transverse dimensions, consecutive
// columns contiguous in memory), the waves of a workgroup take consecutive
// row chunks of the same columns.  The halo row a wave loads is the last row
// its neighbour wave loads, so it is served by the CU's caches, and the
// waves share the columns' s, A, B in L1.  Tiles (x: column block, z: row
// chunk group, y: tuple run) are ordered z fastest, then x, then y, and laid
// over the XCDs so that tiles sharing lines (the halo row between row chunk
// groups, the cache lines split between column blocks when the rows are
// short) run on one XCD, one after the other.
template <int K, int TIER, int L, int NDMAX, int NT>
__global__ __launch_bounds__(256) void sweep_strided_kernel(SweepArgs a) {
  uint32_t bx, by, bz;
  strided_tile(a, bx, by, bz);
  const uint32_t gx = gridDim.x;
  // the workgroup's waves: cw side by side along the columns, waves / cw
  // stacked along the row chunks
  // the wave index is uniform across the wave: said so, the row chunk and
  // its length are scalar and the full-chunk test is a scalar branch
  const int32_t waves = (int32_t)(blockDim.x >> 6);
  const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  const int32_t cw = a.colwaves, zw = waves / cw;
  const int32_t wc = wave % cw, wz = wave / cw;
  const int32_t col = ((int32_t)bx * cw + wc) * 64 + (int32_t)(threadIdx.x & 63);
  const int32_t chunk = (int32_t)bz * zw + wz;
  const int32_t q = by * a.tuples;
  strided_cell<K, TIER, L, NDMAX, NT>(a, col, chunk, q, min(a.nspec, q + a.tuples),
                                  (int32_t)(bz * gx + bx) * waves + wave);
}

template <int K, int TIER, int NDMAX, int NT>
__global__ __launch_bounds__(256) void sweep_lane_kernel(SweepArgs a) {
  uint32_t bx = blockIdx.x, by = blockIdx.y;
  if (a.xcd) {                 // tile order: x fastest, then y
    const uint32_t t = xcd_tile(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y, a.xcd);
    by = t / gridDim.x;
    bx = t - by * gridDim.x;
  }
  const int64_t c = (int64_t)bx * blockDim.x + threadIdx.x;
  const int32_t q = by * a.tuples;
  lane_cell<K, TIER, NDMAX, NT>(a, c, q, min(a.nspec, q + a.tuples),
                              (int32_t)(bx * (blockDim.x >> 6) + (threadIdx.x >> 6)));
}

// Launch shape of a sweep: form 0 window, 1 group (dimension 0), 2 strided,
// 3 lane (any dimension).
inline bool sweep_grid(int dim, const SweepArgs& a, int& form, dim3& grid, dim3& block) {
  if (dim > 0 && a.lane) {
    form = 3;
    grid = dim3((unsigned)((a.cells + 255) / 256), (unsigned)((a.nspec + a.tuples - 1) / a.tuples));
    block = dim3(256);
    return true;
  }
  if (dim == 0) {
    if (contig_window_ok(a)) {
      const int64_t groups = a.cells >> 2;
      form = 0;
      grid = dim3((unsigned)((groups + 255) / 256), (unsigned)((a.nspec + a.tuples - 1) / a.tuples));
      block = dim3(256);
    } else if (!a.lane) {
      const int64_t groups = (int64_t)a.Q * ((a.N + 3) / 4);
      form = 1;
      grid = dim3((unsigned)((groups + 255) / 256), (unsigned)((a.nspec + a.tuples - 1) / a.tuples));
      block = dim3(256);
    } else {
      form = 3;
      grid = dim3((unsigned)((a.cells + 255) / 256), (unsigned)((a.nspec + a.tuples - 1) / a.tuples));
      block = dim3(256);
    }
    return true;
  }
  const int64_t ncol = (int64_t)a.P * a.Q;
  const int cw = a.colwaves;                         // waves side by side (columns)
  const int zw = std::min(a.nchunk, 4 / cw);         // waves stacked (row chunks)
  const int64_t gx = (ncol + 64 * cw - 1) / (64 * cw), gz = (a.nchunk + zw - 1) / zw;
  if (gz > 65535 || gx > 0x7fffffff) return false;
  form = 2;
  grid = dim3((unsigned)gx, (unsigned)((a.nspec + a.tuples - 1) / a.tuples), (unsigned)gz);
  block = dim3(64 * cw * zw);
  return true;
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

template <int K, int TIER, int KIND, int L>
__global__ __launch_bounds__(256) void batch_class_kernel(const SweepArgs* __restrict__ args,
                                                          const BatchItem* __restrict__ items,
                                                          int32_t xcd) {
  const BatchItem w = items[xcd_tile(blockIdx.x, gridDim.x, xcd)];
  const SweepArgs& a = args[w.prob];
  const int32_t q = w.qg * a.tuples;
  const int32_t qe = min(a.nspec, q + a.tuples);
  if constexpr (KIND == 0) {
    contig_group<K, TIER, 1>(a, (int64_t)w.x * blockDim.x + threadIdx.x, q, qe, 0);
  } else if constexpr (KIND == 1) {
    contig_group_any<K, TIER, 1>(a, (int64_t)w.x * blockDim.x + threadIdx.x, q, qe, 0);
  } else if constexpr (KIND == 3) {          // kinds 1 (rows 1) and 2 (rows 0) in the lane form
    lane_cell<K, TIER, 1, 0>(a, (int64_t)w.x * blockDim.x + threadIdx.x, q, qe, 0);
  } else {
    const int32_t col = w.x * 64 + (int32_t)(threadIdx.x & 63);
    const int32_t chunk = w.z * (int32_t)(blockDim.x >> 6) +
                          __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    strided_cell<K, TIER, L, 1, 0>(a, col, chunk, q, qe, 0);
  }
}

}  // namespace sldg
