// Strided projection sweep with its sources staged through LDS (L. Einkemmer,
// arXiv 1603.07008, section II-A update rule out[i] = A in[i-s] + B in[i-s-1]
// along a dimension d > 0).
//
// The direct strided kernel (sldg_sweep.h) loads one value per lane per plane
// and row: 128 bytes per wave instruction for the 16-bit tiers, 256 for FP32.
// The address unit of a CU takes a wave instruction in the same number of
// cycles whatever the lane width up to 4 bytes, so the narrow tiers issue
// twice (FP32) or four times (16-bit) the instructions per byte of the FP64
// tier, and the 16-bit sweeps are capped by instruction issue, not by HBM.
// Here a workgroup loads the rows its threads need for one spectator tuple
// with 16-byte lane accesses into LDS; each thread then takes its own column
// from LDS with its own shift (the shift may differ from column to column),
// and computes and stores its L output rows exactly as the direct kernel does
// (same Mat evaluation, same rounding, same stores), so the results are
// bitwise the direct kernel's.
//
// Tile: C = 64 cw consecutive columns (one run of a row: P % C == 0) and
// RT = (4 / cw) L output rows from r0.  With the shifts of its columns within
// [sref + dmin, sref + dmax] (circularly, around the shift sref of its first
// column), its threads read rows r0 - sref - dmax - 1 .. r0 + RT - 1 - sref -
// dmin of each plane: U = RT + 1 + (dmax - dmin) rows.  A tile whose spread
// needs more rows than the LDS holds runs the direct per-thread path.  Tuples
// alternate between two LDS buffers, and the loads of the next tuple are
// issued before the current one is computed: one barrier per tuple.
#pragma once

#include "sldg_sweep.h"

namespace sldg {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // one 16-byte access

// Shape constants of a staged tile (storage type size SZ bytes).
template <int K, int SZ, int L, int CW>
struct StagedShape {
  static constexpr int O = K + 1;
  static constexpr int C = 64 * CW;          // columns
  static constexpr int Z = 4 / CW;           // waves stacked along the rows
  static constexpr int RT = Z * L;           // output rows
  static constexpr int VPC = 16 / SZ;        // values per 16-byte access
  static constexpr int CH = C / VPC;         // 16-byte accesses per row
  static constexpr int SLOTS = staged_slots(K, SZ, L, CW);   // 16-byte loads per thread
  static constexpr int UMAX = staged_umax(K, SZ, L, CW);     // rows per plane they cover
  static constexpr int BUF = O * UMAX * C;                   // values per LDS buffer
  static constexpr int64_t LDS_BYTES = staged_lds_bytes(K, SZ, L, CW);
  static_assert(SLOTS * 256 >= O * (RT + 1) * CH, "slots cover a tile without spread");
  static_assert(2LL * BUF * SZ == LDS_BYTES, "LDS size");
};

// Direct path of the staged kernel's thread (tiles whose shift spread does not
// fit, and the cell mean's tuple): tuples [q, qe) of its column and row chunk
// one after the other, with one register set (the staged path's registers
// bound the kernel, not this path's).
template <int K, int TIER, int L, int NT>
__device__ __forceinline__ void staged_direct(const SweepArgs& a, int32_t ilow, int32_t chunk,
                                           int32_t ihigh, int32_t t, int32_t q, int32_t qe,
                                           int32_t slot) {
  constexpr int O = K + 1;
  const int32_t s = a.s_tab[t];
  const int32_t N = a.N, P = a.P, ms = a.mstride;
  const int64_t base = (int64_t)ihigh * P * N + ilow;
  const int32_t r0 = chunk * L;
  const int32_t n = min(L, N - r0);
  int32_t roff[L + 1];
  int32_t row = r0 - s - 1;
  if (row < 0) row += N;
#pragma unroll
  for (int u = 0; u <= L; ++u) {
    roff[u] = row * P;
    if (++row == N) row = 0;
  }
  Mat<K, TIER> M;
  M.load(a.ab_tab + t, a.ab_cs);
  for (; q < qe; ++q) {
    const int32_t low = q % ms;
    const TupleMap tm = tuple_map<1>(a, low + (q / ms) * ms * O, ms, O);
    dispatch_nd<1>(tm.nd, [&](auto ndc) {
      strided_single<K, TIER, decltype(ndc)::value, L, NT>(a, tm, M, base, roff, r0, n, false,
                                                         slot, true);
    });
  }
}

template <int K, int TIER, int L, int CW, int NT>
__global__ __launch_bounds__(256) void sweep_staged_kernel(SweepArgs a) {
  using T = typename Tier<TIER>::T;
  using S = StagedShape<K, (int)sizeof(T), L, CW>;
  constexpr int O = S::O, C = S::C, RT = S::RT, VPC = S::VPC, CH = S::CH;
  constexpr int SLOTS = S::SLOTS, UMAX = S::UMAX;
  extern __shared__ __align__(16) unsigned char staged_lds[];
  T* tile = reinterpret_cast<T*>(staged_lds);
  __shared__ int32_t red[3];

  // tile coordinates: as the direct kernel (x column block, y tuple run,
  // z row chunk group, in the same order)
  uint32_t bx, by, bz;
  strided_tile(a, bx, by, bz);
  const uint32_t gx = gridDim.x;
  const int32_t tid = (int32_t)threadIdx.x;
  const int32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int32_t wc = wave % CW, wz = wave / CW;
  const int32_t cl = wc * 64 + (tid & 63);           // column within the tile
  const int32_t col0 = (int32_t)bx * C;
  const int32_t col = col0 + cl;
  const int32_t chunk = (int32_t)bz * S::Z + wz;     // the thread's row chunk
  const bool rows_ok = chunk < a.nchunk;             // wave-uniform
  int32_t q = (int32_t)by * a.tuples;
  const int32_t qe = min(a.nspec, q + a.tuples);
  const int32_t slot = (int32_t)(bz * gx + bx) * 4 + wave;
  const int32_t N = a.N, P = a.P, ms = a.mstride;

  const uint32_t ih = a.fP.div((uint32_t)col);
  const int32_t ilow = col - (int32_t)ih * P;
  const int32_t ihigh = (int32_t)ih;
  const int32_t t = table_index(a.map, ilow, ihigh);
  const int32_t s = a.s_tab[t];

  // circular spread of the tile's shifts around that of its first column
  if (tid == 0) {
    red[0] = s;
    red[1] = INT32_MAX;
    red[2] = INT32_MIN;
  }
  __syncthreads();
  const int32_t sref = red[0];
  int32_t ds = s - sref;                             // in (-N, N)
  if (2 * ds > N) ds -= N;
  else if (2 * ds <= -N) ds += N;
  atomicMin(&red[1], ds);
  atomicMax(&red[2], ds);
  __syncthreads();
  const int32_t dmin = red[1], dmax = red[2];
  const int32_t U = RT + 1 + (dmax - dmin);
  // workgroup-uniform: a spread the buffers do not hold, or a ragged last
  // tile (the host stages only grids of whole tiles, N % RT == 0, so that
  // the staged loop has no partial chunk and no idle wave)
  if (U > UMAX || N % RT != 0) {
    if (rows_ok) staged_direct<K, TIER, L, NT>(a, ilow, chunk, ihigh, t, q, qe, slot);
    return;
  }

  // tuple qq: its first mode (qq mod ms) + (qq - qq mod ms) O; a tuple
  // without FP64 modes has its plane l at hi plane (first mode - n_lo) + l ms
  auto mode0 = [&](int32_t qq) {
    const int32_t lw = qq % ms;
    return lw + (qq - lw) * O;
  };
  // the cell mean's tuple (the first tuple, when the mean is FP64) takes the
  // direct path: its FP64 plane is not staged
  if (q < qe && mode0(q) < a.n_lo) {
    if (rows_ok) staged_direct<K, TIER, L, NT>(a, ilow, chunk, ihigh, t, q, q + 1, slot);
    ++q;
  }
  if (q >= qe) return;

  // Every access of the staged path is a buffer access relative to the
  // tuple's plane 0 (a buffer over the tuple's planes; the host keeps its
  // byte extent below 2^31).  Offsets at or past the extent read zeros and
  // drop stores without touching memory: lanes past the tile use the offset
  // kOut, and the loads past the last tuple an empty buffer.  So every round
  // issues the same loads and stores, and the waits for a tuple's loads do not
  // wait for the stores issued after them.
  constexpr uint32_t kOut = 0x80000000u;
  constexpr int32_t kRsrcFlags = 0x00020000;   // raw buffer, 32-bit data format
  const uint32_t extent = (uint32_t)(((int64_t)(O - 1) * ms + 1) * a.cells * (int64_t)sizeof(T));

  // load slots: 16-byte access i = j * 256 + tid of the tile, i = (l U + u)
  // CH + c (plane l, tile row u, access c of the row), at byte offset goff[j]
  // from the tuple's plane 0 (plane l is l * ms planes further); rows wrap
  // periodically
  const int32_t r0 = (int32_t)bz * RT;
  const int32_t rb = r0 - sref - dmax - 1;
  const uint32_t ih0 = a.fP.div((uint32_t)col0);
  const uint32_t tbase = ih0 * (uint32_t)P * (uint32_t)N + (uint32_t)(col0 - (int32_t)ih0 * P);
  const int32_t per_plane = U * CH;
  const int32_t total = O * per_plane;
  uint32_t goff[SLOTS];
  uint32_t used = 0;
#pragma unroll
  for (int j = 0; j < SLOTS; ++j) {
    const int32_t i = j * 256 + tid;
    goff[j] = kOut;
    if (i < total) {
      used |= 1u << j;
      const int32_t l = i / per_plane;
      const int32_t rem = i - l * per_plane;
      const int32_t u = rem / CH;
      const int32_t c = rem - u * CH;
      int32_t row = (rb + u) % N;
      if (row < 0) row += N;
      goff[j] = ((uint32_t)l * (uint32_t)ms * (uint32_t)a.cells + tbase + (uint32_t)row * P +
                 (uint32_t)(c * VPC)) * (uint32_t)sizeof(T);
    }
  }
  // store slots: 16-byte access i = j * 256 + tid of the output tile
  // [plane l][row r < RT][column], rows r0 .. r0 + RT - 1 (< N)
  constexpr int OSLOTS = (O * RT * CH + 255) / 256;
  uint32_t ooff[OSLOTS];
  int32_t oread[OSLOTS];       // its element in the output tile (0 for lanes past it)
#pragma unroll
  for (int j = 0; j < OSLOTS; ++j) {
    const int32_t i = j * 256 + tid;
    ooff[j] = kOut;
    oread[j] = 0;
    if (i < O * RT * CH) {
      const int32_t l = i / (RT * CH);
      const int32_t rem = i - l * (RT * CH);
      const int32_t r = rem / CH;
      const int32_t c = rem - r * CH;
      ooff[j] = ((uint32_t)l * (uint32_t)ms * (uint32_t)a.cells + tbase + (uint32_t)(r0 + r) * P +
                 (uint32_t)(c * VPC)) * (uint32_t)sizeof(T);
      oread[j] = i * VPC;
    }
  }
  const T* hin = reinterpret_cast<const T*>(a.in_hi);
  T* hout = reinterpret_cast<T*>(a.out_hi);
  auto fetch = [&](u32x4 (&buf)[SLOTS], int32_t qq) {
    const bool live = qq < qe;                       // uniform
    const T* base = hin + (live ? (int64_t)(mode0(qq) - a.n_lo) * a.cells : 0);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(base), (short)0, live ? (int32_t)extent : 0, kRsrcFlags);
#pragma unroll
    for (int j = 0; j < SLOTS; ++j)
      buf[j] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int32_t)goff[j], 0, 0));
  };
  auto put = [&](const u32x4 (&buf)[SLOTS], T* dst) {
#pragma unroll
    for (int j = 0; j < SLOTS; ++j)
      if (used & (1u << j)) *reinterpret_cast<u32x4*>(dst + (j * 256 + tid) * VPC) = buf[j];
  };

  // the thread's column: its source rows start at tile row u0 of each plane,
  // its outputs are rows wz L .. wz L + L - 1 of the output tile
  const int32_t u0 = wz * L + (dmax - ds);
  Mat<K, TIER> M;
  M.load(a.ab_tab + t, a.ab_cs);
  Planes<K, TIER, 0> pl;
  auto bind = [&](int32_t qq) { pl.bind(a, tuple_map<1>(a, mode0(qq), ms, O)); };

  // Two LDS buffers (X: this tuple, Y: the next) and two register sets (the
  // loads of the next two tuples in flight).  A round: read the thread's
  // source rows from X; barrier; compute, writing the outputs over X (as the
  // output tile); write the next tuple from its register set into Y and
  // reload that set with the tuple three ahead; barrier; store X's outputs.
  // The first two rounds are peeled off the loop, so that the loop is
  // entered after the same sequence of loads and stores it repeats.
  u32x4 bufA[SLOTS], bufB[SLOTS];
  fetch(bufA, q);
  fetch(bufB, q + 1);
  put(bufA, tile);
  fetch(bufA, q + 2);
  bind(q);
  __syncthreads();
  int32_t par = 0;
  auto round = [&](u32x4 (&buf)[SLOTS]) {
    T* X = tile + par * S::BUF;
    Rows<K, TIER, 0, L> R;
    {
      const T* src = X + u0 * C + cl;
#pragma unroll
      for (int v = 0; v <= L; ++v)
#pragma unroll
        for (int l = 0; l < O; ++l)
          R.v[v].h[l] = to_reg<TIER>(src[(l * U + v) * C], pl.fin[l]);
    }
    __syncthreads();
    {
      float am[O];
      zero_amax(am);
      T* dst = X + (wz * L) * C + cl;
#pragma unroll
      for (int u = 0; u < L; ++u)
#pragma unroll
        for (int j = 0; j < O; ++j)
          dst[(j * RT + u) * C] = pl.put(j, M.template out_acc<0>(j, R.v[u + 1], R.v[u]), am);
      flush_amax<K, TIER, 0>(a, pl, am, slot);
    }
    const __amdgpu_buffer_rsrc_t ws = __builtin_amdgcn_make_buffer_rsrc(
        hout + (int64_t)(mode0(q) - a.n_lo) * a.cells, (short)0, (int32_t)extent, kRsrcFlags);
    // the next tuple's write and the reload run in every round (past the
    // last tuple they move zeros from an empty buffer into a buffer no round
    // reads), so that every round issues the same memory operations
    const bool has_next = q + 1 < qe;
    put(buf, tile + (par ^ 1) * S::BUF);
    fetch(buf, q + 3);
    if (has_next) bind(q + 1);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < OSLOTS; ++j)
      __builtin_amdgcn_raw_buffer_store_b128(
          __builtin_bit_cast(__attribute__((ext_vector_type(4))) uint32_t,
                             *reinterpret_cast<const u32x4*>(X + oread[j])),
          ws, (int32_t)ooff[j], 0, NT > 0 ? 2 : 0);
    par ^= 1;
    ++q;
    return has_next;
  };
  if (round(bufB) && round(bufA))
    while (round(bufB) && round(bufA)) {
    }
}

}  // namespace sldg
