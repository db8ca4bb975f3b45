// Internal interface between the host library and the HIP kernels of libsldg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sldg.h"

namespace sldg {

constexpr int kMaxDim = 6;

// Division by a runtime-invariant divisor d >= 1 by multiply and shift
// (T. Granlund, P. Montgomery, "Division by invariant integers using
// multiplication", 1994): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, floor(n / d) = (mulhi(n, m) + n) >> l for
// every 0 <= n < 2^31.
struct FastDiv {
  uint32_t d, m, l;
  static FastDiv make(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    f.l = l;
    f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    return f;
  }
  __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return ((uint32_t)(((uint64_t)n * m) >> 32) + n) >> l;   // mulhi: v_mul_hi_u32
  }
  __host__ __device__ __forceinline__ uint32_t mod(uint32_t n) const { return n - div(n) * d; }
};

// Maps a line (a fixed transverse cell) to its entry in the per-line table.
// The table is indexed over the dimensions the displacement depends on,
// lowest dimension fastest.  A line is identified by two flattened indices:
// `lo` over the dimensions below the swept one and `hi` over those above it.
// Entry = sum over dependent dims e of ((idx / div_e) % mod_e) * str_e, where
// idx is lo or hi depending on the side of e.
struct LineMap {
  int nlo, nhi;
  FastDiv lo_div[kMaxDim], lo_mod[kMaxDim];
  int32_t lo_str[kMaxDim];
  FastDiv hi_div[kMaxDim], hi_mod[kMaxDim];
  int32_t hi_str[kMaxDim];
};

struct SweepArgs {
  const double* in_lo;    // FP64 modes (mode-major planes, increasing mode id)
  const void* in_hi;      // the other modes, in the tier's storage type
  double* out_lo;
  void* out_hi;
  const int32_t* pmap;    // per mode id: >= 0 plane in hi, < 0 plane -1-v in lo
  int32_t n_lo;           // planes in lo (kernels without extra FP64 modes: 0 or 1)
  int32_t wide_fp64;      // 1: more than the cell mean may be FP64 (general kernels)
  const int32_t* s_tab;   // per table entry: s mod N, in [0, N)
  const double* ab_tab;   // per table entry t: A then B, (k+1)^2 each, row-major,
                          // component e of entry t at ab_tab[e * ab_cs + t]
  int64_t ab_cs;          // component stride of the table (= its entry count)
  int64_t cells;          // cells of the grid (plane length)
  int32_t P;              // product of the extents below the swept dim (row stride)
  int32_t N;              // extent of the swept dim
  int32_t Q;              // product of the extents above the swept dim
  int32_t mstride;        // (k+1)^dim: mode-id distance between j_dim and j_dim+1
  int32_t nspec;          // (k+1)^(ndim-1) spectator mode tuples
  int32_t nchunk;         // strided sweep: chunks along the swept dim
  int32_t chunk;          // strided sweep: rows per thread (1, 2, 4 or 8)
  int32_t tuples;         // spectator tuples per thread (a run; blockIdx.y picks it)
  int32_t colwaves;       // strided sweep: waves of a workgroup side by side (1, 2 or 4)
  int32_t lane;           // dimension-0 sweep without the window form: 1 lane form, 0 group form
  int32_t ntmask;         // one-value-per-lane stores with the non-temporal hint: bits 0, 1, 2
                          // for 2-, 4-, 8-byte values (set where a wave writes whole lines)
  FastDiv fP;             // division by P
  FastDiv fN;             // division by N
  FastDiv fchunk;         // division by nchunk
  FastDiv fG;             // division by ceil(N / 4) (dimension-0 group form)
  LineMap map;
  int32_t xcd;            // XCD-aware tile order: run length G (0 off, -1 one range per XCD)
  int32_t nblk;           // strided sweep: column blocks per slab (P / columns per tile) for
                          // tiles in memory order, 0 for row chunk groups fastest
  // FP16 storage with per-plane power-of-two scaling (all null: unscaled)
  const int32_t* in_exp;  // [n_hi] storage exponent of every input hi plane
  const int32_t* out_exp; // [n_hi] exponent every output hi plane is written with
  float* amax_part;       // [n_hi][nslot] per-wave absmax of the outputs (before scaling)
  int32_t nslot;          // partial slots per plane of the launch (sweep_slots)
  int32_t stage;          // strided sweep: 1 stages the tile's sources through LDS
                          // (sldg_staged.h; the host sets it where staged_fits)
};

// Shape of a staged strided tile (sldg_staged.h) for degree k, storage size
// sz bytes, rows per thread L and column waves cw: 16-byte load slots per
// thread (the tile without shift spread, plus one for the 16-bit tiers; the
// single-row-chunk tiles, cw = 4, take enough for a spread of two rows),
// tile rows per plane they cover, and the LDS bytes of its two buffers.
constexpr int staged_slots(int k, int sz, int L, int cw) {
  const int ch = 64 * cw / (16 / sz), rt = (4 / cw) * L;
  const int base = ((k + 1) * (rt + 1) * ch + 255) / 256 + (sz == 2 ? 1 : 0);
  const int two = ((k + 1) * (rt + 3) * ch + 255) / 256;
  return cw == 4 && two > base ? two : base;
}
constexpr int staged_umax(int k, int sz, int L, int cw) {
  return staged_slots(k, sz, L, cw) * 256 / ((k + 1) * (64 * cw / (16 / sz)));
}
constexpr int64_t staged_lds_bytes(int k, int sz, int L, int cw) {
  return 2LL * (k + 1) * staged_umax(k, sz, L, cw) * (64 * cw) * sz;
}
constexpr int64_t kStagedLdsMax = 64 * 1024;

// One workgroup-sized tile of one problem of a batched sweep.
//   kind 0: dimension-0 sweep, window form: groups [x*256, x*256+256) of 4 cells
//   kind 1: dimension-0 sweep, group form: groups [x*256, x*256+256), or in the
//           lane form (class rows 1) cells [x*256, x*256+256)
//   kind 2: strided sweep: columns [64x, 64x+64), row chunks from z*(blockDim/64),
//           or in the lane form (class rows 0) cells [x*256, x*256+256)
// qg selects the run of spectator tuples.
struct BatchItem {
  int32_t prob, kind, x, qg, z;
};

// The line tables of up to kMaxTableSet sweeps computed in one launch
// (forward tables, component-major): sweep q has first[q + 1] - first[q]
// entries, period[q] cells along its dimension and displacements sigma[q].
constexpr int kMaxTableSet = 16;
struct TableSet {
  int32_t count;
  int64_t first[kMaxTableSet + 1];
  int64_t period[kMaxTableSet];
  const double* sigma[kMaxTableSet];
};

// Launchers (defined in sldg_kernels.hip).  All return hipGetLastError().
hipError_t launch_line_tables(int k, int64_t n, int64_t period, const double* sigma,
                              int32_t* s_out, double* ab_out, bool component_major,
                              bool adjoint, hipStream_t st);
hipError_t launch_line_tables_set(int k, const TableSet& set, int32_t* s_out, double* ab_out,
                                  hipStream_t st);
hipError_t launch_sweep(int k, int tier, int dim, const SweepArgs& a, hipStream_t st);
hipError_t launch_mass(const double* mass, int64_t n, double* partial, int nblocks,
                       double* result, hipStream_t st);

// One class (tile kind, degree k) of a batched sweep: nitems workgroups, one
// per item of `items` (kinds as in BatchItem; rows: 2, 4 or 8 for kind 2).
hipError_t launch_batch_class(int tier, int k, int kind, int rows, const SweepArgs* args,
                              const BatchItem* items, int32_t nitems, int32_t xcd,
                              hipStream_t st);
bool contig_window_ok(const SweepArgs& a);

// The launchers of one (degree K, storage tier) pair, explicitly
// instantiated in sldg_sweep_inst.hip (compiled once per pair); launch_sweep
// and launch_batch_class dispatch to them.
template <int K, int TIER>
hipError_t launch_sweep_inst(int dim, const SweepArgs& a, hipStream_t st);
template <int K, int TIER>
hipError_t launch_class_inst(int kind, int rows, const SweepArgs* args, const BatchItem* items,
                             int32_t nitems, int32_t xcd, hipStream_t st);
// The fused pair of sweeps along dimensions 0 and 1 (sldg_fused.h):
// nblocks workgroups of 256 threads with lds_bytes of dynamic LDS.
struct XYArgs;
hipError_t launch_xy(int k, int tier, const XYArgs& a, int64_t lds_bytes, int32_t nblocks,
                     hipStream_t st);
template <int K, int TIER>
hipError_t launch_xy_inst(const XYArgs& a, int64_t lds_bytes, int32_t nblocks, hipStream_t st);
// Waves of one sweep launch that compute a given output plane (the absmax
// partial slots per plane of a scaled FP16 sweep).
int64_t sweep_slots(int dim, const SweepArgs& a);
// Kernel form of a sweep launch: 0 dimension-0 window, 1 group, 2 strided,
// 3 lane, 4 strided staged through LDS; -1 if the grid does not launch.
int sweep_form(int dim, const SweepArgs& a);

// Scaled FP16 storage (sldg_kernels.hip).  A scale block holds int32 exp[n_hi]
// followed by float amax[n_hi].
//   predict: out exp from the input's absmax (or the input exp when that is
//            0) with `headroom` binades; zeroes the partials and the count of
//            planes to redo.
//   decide:  out amax = max of the partials; a plane whose absmax reaches
//            2^15 at its predicted exponent gets the exponent of its absmax
//            with one binade of headroom, is flagged in redo[] and counted.
//   redo:    recomputes the flagged planes with their final exponents.
hipError_t launch_scale_predict(int64_t n_hi, const int32_t* in_exp, const float* in_amax,
                                int32_t* out_exp, int headroom, float* part, int64_t npart,
                                int32_t* nredo, hipStream_t st);
hipError_t launch_scale_decide(int64_t n_hi, const float* part, int32_t nslot, int32_t* out_exp,
                               float* out_amax, int32_t* redo, int32_t* nredo, hipStream_t st);
hipError_t launch_scale_redo(int k, int dim, const SweepArgs& a, int64_t n_hi,
                             const int32_t* redo, const int32_t* nredo, const int32_t* hi_mode,
                             hipStream_t st);
// import: absmax and exponent of every plane of an FP64 array [n_hi][cells],
// then the scaled RNE conversion to FP16.  export: the values the FP16 planes
// represent, in FP64.
hipError_t launch_scale_import(const double* src, int64_t n_hi, int64_t cells, int headroom,
                               float* part, int32_t nslot, void* dst, int32_t* exp, float* amax,
                               hipStream_t st);
hipError_t launch_scale_export(const void* src, int64_t n_hi, int64_t cells, const int32_t* exp,
                               double* dst, hipStream_t st);
constexpr int kImportSlots = 256;
hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t st);

int mass_blocks(int64_t n);

// Device memory of the library's own buffers (plan tables, scratch, batch work
// lists): every allocation goes through dev_malloc / dev_free, which count the
// live bytes and honour the process-wide limit of sldg_set_device_alloc_limit
// (an allocation that would pass it fails with hipErrorOutOfMemory, without
// calling hipMalloc).  dev_alloc_fits tells whether `bytes` more would fit.
hipError_t dev_malloc_raw(void** p, size_t bytes);
template <class T>
hipError_t dev_malloc(T** p, size_t bytes) {
  void* v = nullptr;
  const hipError_t e = dev_malloc_raw(&v, bytes);
  *p = static_cast<T*>(v);
  return e;
}
void dev_free(void* p);
bool dev_alloc_fits(int64_t bytes);

// Host helpers shared by the plan and batch front ends (sldg_host.hip).
sldg_status fail(sldg_status st, const char* fmt, ...);
sldg_status ok();
const char* last_error_text();
int64_t elem_size(sldg_tier t);
bool overlap(const void* a, int64_t na, const void* b, int64_t nb);
sldg_status device_error(hipError_t e, const char* what);
// Everything a sweep kernel needs to know about one grid except the buffers
// and tables; ntab = entries of the sweep's per-line table.
void describe_grid(int ndim, const int64_t* n, int o, int64_t modes, int dim, uint32_t dep_mask,
                   int rows_per_thread, int tuples_per_thread, SweepArgs& a, int64_t& ntab);

}  // namespace sldg
