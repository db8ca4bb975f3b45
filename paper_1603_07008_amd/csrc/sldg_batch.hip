// Batched sweeps (C ABI in include/sldg.h): many independent sLdG problems,
// each with its own grid, degree and displacement fields, advanced together.
// Every sweep of a split step (section II: Cheng-Knorr splitting into 1D
// advections) runs from one work list of tiles of all problems, sorted by
// class (tile kind and degree): one launch per class, of a kernel compiled
// for that class alone.  The split step can be captured once into a HIP graph
// and replayed; a tuner times launch shapes on the bound data and keeps the
// fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "sldg.h"
#include "sldg_internal.h"

using namespace sldg;

struct sldg_batch_s {
  int nprob = 0, ndim = 0;
  sldg_tier tier = SLDG_TIER_FP64;
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<int64_t> n;                 // [nprob * ndim]
  std::vector<int> k;
  std::vector<int64_t> cells, modes, hi_bytes;
  bool bound = false;
  std::vector<double*> mass[2];
  std::vector<void*> hi[2];
  // sequence
  int nseq = 0;
  std::vector<int> dims;
  std::vector<uint32_t> masks;            // [nseq * nprob]
  std::vector<int64_t> tab_off, ab_off, tab_n;   // [nseq * nprob]: s / matrix offsets, entries
  int32_t* d_s = nullptr;
  double* d_ab = nullptr;
  int32_t* d_pmap = nullptr;              // mode -> plane maps (FP64 cell mean only), per problem
  std::vector<int64_t> pmap_off;
  // launch shape per sweep of the sequence and work-list class, [q * kClasses + c]
  std::vector<int> rows, tuples;
  std::vector<double> tuned_ms;
  // device work description per sweep q: args for source buffer b at [q*2+b]
  std::vector<SweepArgs*> d_args;
  std::vector<BatchItem*> d_items;
  std::vector<int32_t> nitems;
  std::vector<int32_t> cls_off;           // [nseq * (kClasses + 1)] class offsets in the list
  bool ready = false;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
};

namespace {

// Work-list classes: kind (0 window, 1 group, 2 strided) x degree (1..3).
constexpr int kClasses = 9;
int class_of(int kind, int k) { return kind * 3 + (k - 1); }

// XCD run lengths of the class launches: twice those of the single-problem
// sweeps (measured on the batched Landau workload: 2.50 ms per step against
// 2.53 ms with 8 and 16).
constexpr int32_t kXcdContigDefault = 16, kXcdStridedDefault = 32;

// XCD group sizes of the work lists (SLDG_BATCH_XCD_CONTIG / _STRIDED
// override them, -1 .. 64).
static int32_t xcd_group(bool strided) {
  static const int32_t v[2] = {
      [] {
        const char* e = getenv("SLDG_BATCH_XCD_CONTIG");
        return e ? std::max(-1, std::min(64, atoi(e))) : kXcdContigDefault;
      }(),
      [] {
        const char* e = getenv("SLDG_BATCH_XCD_STRIDED");
        return e ? std::max(-1, std::min(64, atoi(e))) : kXcdStridedDefault;
      }()};
  return v[strided ? 1 : 0];
}

void drop_graphs(sldg_batch_s* b) {
  for (int i = 0; i < 2; ++i)
    if (b->graph[i]) {
      (void)hipGraphExecDestroy(b->graph[i]);
      b->graph[i] = nullptr;
    }
}

void free_work(sldg_batch_s* b) {
  for (auto* p : b->d_args) if (p) dev_free(p);
  for (auto* p : b->d_items) if (p) dev_free(p);
  b->d_args.clear();
  b->d_items.clear();
  b->nitems.clear();
  b->cls_off.clear();
  b->ready = false;
}

void free_batch(sldg_batch_s* b) {
  if (!b) return;
  drop_graphs(b);
  free_work(b);
  if (b->d_s) dev_free(b->d_s);
  if (b->d_ab) dev_free(b->d_ab);
  if (b->d_pmap) dev_free(b->d_pmap);
  delete b;
}

const int64_t* ext(const sldg_batch_s* b, int p) { return b->n.data() + (size_t)p * b->ndim; }

bool aligned16(const void* x) { return ((uintptr_t)x & 15) == 0; }

// Build the device argument blocks and work list of sweep q.
sldg_status build_sweep_impl(sldg_batch_s* b, int q) {
  const int dim = b->dims[q];
  std::vector<SweepArgs> args[2];
  std::vector<BatchItem> bucket[kClasses];
  for (int s = 0; s < 2; ++s) args[s].resize(b->nprob);
  for (int p = 0; p < b->nprob; ++p) {
    const int o = b->k[p] + 1;
    const uint32_t mask = b->masks[(size_t)q * b->nprob + p];
    // the problem's class: tile kind (window needs N_0 % 4 == 0 and aligned buffers) x degree
    int kind = 2;
    if (dim == 0) {
      bool window = ext(b, p)[0] % 4 == 0;
      for (int s = 0; s < 2; ++s)
        window = window && aligned16(b->mass[s][p]) && aligned16(b->hi[s][p]);
      kind = window ? 0 : 1;
    }
    const size_t sc = (size_t)q * kClasses + class_of(kind, b->k[p]);
    for (int src = 0; src < 2; ++src) {
      SweepArgs& a = args[src][p];
      a = SweepArgs{};
      int64_t ntab = 0;
      describe_grid(b->ndim, ext(b, p), o, b->modes[p], dim, mask, b->rows[sc], b->tuples[sc], a,
                    ntab);
      // the lane form (one cell per lane): rows 1 for the non-window
      // dimension-0 classes, rows 0 for strided classes (the launch picks the
      // kernel from the same rows)
      a.lane = ((kind == 1 && b->rows[sc] == 1) || (kind == 2 && b->rows[sc] == 0)) ? 1 : 0;
      a.in_lo = b->mass[src][p];
      a.in_hi = b->hi[src][p];
      a.out_lo = b->mass[1 - src][p];
      a.out_hi = b->hi[1 - src][p];
      a.pmap = b->d_pmap + b->pmap_off[p];
      a.n_lo = 1;                             // the cell mean in FP64, mode m at hi plane m-1
      a.s_tab = b->d_s + b->tab_off[(size_t)q * b->nprob + p];
      a.ab_tab = b->d_ab + b->ab_off[(size_t)q * b->nprob + p];
      a.ab_cs = ntab;
    }
    const SweepArgs& a = args[0][p];
    const int32_t nq = (a.nspec + a.tuples - 1) / a.tuples;
    if (dim == 0) {
      const int64_t groups = kind == 0 ? a.cells / 4
                             : a.lane ? a.cells
                                      : (int64_t)a.Q * ((a.N + 3) / 4);
      const int64_t tiles = (groups + 255) / 256;
      auto& bk = bucket[class_of(kind, b->k[p])];
      for (int32_t qg = 0; qg < nq; ++qg)
        for (int64_t x = 0; x < tiles; ++x) bk.push_back({p, kind, (int32_t)x, qg, 0});
    } else if (a.lane) {
      const int64_t tiles = (a.cells + 255) / 256;
      auto& bk = bucket[class_of(2, b->k[p])];
      for (int32_t qg = 0; qg < nq; ++qg)
        for (int64_t x = 0; x < tiles; ++x) bk.push_back({p, 2, (int32_t)x, qg, 0});
    } else {
      const int64_t xt = ((int64_t)a.P * a.Q + 63) / 64;
      const int64_t zt = ((int64_t)a.nchunk + 3) / 4;
      auto& bk = bucket[class_of(2, b->k[p])];
      // Memory order: the column blocks of a row chunk group first.  Rows of
      // N_x cells rarely start on a cache line, so neighbouring blocks share a
      // line in every row; with the blocks of a group next to each other (and
      // the next group N_x / 64 items later) those lines meet on one XCD.
      // Measured on the batched Landau workload: the v classes fetched
      // 1.21-1.32 x the state per launch with the row chunk groups of a
      // block together, 1.09-1.16 x in this order; the step went from 2.51
      // to 2.43 ms.
      for (int32_t qg = 0; qg < nq; ++qg)
        for (int64_t z = 0; z < zt; ++z)
          for (int64_t x = 0; x < xt; ++x) bk.push_back({p, 2, (int32_t)x, qg, (int32_t)z});
    }
  }
  std::vector<BatchItem> items;
  std::vector<int32_t> off(kClasses + 1, 0);
  for (int c = 0; c < kClasses; ++c) {
    off[c] = (int32_t)std::min<size_t>(items.size(), 0x7fffffff);
    items.insert(items.end(), bucket[c].begin(), bucket[c].end());
    if (bucket[c].size() > 0x7fffffff || items.size() > 0x7fffffff)
      return fail(SLDG_ERR_UNSUPPORTED, "work list too long");
  }
  off[kClasses] = (int32_t)items.size();
  b->cls_off.resize((size_t)b->nseq * (kClasses + 1));
  std::copy(off.begin(), off.end(), b->cls_off.begin() + (size_t)q * (kClasses + 1));
  for (int s = 0; s < 2; ++s) {
    SweepArgs*& d = b->d_args[(size_t)q * 2 + s];
    if (!d) {
      hipError_t e = dev_malloc(&d, sizeof(SweepArgs) * b->nprob);
      if (e != hipSuccess) return fail(SLDG_ERR_NOMEM, "batch arguments: %s", hipGetErrorString(e));
    }
    hipError_t e = hipMemcpy(d, args[s].data(), sizeof(SweepArgs) * b->nprob, hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_error(e, "batch arguments upload");
  }
  BatchItem*& di = b->d_items[q];
  if (di) {
    dev_free(di);
    di = nullptr;
  }
  if (!items.empty()) {
    hipError_t e = dev_malloc(&di, sizeof(BatchItem) * items.size());
    if (e != hipSuccess) return fail(SLDG_ERR_NOMEM, "batch work list: %s", hipGetErrorString(e));
    e = hipMemcpy(di, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_error(e, "batch work list upload");
  }
  b->nitems[q] = (int32_t)items.size();
  return SLDG_OK;
}

// A sweep whose work list could not be built leaves the batch not ready (run
// refuses) until the states or the sequence are set again.
sldg_status build_sweep(sldg_batch_s* b, int q) {
  const sldg_status st = build_sweep_impl(b, q);
  if (st != SLDG_OK) b->ready = false;
  return st;
}

sldg_status build_all(sldg_batch_s* b) {
  drop_graphs(b);
  b->ready = false;
  if (!b->bound || b->nseq == 0) return SLDG_OK;
  b->d_args.resize((size_t)b->nseq * 2, nullptr);
  b->d_items.resize(b->nseq, nullptr);
  b->nitems.resize(b->nseq, 0);
  for (int q = 0; q < b->nseq; ++q) {
    sldg_status st = build_sweep(b, q);
    if (st != SLDG_OK) return st;
  }
  b->ready = true;
  return SLDG_OK;
}

sldg_status launch(sldg_batch_s* b, int q, int src) {
  const int32_t* off = b->cls_off.data() + (size_t)q * (kClasses + 1);
  for (int c = 0; c < kClasses; ++c) {
    const int32_t n = off[c + 1] - off[c];
    if (n <= 0) continue;
    const int kind = c / 3, k = c % 3 + 1;
    hipError_t e = launch_batch_class((int)b->tier, k, kind, b->rows[(size_t)q * kClasses + c],
                                      b->d_args[(size_t)q * 2 + src], b->d_items[q] + off[c], n,
                                      xcd_group(kind == 2), b->stream);
    if (e != hipSuccess) return device_error(e, "batched sweep launch");
  }
  return SLDG_OK;
}

}  // namespace

extern "C" {

sldg_status sldg_batch_create(sldg_batch_t* out, int nprob, int ndim, const int64_t* ncells,
                              const int* k, sldg_tier tier, void* stream) {
  if (!out) return fail(SLDG_ERR_ARG, "batch out-pointer is NULL");
  *out = nullptr;
  if (nprob < 1) return fail(SLDG_ERR_ARG, "nprob %d < 1", nprob);
  if (ndim < 1 || ndim > kMaxDim) return fail(SLDG_ERR_ARG, "ndim %d not in [1, %d]", ndim, kMaxDim);
  if (!ncells || !k) return fail(SLDG_ERR_ARG, "null ncells or k");
  if ((int)tier < 0 || (int)tier > 3) return fail(SLDG_ERR_UNSUPPORTED, "tier %d unknown", (int)tier);
  sldg_batch_s* b = new (std::nothrow) sldg_batch_s();
  if (!b) return fail(SLDG_ERR_NOMEM, "host allocation failed");
  b->nprob = nprob;
  b->ndim = ndim;
  b->tier = tier;
  b->stream = static_cast<hipStream_t>(stream);
  b->n.assign(ncells, ncells + (size_t)nprob * ndim);
  b->k.assign(k, k + nprob);
  for (int p = 0; p < nprob; ++p) {
    if (b->k[p] < 1 || b->k[p] > 3) {
      free_batch(b);
      return fail(SLDG_ERR_UNSUPPORTED, "problem %d: degree %d not in [1, 3]", p, k[p]);
    }
    int64_t c = 1, m = 1;
    for (int e = 0; e < ndim; ++e) {
      const int64_t ne = b->n[(size_t)p * ndim + e];
      if (ne < 1) {
        free_batch(b);
        return fail(SLDG_ERR_ARG, "problem %d: ncells[%d] = %lld < 1", p, e, (long long)ne);
      }
      c *= ne;
      m *= b->k[p] + 1;
      if (c >= (1LL << 31)) {
        free_batch(b);
        return fail(SLDG_ERR_UNSUPPORTED, "problem %d: >= 2^31 cells", p);
      }
    }
    b->cells.push_back(c);
    b->modes.push_back(m);
    b->hi_bytes.push_back((m - 1) * c * elem_size(tier));
  }
  hipError_t e = hipGetDevice(&b->device);
  // mode -> plane maps: mode 0 in the FP64 array, mode m >= 1 at hi plane m-1
  std::vector<int32_t> pm;
  for (int p = 0; p < nprob; ++p) {
    b->pmap_off.push_back((int64_t)pm.size());
    pm.push_back(-1);
    for (int64_t m = 1; m < b->modes[p]; ++m) pm.push_back((int32_t)(m - 1));
  }
  if (e == hipSuccess) e = dev_malloc(&b->d_pmap, sizeof(int32_t) * pm.size());
  if (e == hipSuccess)
    e = hipMemcpy(b->d_pmap, pm.data(), sizeof(int32_t) * pm.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_batch(b);
    return e == hipErrorOutOfMemory ? fail(SLDG_ERR_NOMEM, "batch mode maps: %s", hipGetErrorString(e))
                                    : device_error(e, "batch create");
  }
  *out = b;
  return ok();
}

void sldg_batch_destroy(sldg_batch_t b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
}

sldg_status sldg_batch_bind(sldg_batch_t b, double* const* mass0, void* const* hi0,
                            double* const* mass1, void* const* hi1) {
  if (!b) return fail(SLDG_ERR_ARG, "batch is NULL");
  if (!mass0 || !hi0 || !mass1 || !hi1) return fail(SLDG_ERR_ARG, "null pointer array");
  for (int p = 0; p < b->nprob; ++p) {
    const void* bufs[4] = {mass0[p], hi0[p], mass1[p], hi1[p]};
    const int64_t sz[4] = {b->cells[p] * 8, b->hi_bytes[p], b->cells[p] * 8, b->hi_bytes[p]};
    for (int i = 0; i < 4; ++i)
      if (!bufs[i]) return fail(SLDG_ERR_ARG, "problem %d: null state pointer", p);
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (overlap(bufs[i], sz[i], bufs[j], sz[j]))
          return fail(SLDG_ERR_ALIAS, "problem %d: state buffers overlap", p);
  }
  for (int s = 0; s < 2; ++s) {
    b->mass[s].assign(s ? mass1 : mass0, (s ? mass1 : mass0) + b->nprob);
    b->hi[s].assign(s ? hi1 : hi0, (s ? hi1 : hi0) + b->nprob);
  }
  b->bound = true;
  sldg_status st = build_all(b);
  return st == SLDG_OK ? ok() : st;
}

sldg_status sldg_batch_set_sequence(sldg_batch_t b, int nseq, const int* dims,
                                    const uint32_t* masks, const double* const* shifts) {
  if (!b) return fail(SLDG_ERR_ARG, "batch is NULL");
  if (nseq < 1 || !dims || !masks || !shifts) return fail(SLDG_ERR_ARG, "bad sequence");
  for (int q = 0; q < nseq; ++q) {
    if (dims[q] < 0 || dims[q] >= b->ndim) return fail(SLDG_ERR_ARG, "sweep %d: dim %d", q, dims[q]);
    for (int p = 0; p < b->nprob; ++p) {
      const uint32_t m = masks[(size_t)q * b->nprob + p];
      if ((m >> b->ndim) || (m & (1u << dims[q])))
        return fail(SLDG_ERR_ARG, "sweep %d problem %d: bad dep_mask 0x%x", q, p, m);
      if (!shifts[(size_t)q * b->nprob + p])
        return fail(SLDG_ERR_ARG, "sweep %d problem %d: null shift", q, p);
    }
  }
  drop_graphs(b);
  free_work(b);
  if (b->d_s) dev_free(b->d_s);
  if (b->d_ab) dev_free(b->d_ab);
  b->d_s = nullptr;
  b->d_ab = nullptr;
  b->nseq = nseq;
  b->dims.assign(dims, dims + nseq);
  b->masks.assign(masks, masks + (size_t)nseq * b->nprob);
  b->tab_off.assign((size_t)nseq * b->nprob, 0);
  b->ab_off.assign((size_t)nseq * b->nprob, 0);
  b->tab_n.assign((size_t)nseq * b->nprob, 0);
  int64_t tot_s = 0, tot_ab = 0;
  for (int q = 0; q < nseq; ++q)
    for (int p = 0; p < b->nprob; ++p) {
      int64_t nt = 1;
      const uint32_t m = b->masks[(size_t)q * b->nprob + p];
      for (int e = 0; e < b->ndim; ++e)
        if (m & (1u << e)) nt *= ext(b, p)[e];
      const int o = b->k[p] + 1;
      const size_t i = (size_t)q * b->nprob + p;
      b->tab_off[i] = tot_s;
      b->ab_off[i] = tot_ab;
      b->tab_n[i] = nt;
      tot_s += nt;
      tot_ab += nt * 2 * o * o;
    }
  // on failure the batch keeps no sequence (and so cannot run on missing tables)
  auto drop_sequence = [&](sldg_status st) {
    if (b->d_s) dev_free(b->d_s);
    if (b->d_ab) dev_free(b->d_ab);
    b->d_s = nullptr;
    b->d_ab = nullptr;
    b->nseq = 0;
    return st;
  };
  hipError_t e = dev_malloc(&b->d_s, sizeof(int32_t) * std::max<int64_t>(1, tot_s));
  if (e == hipSuccess) e = dev_malloc(&b->d_ab, sizeof(double) * std::max<int64_t>(1, tot_ab));
  if (e != hipSuccess)
    return drop_sequence(fail(SLDG_ERR_NOMEM, "batch tables: %s", hipGetErrorString(e)));
  for (int q = 0; q < nseq; ++q)
    for (int p = 0; p < b->nprob; ++p) {
      const size_t i = (size_t)q * b->nprob + p;
      e = launch_line_tables(b->k[p], b->tab_n[i], ext(b, p)[dims[q]], shifts[i],
                             b->d_s + b->tab_off[i], b->d_ab + b->ab_off[i], true, false,
                             b->stream);
      if (e != hipSuccess) return drop_sequence(device_error(e, "batch line tables"));
    }
  b->rows.assign((size_t)nseq * kClasses, 4);
  b->tuples.assign((size_t)nseq * kClasses, 9);
  b->tuned_ms.assign((size_t)nseq * kClasses, -1.0);
  sldg_status st = build_all(b);
  return st == SLDG_OK ? ok() : st;
}

sldg_status sldg_batch_run(sldg_batch_t b, int nsteps, int use_graph, int* result_buffer) {
  if (!b) return fail(SLDG_ERR_ARG, "batch is NULL");
  if (!b->ready) return fail(SLDG_ERR_ARG, "bind the states and set the sequence first");
  if (nsteps < 0) return fail(SLDG_ERR_ARG, "nsteps %d < 0", nsteps);
  int cur = 0;
  if (use_graph) {
    if (!b->stream) return fail(SLDG_ERR_ARG, "graph replay needs a non-null stream");
    for (int n = 0; n < nsteps; ++n) {
      if (!b->graph[cur]) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return device_error(e, "hipStreamBeginCapture");
        int c = cur;
        sldg_status st = SLDG_OK;
        for (int q = 0; q < b->nseq && st == SLDG_OK; ++q) {
          st = launch(b, q, c);
          c = 1 - c;
        }
        e = hipStreamEndCapture(b->stream, &g);
        if (st != SLDG_OK) {
          if (g) (void)hipGraphDestroy(g);
          return st;
        }
        if (e != hipSuccess) return device_error(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&b->graph[cur], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return device_error(e, "hipGraphInstantiate");
      }
      hipError_t e = hipGraphLaunch(b->graph[cur], b->stream);
      if (e != hipSuccess) return device_error(e, "hipGraphLaunch");
      if (b->nseq % 2) cur = 1 - cur;
    }
  } else {
    for (int n = 0; n < nsteps; ++n)
      for (int q = 0; q < b->nseq; ++q) {
        sldg_status st = launch(b, q, cur);
        if (st != SLDG_OK) return st;
        cur = 1 - cur;
      }
  }
  if (result_buffer) *result_buffer = cur;
  return ok();
}

sldg_status sldg_batch_set_tuning(sldg_batch_t b, int q, int rows, int tuples) {
  if (!b) return fail(SLDG_ERR_ARG, "batch is NULL");
  if (q < 0 || q >= b->nseq) return fail(SLDG_ERR_ARG, "sweep %d out of range", q);
  if (!(rows == 2 || rows == 4 || rows == 8 || (rows == 1 && b->dims[q] == 0) ||
        (rows == 0 && b->dims[q] > 0)) ||
      tuples < 0)
    return fail(SLDG_ERR_ARG,
                "rows %d not in {2, 4, 8} (or 1 along dimension 0, 0 along others) or tuples %d < 0",
                rows, tuples);
  for (int c = 0; c < kClasses; ++c) {
    b->rows[(size_t)q * kClasses + c] = rows;
    b->tuples[(size_t)q * kClasses + c] = tuples;
    b->tuned_ms[(size_t)q * kClasses + c] = -1.0;
  }
  if (b->bound) {
    drop_graphs(b);
    sldg_status st = build_sweep(b, q);
    if (st != SLDG_OK) return st;
  }
  return ok();
}

sldg_status sldg_batch_set_class_tuning(sldg_batch_t b, int q, int cls, int rows, int tuples) {
  if (!b) return fail(SLDG_ERR_ARG, "batch is NULL");
  if (q < 0 || q >= b->nseq) return fail(SLDG_ERR_ARG, "sweep %d out of range", q);
  if (cls < 0 || cls >= kClasses) return fail(SLDG_ERR_ARG, "class %d out of range", cls);
  if (!(rows == 2 || rows == 4 || rows == 8 || (rows == 1 && cls / 3 != 2) ||
        (rows == 0 && cls / 3 == 2)) ||
      tuples < 0)
    return fail(SLDG_ERR_ARG,
                "rows %d not in {2, 4, 8} (or 1 for classes 0-5, 0 for 6-8) or tuples %d < 0", rows,
                tuples);
  const size_t i = (size_t)q * kClasses + cls;
  b->rows[i] = rows;
  b->tuples[i] = tuples;
  b->tuned_ms[i] = -1.0;
  if (b->bound) {
    drop_graphs(b);
    sldg_status st = build_sweep(b, q);
    if (st != SLDG_OK) return st;
  }
  return ok();
}

sldg_status sldg_batch_get_class_tuning(sldg_batch_t b, int q, int cls, int* rows, int* tuples,
                                        double* ms, int* nitems) {
  if (!b) return fail(SLDG_ERR_ARG, "batch is NULL");
  if (q < 0 || q >= b->nseq) return fail(SLDG_ERR_ARG, "sweep %d out of range", q);
  if (cls < 0 || cls >= kClasses) return fail(SLDG_ERR_ARG, "class %d out of range", cls);
  const size_t i = (size_t)q * kClasses + cls;
  if (rows) *rows = b->rows[i];
  if (tuples) *tuples = b->tuples[i];
  if (ms) *ms = b->tuned_ms[i];
  if (nitems) {
    *nitems = 0;
    if (b->ready && b->cls_off.size() >= (size_t)(q + 1) * (kClasses + 1)) {
      const int32_t* off = b->cls_off.data() + (size_t)q * (kClasses + 1);
      *nitems = off[cls + 1] - off[cls];
    }
  }
  return ok();
}

sldg_status sldg_batch_get_tuning(sldg_batch_t b, int q, int* rows, int* tuples, double* ms) {
  if (!b) return fail(SLDG_ERR_ARG, "batch is NULL");
  if (q < 0 || q >= b->nseq) return fail(SLDG_ERR_ARG, "sweep %d out of range", q);
  // the shape of the class with the most tiles, and the tuned time of the whole sweep
  int best = 0;
  int32_t most = -1;
  double tot = 0.0;
  bool tuned = true;
  for (int c = 0; c < kClasses; ++c) {
    int n = 0;
    (void)sldg_batch_get_class_tuning(b, q, c, nullptr, nullptr, nullptr, &n);
    if (n > most) {
      most = n;
      best = c;
    }
    const double t = b->tuned_ms[(size_t)q * kClasses + c];
    if (n > 0) {
      if (t < 0) tuned = false;
      else tot += t;
    }
  }
  if (rows) *rows = b->rows[(size_t)q * kClasses + best];
  if (tuples) *tuples = b->tuples[(size_t)q * kClasses + best];
  if (ms) *ms = tuned ? tot : -1.0;
  return ok();
}

sldg_status sldg_batch_tune(sldg_batch_t b, int reps) {
  if (!b) return fail(SLDG_ERR_ARG, "batch is NULL");
  if (!b->ready) return fail(SLDG_ERR_ARG, "bind the states and set the sequence first");
  if (reps < 1) reps = 1;
  hipEvent_t ev[kClasses + 1];
  int nev = 0;
  hipError_t e = hipSuccess;
  for (; nev < kClasses + 1 && e == hipSuccess; ++nev) e = hipEventCreate(&ev[nev]);
  if (e != hipSuccess) {
    for (int i = 0; i < nev - 1; ++i) (void)hipEventDestroy(ev[i]);
    return device_error(e, "hipEventCreate");
  }
  const int rows_c[4] = {2, 4, 8, 0};          // strided: rows per thread, or the lane form
  const int rows_c0[2] = {4, 1};              // dimension 0: group, lane form
  const int tup_c[4] = {1, 3, 9, 0};
  sldg_status st = SLDG_OK;
  for (int q = 0; q < b->nseq && st == SLDG_OK; ++q) {
    int best_r[kClasses], best_t[kClasses];
    double best[kClasses];
    for (int c = 0; c < kClasses; ++c) {
      best_r[c] = b->rows[(size_t)q * kClasses + c];
      best_t[c] = b->tuples[(size_t)q * kClasses + c];
      best[c] = 1e300;
    }
    const int nr = b->dims[q] == 0 ? 2 : 4;
    for (int ir = 0; ir < nr && st == SLDG_OK; ++ir)
      for (int it = 0; it < 4 && st == SLDG_OK; ++it) {
        // every class of the sweep takes the candidate; each class is timed alone
        for (int c = 0; c < kClasses; ++c) {
          b->rows[(size_t)q * kClasses + c] = b->dims[q] == 0 ? rows_c0[ir] : rows_c[ir];
          b->tuples[(size_t)q * kClasses + c] = tup_c[it];
        }
        st = build_sweep(b, q);
        if (st != SLDG_OK) break;
        st = launch(b, q, 0);                 // warm-up
        const int32_t* off = b->cls_off.data() + (size_t)q * (kClasses + 1);
        for (int c = 0; c < kClasses && st == SLDG_OK; ++c) {
          const int32_t n = off[c + 1] - off[c];
          (void)hipEventRecord(ev[c], b->stream);
          for (int r = 0; r < reps && n > 0 && st == SLDG_OK; ++r) {
            e = launch_batch_class((int)b->tier, c % 3 + 1, c / 3,
                                   b->rows[(size_t)q * kClasses + c],
                                   b->d_args[(size_t)q * 2], b->d_items[q] + off[c], n,
                                   xcd_group(c / 3 == 2), b->stream);
            if (e != hipSuccess) st = device_error(e, "tuning launch");
          }
        }
        (void)hipEventRecord(ev[kClasses], b->stream);
        e = hipEventSynchronize(ev[kClasses]);
        if (st == SLDG_OK && e != hipSuccess) st = device_error(e, "tuning");
        for (int c = 0; c < kClasses && st == SLDG_OK; ++c) {
          if (off[c + 1] == off[c]) continue;
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, ev[c], ev[c + 1]);
          if (ms / reps < best[c]) {
            best[c] = ms / reps;
            best_r[c] = b->rows[(size_t)q * kClasses + c];
            best_t[c] = b->tuples[(size_t)q * kClasses + c];
          }
        }
      }
    for (int c = 0; c < kClasses; ++c) {
      b->rows[(size_t)q * kClasses + c] = best_r[c];
      b->tuples[(size_t)q * kClasses + c] = best_t[c];
      b->tuned_ms[(size_t)q * kClasses + c] = best[c] < 1e299 ? best[c] : -1.0;
    }
    if (st == SLDG_OK) st = build_sweep(b, q);
  }
  for (int i = 0; i < kClasses + 1; ++i) (void)hipEventDestroy(ev[i]);
  drop_graphs(b);
  return st == SLDG_OK ? ok() : st;
}

}  // extern "C"
