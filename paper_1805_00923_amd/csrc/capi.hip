// C ABI: argument checks, graph ownership, schedules and the host side of
// each algorithm.  Everything here is host code; the per-step work runs in
// the kernels of bfs_cc.hip, pagerank.hip, sssp.hip and frontier.hip.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.h"

using namespace gi;

// ---------------------------------------------------------------- errors --

static thread_local std::string g_err;

static gi_status fail(gi_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static gi_status fail(gi_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(GI_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

#define LAUNCH_TRY(call)                                                               \
  do {                                                                                 \
    if ((call) != 0) {                                                                 \
      hipError_t e_ = hipGetLastError();                                               \
      return fail(GI_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));       \
    }                                                                                  \
  } while (0)

extern "C" const char* gi_last_error(void) { return g_err.c_str(); }
extern "C" int32_t gi_abi_version(void) { return GI_ABI_VERSION; }

// ------------------------------------------------------- device memory --
//
// Every device allocation of the library goes through dmem_alloc and every
// release through dmem_free.  Sources, in order: the graph's workspace, when
// the caller gave one to gi_graph_create_ex (bump-allocated in 256-byte
// steps, released with the graph); the allocator registered with
// gi_set_allocator (the Python binding registers torch's caching allocator);
// hipMalloc.  The source of each live allocation is recorded, so a release
// goes back where the memory came from even if the registered allocator
// changed meanwhile.

namespace {

struct Provider {
  gi_alloc_fn alloc = nullptr;
  gi_free_fn release = nullptr;
  void* ctx = nullptr;
};

struct LiveAlloc {
  Provider from;
  int device;
};

std::mutex g_dmem_mu;
Provider g_provider;
std::unordered_map<void*, LiveAlloc> g_dmem_live;

// A caller-given region for a graph's core arrays.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
};

constexpr size_t kArenaAlign = 256;

size_t arena_round(size_t bytes) {
  return (std::max<size_t>(1, bytes) + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
}

}  // namespace

static void* dmem_alloc(size_t bytes, Arena* arena) {
  bytes = std::max<size_t>(1, bytes);
  if (arena && arena->base) {
    if (arena->used + arena_round(bytes) <= arena->size) {
      void* p = arena->base + arena->used;
      arena->used += arena_round(bytes);
      return p;
    }
    return nullptr;  // the workspace was sized for exactly these arrays
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  Provider pv;
  {
    std::lock_guard<std::mutex> lock(g_dmem_mu);
    pv = g_provider;
  }
  void* p = nullptr;
  if (pv.alloc) {
    p = pv.alloc(bytes, dev, pv.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) {
    std::lock_guard<std::mutex> lock(g_dmem_mu);
    g_dmem_live[p] = LiveAlloc{pv, dev};
  }
  return p;
}

// Memory from a graph's workspace is not recorded and is left alone here.
static void dmem_free(void* p) {
  if (!p) return;
  LiveAlloc la;
  {
    std::lock_guard<std::mutex> lock(g_dmem_mu);
    auto it = g_dmem_live.find(p);
    if (it == g_dmem_live.end()) return;
    la = it->second;
    g_dmem_live.erase(it);
  }
  if (la.from.release) la.from.release(p, la.device, la.from.ctx);
  else (void)hipFree(p);
}

template <typename T>
static bool dmem_alloc_n(T** p, size_t count) {
  *p = static_cast<T*>(dmem_alloc(count * sizeof(T), nullptr));
  return *p != nullptr;
}

// hipMalloc-shaped: hipSuccess, or hipErrorOutOfMemory with *p = NULL.
static hipError_t dmem_get(void** p, size_t bytes) {
  *p = dmem_alloc(bytes, nullptr);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

extern "C" gi_status gi_set_allocator(gi_alloc_fn alloc, gi_free_fn release, void* ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(GI_ERR_INVALID_ARG, "give both allocator functions or neither");
  std::lock_guard<std::mutex> lock(g_dmem_mu);
  g_provider = Provider{alloc, release, ctx};
  return GI_OK;
}

extern "C" gi_status gi_live_allocations(int64_t* count, int64_t* from_registered) {
  if (!count) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lock(g_dmem_mu);
  int64_t r = 0;
  for (const auto& kv : g_dmem_live) r += kv.second.from.alloc != nullptr;
  *count = (int64_t)g_dmem_live.size();
  if (from_registered) *from_registered = r;
  return GI_OK;
}

// ------------------------------------------------------------ the graph --

namespace {

struct SegDev {
  int32_t* off = nullptr;
  int32_t* idx = nullptr;
  int32_t* dst = nullptr;
  int4* table = nullptr;
  int ntab = 0;
  int nrows = 0;
  int64_t nnz = 0;
};

}  // namespace

struct gi_graph {
  int32_t n = 0;
  int64_t m = 0;
  Arena arena;               // caller-given workspace for the core arrays (may be empty)
  int stats_pending = 0;     // launches of an enqueued run whose times are not read yet
  hipStream_t last_stream = nullptr;
  int32_t max_out = 0, max_in = 0;
  bool weighted = false;
  int device = 0;
  std::vector<void*> allocs;       // graph-lifetime device allocations
  std::vector<void*> sched_allocs; // schedule-lifetime device allocations
  std::vector<void*> seg_allocs;   // PageRank segments (built on first segmented use)
  int seg_p = 0, seg_strategy = -1, seg_cap = 0;
  std::vector<void*> ccseg_allocs; // CC pull segments (built on first segmented use)
  int ccseg_p = 0, ccseg_strategy = -1;
  CcSeg* ccsegs = nullptr;
  uint32_t* cc_segmin = nullptr;
  // adjacency on the device
  int32_t *out_off = nullptr, *out_idx = nullptr, *in_off = nullptr, *in_idx = nullptr;
  int32_t *outdeg = nullptr, *udeg = nullptr;
  int32_t* in_probe = nullptr;  // in-neighbour of largest out-degree (BFS pull's first test)
  int32_t* hubs = nullptr;      // vertices with more than kHubDeg out-edges
  int nhubs = 0;
  uint32_t *out_w = nullptr, *in_w = nullptr;
  // host copies of the offsets (destination blocks and segments are built from them)
  std::vector<int32_t> h_in_off, h_in_idx, h_out_off, h_outdeg;
  gi_schedule sched{};
  // destination blocks of the in-rows (PageRank, CC pull pass 0) and out-rows
  int4* pr_table = nullptr;
  int pr_ntab = 0, pr_cap_e = 0, pr_cap_v = 0, pr_nlong = 0;
  double* lr_acc = nullptr;
  unsigned* lr_cnt = nullptr;
  int32_t* lr_chunks = nullptr;
  // symmetric adjacency and its destination blocks (CC; built on first use)
  int32_t* sym_off = nullptr;
  int32_t* sym_idx = nullptr;
  int4* sym_table = nullptr;
  int sym_ntab = 0;
  // CC over the CSR and CSC rows directly: their destination blocks
  int4* ccd_out_table = nullptr;
  int4* ccd_in_table = nullptr;
  int ccd_out_ntab = 0, ccd_in_ntab = 0;
  std::vector<SegDev> segs;
  // degree-ordered in-adjacency and its merge-path tiles (PageRank with
  // vertex_order = GI_ORDER_OUT_DEGREE; built on first use)
  // in-rows by decreasing source out-degree, ties by id (the BFS pull's scan
  // order: a row starts with its probe; built on first use)
  std::vector<void*> bfsr_allocs;
  int32_t* bfs_idx = nullptr;
  std::vector<void*> ord_allocs;  // the ordered copy (graph lifetime once built)
  std::vector<void*> ordt_allocs; // tiles and split slots (rebuilt when the tile size changes)
  int32_t *ord_off = nullptr, *ord_idx = nullptr, *ord_outdeg = nullptr, *ord_old = nullptr;
  std::vector<int32_t> h_ord_off;
  int32_t ord_nsrc = 0;            // vertices with out-degree > 0 (new ids [0, ord_nsrc))
  int2 *ord_tiles = nullptr, *ord_tslot = nullptr;
  int32_t* ord_srow = nullptr;
  double* ord_sacc = nullptr;
  int ord_ntiles = 0, ord_T = 0, ord_nslots = 0;
  int ncu = 0;                     // compute units of the device
  double* pr_acc = nullptr;
  PrRows* seg_rows = nullptr;  // device copy of the segments' row blocks
  // frontier-loop workspace
  uint64_t* fbv[2] = {nullptr, nullptr};  // dense frontiers (bitvectors)
  uint8_t* fbm[2] = {nullptr, nullptr};   // dense frontiers (bool maps, padded to 64)
  uint64_t* vis = nullptr;                // BFS visited
  uint64_t* far = nullptr;                // SSSP far set
  int32_t* lab = nullptr;                 // CC second label buffer
  float* contrib[2] = {nullptr, nullptr};
  Part* part = nullptr;
  Blk* blk = nullptr;
  unsigned long long* fmin = nullptr;
  int32_t* ids = nullptr;
  long long* excl = nullptr;
  int32_t* chunk_item = nullptr;
  Control* ctl = nullptr;
  HostFlags* hflags = nullptr; // pinned, written by the decide kernels
  HostFlags* dflags = nullptr; // device address of hflags
  Engine eng{};
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t evb[2] = {nullptr, nullptr};  // batch completion events
  // the degree-ordered PageRank run as a HIP graph, replayed when a call
  // repeats the previous call's arguments (its own stream, ordered after
  // the caller's by an event)
  struct PrGraphKey {
    float* ranks = nullptr;
    int iters = -1;
    float damping = 0.0f;
    int bt = 0, u = 0, hot = 0, grid = 0, ntiles = 0, nslots = 0;
    const void* tiles = nullptr;
    const void* idx = nullptr;
    bool operator==(const PrGraphKey& o) const {
      return ranks == o.ranks && iters == o.iters && damping == o.damping && bt == o.bt &&
             u == o.u && hot == o.hot && grid == o.grid && ntiles == o.ntiles &&
             nslots == o.nslots && tiles == o.tiles && idx == o.idx;
    }
  } prg_key;
  hipStream_t prg_stream = nullptr;
  hipEvent_t prg_evw = nullptr;
  hipGraph_t prg_graph = nullptr;
  hipGraphExec_t prg_exec = nullptr;
  gi_run_stats stats{};
  // per-step timing (optional)
  int step_timing = 0;
  bool timing_failed = false;
  std::vector<StepEvents> tev;
  int tev_count = 0;        // steps of the last run that carry events
  int last_steps[6] = {0, 0, 0, 0, 0, 0};  // steps of the previous run, per algorithm
  void* bc = nullptr;  // betweenness scratch: sigma, fs, bw, bounds, level, order
  int4* bc_tab = nullptr;  // in-row blocks for the betweenness pull levels
  int bc_ntab = 0;
  int4* prec_tab = nullptr;  // in-row blocks for PageRank + eigenvector
  int prec_ntab = 0;
  int32_t* prec_lrow = nullptr;  // long rows (chunked) and their FP64 sum slots
  double* prec_lacc = nullptr;
  int prec_nlong = 0;
  float2* prec_aos = nullptr;  // 2 n pairs
  float* prec_y = nullptr;     // 2 n
  // the fused pass over the degree-ordered in-adjacency: its blocks, long
  // rows and sum slots, and the results before they return to caller ids
  // (2 n floats); built on first use, freed with the ordered copy
  int4* preco_tab = nullptr;
  int preco_ntab = 0;
  int32_t* preco_lrow = nullptr;
  double* preco_lacc = nullptr;
  int preco_nlong = 0;
  float* preco_tmp = nullptr;
  double* prec_norm = nullptr;
  int prec_norm_cap = 0;
  double* prd = nullptr;  // PageRankDelta: delta, contrib, dsum (3 n doubles)
  // selector features (graph level) and the attached selector
  FeatConst fc_bfs{}, fc_cc{}, fc_pr{};
  float* sel_p = nullptr;      // fp32 parameters, then mu[12], isd[12]
  uint16_t* sel_wb = nullptr;  // bf16 parameters
  float* sel_io = nullptr;     // PageRank decision: 12 features in, 4 predictions out
};

// A device array of the graph, listed for release; from the graph's
// workspace when `core` (the arrays gi_graph_create_ex sizes) and the graph
// has one.
template <typename T>
static gi_status dev_alloc(gi_graph* g, std::vector<void*>& list, T** p, size_t count,
                           bool core = false) {
  const size_t bytes = std::max<size_t>(1, count * sizeof(T));
  void* q = dmem_alloc(bytes, core ? &g->arena : nullptr);
  if (!q) {
    if (core && g->arena.base)
      return fail(GI_ERR_INVALID_ARG, "workspace of %zu bytes too small for the graph",
                  g->arena.size);
    return fail(GI_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes failed", bytes);
  }
  list.push_back(q);
  *p = static_cast<T*>(q);
  return GI_OK;
}

static void free_list(std::vector<void*>& list) {
  for (void* p : list) dmem_free(p);
  list.clear();
}

// Host worker threads for the O(m) ingest and set-up passes: fn(t) runs on
// worker t of host_workers(), worker 0 on the calling thread.
static unsigned host_workers() {
  return std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
}

// Returns false if a worker ran out of host memory (its exception is caught
// in the worker, so it cannot end the process).
static bool run_workers(const std::function<void(unsigned)>& fn) {
  const unsigned nth = host_workers();
  std::vector<char> ok(nth, 1);
  auto guarded = [&](unsigned t) {
    try {
      fn(t);
    } catch (...) {
      ok[t] = 0;
    }
  };
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < nth; ++t) pool.emplace_back(guarded, t);
  guarded(0);
  for (auto& th : pool) th.join();
  return std::all_of(ok.begin(), ok.end(), [](char c) { return c != 0; });
}

// Row range [lo, hi) of worker t out of nth over n rows.
static inline int32_t worker_row(int32_t n, unsigned t, unsigned nth) {
  return (int32_t)((int64_t)n * t / nth);
}

// ------------------------------------------------------ adjacency checks --

static gi_status check_adjacency(int32_t n, int64_t m, const int32_t* off, const int32_t* idx,
                                 const char* what) {
  if (!off || (m > 0 && !idx)) return fail(GI_ERR_INVALID_ARG, "%s: NULL array", what);
  if (off[0] != 0) return fail(GI_ERR_INVALID_ARG, "%s: off[0] = %d, expected 0", what, off[0]);
  if ((int64_t)off[n] != m)
    return fail(GI_ERR_INVALID_ARG, "%s: off[n] = %d does not equal m = %lld", what, off[n],
                (long long)m);
  for (int32_t v = 0; v < n; ++v) {
    const int32_t b = off[v], e = off[v + 1];
    if (e < b) return fail(GI_ERR_INVALID_ARG, "%s: offsets decrease at row %d", what, v);
    for (int32_t k = b; k < e; ++k) {
      const int32_t u = idx[k];
      if (u < 0 || u >= n)
        return fail(GI_ERR_INVALID_ARG, "%s: neighbour %d of row %d out of range", what, u, v);
      if (k > b && idx[k - 1] >= u)
        return fail(GI_ERR_INVALID_ARG, "%s: row %d not strictly ascending", what, v);
    }
  }
  return GI_OK;
}

// ------------------------------------------------------------- ingest ----

// Adjacency from raw records: rows bucketed by source, each row sorted by
// (neighbour, weight) packed into 64-bit keys, repeated neighbours dropped so
// that the smallest weight survives.
extern "C" gi_status gi_build_adjacency(int32_t n, int64_t nrec, const int32_t* src,
                                        const int32_t* dst, const uint32_t* w, int32_t* off,
                                        int32_t* idx, uint32_t* w_out, int64_t* m_out) {
  if (n < 1) return fail(GI_ERR_INVALID_ARG, "n must be >= 1 (got %d)", n);
  if (nrec < 0) return fail(GI_ERR_INVALID_ARG, "negative record count");
  if ((nrec > 0 && (!src || !dst || !idx)) || !off || !m_out)
    return fail(GI_ERR_INVALID_ARG, "NULL array");
  if (w_out && !w) return fail(GI_ERR_INVALID_ARG, "w_out given without input weights");
  // Worker threads: records are checked in slices; rows are split into
  // contiguous ranges, and each worker scans every record but counts and
  // places only those of its own rows, so the random writes stay private
  // to a worker and the placement order within a row is the record order.
  const unsigned nth = host_workers();
  const auto& run = run_workers;
  auto row_lo = [&](unsigned t) { return worker_row(n, t, nth); };
  std::vector<int64_t> first_bad(nth, nrec);
  run([&](unsigned t) {
    const int64_t lo = nrec * (int64_t)t / nth, hi = nrec * (int64_t)(t + 1) / nth;
    for (int64_t k = lo; k < hi; ++k)
      if ((uint32_t)src[k] >= (uint32_t)n || (uint32_t)dst[k] >= (uint32_t)n) {
        first_bad[t] = k;
        break;
      }
  });
  const int64_t bad = *std::min_element(first_bad.begin(), first_bad.end());
  if (bad < nrec)
    return fail(GI_ERR_INVALID_ARG, "record %lld has an endpoint outside [0, %d)", (long long)bad, n);
  std::vector<int64_t> start((size_t)n + 1, 0);
  run([&](unsigned t) {
    const int32_t r0 = row_lo(t), r1 = row_lo(t + 1);
    for (int64_t k = 0; k < nrec; ++k) {
      const int32_t u = src[k];
      if (u >= r0 && u < r1 && u != dst[k]) start[(size_t)u + 1]++;
    }
  });
  for (int32_t v = 0; v < n; ++v) start[(size_t)v + 1] += start[(size_t)v];
  std::vector<uint64_t> keys;
  try {
    keys.resize((size_t)start[(size_t)n]);
  } catch (...) {
    return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  if (!run([&](unsigned t) {
    const int32_t r0 = row_lo(t), r1 = row_lo(t + 1);
    std::vector<int64_t> cur(start.begin() + r0, start.begin() + r1);
    for (int64_t k = 0; k < nrec; ++k) {
      const int32_t u = src[k];
      if (u < r0 || u >= r1 || u == dst[k]) continue;
      keys[(size_t)cur[(size_t)(u - r0)]++] =
          ((uint64_t)(uint32_t)dst[k] << 32) | (uint64_t)(w ? w[k] : 0u);
    }
  }))
    return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed");
  // sort and de-duplicate rows; kept[v] = distinct neighbours of v
  std::vector<int64_t> kept((size_t)n, 0);
  run([&](unsigned t) {
    for (int32_t v = (int32_t)t; v < n; v += (int32_t)nth) {
      uint64_t* b = keys.data() + start[(size_t)v];
      uint64_t* e = keys.data() + start[(size_t)v + 1];
      std::sort(b, e);
      int64_t k = 0;
      for (uint64_t* p = b; p < e; ++p)
        if (k == 0 || (b[k - 1] >> 32) != (*p >> 32)) b[k++] = *p;
      kept[(size_t)v] = k;
    }
  });
  int64_t m = 0;
  off[0] = 0;
  for (int32_t v = 0; v < n; ++v) {
    m += kept[(size_t)v];
    if (m > INT32_MAX) return fail(GI_ERR_OVERFLOW, "more than 2^31-1 edges");
    off[v + 1] = (int32_t)m;
  }
  run([&](unsigned t) {
    for (int32_t v = row_lo(t); v < row_lo(t + 1); ++v) {
      const uint64_t* b = keys.data() + start[(size_t)v];
      for (int64_t k = 0; k < kept[(size_t)v]; ++k) {
        idx[off[v] + k] = (int32_t)(b[k] >> 32);
        if (w_out) w_out[off[v] + k] = (uint32_t)(b[k] & 0xffffffffu);
      }
    }
  });
  *m_out = m;
  return GI_OK;
}

// ------------------------------------------------ destination blocks ----

// Greedy split of rows [0, nrows) into blocks of consecutive rows holding at
// most cap_e edges and cap_v rows; a row above cap_e edges is its own block.
// Long rows are listed first.
static std::vector<int2> make_row_blocks(const int32_t* off, int nrows, int cap_e, int cap_v) {
  std::vector<int2> longs, rest;
  int r = 0;
  while (r < nrows) {
    const int64_t d = (int64_t)off[r + 1] - off[r];
    if (d > cap_e) {
      longs.push_back(make_int2(r, r + 1));
      ++r;
      continue;
    }
    int e = r;
    int64_t sum = 0;
    while (e < nrows && e - r < cap_v) {
      const int64_t de = (int64_t)off[e + 1] - off[e];
      if (de > cap_e || sum + de > cap_e) break;
      sum += de;
      ++e;
    }
    rest.push_back(make_int2(r, e));
    r = e;
  }
  longs.insert(longs.end(), rest.begin(), rest.end());
  return longs;
}

// CC pull blocks: whole-row blocks as above, except that a row longer than
// cap_e becomes ceil(len/cap_e) chunk entries (row, -(c+1)), listed first,
// so that no workgroup walks a hub row alone.
// Each entry also carries its edge range, so a kernel needs no dependent
// load of the row offsets before fetching the edges.
static std::vector<int4> make_cc_table(const int32_t* off, int nrows, int cap_e, int cap_v) {
  std::vector<int2> tab = make_row_blocks(off, nrows, cap_e, cap_v);
  std::vector<int4> out;
  size_t i = 0;
  for (; i < tab.size(); ++i) {
    const int r = tab[i].x;
    const int64_t d = (int64_t)off[r + 1] - off[r];
    if (tab[i].y != r + 1 || d <= cap_e) break;  // past the long rows
    const int64_t nc = (d + cap_e - 1) / cap_e;
    for (int64_t c = 0; c < nc; ++c) {
      const int64_t eb = off[r] + c * cap_e;
      out.push_back(make_int4(r, -(int)(c + 1), (int)eb, (int)std::min<int64_t>(off[r + 1], eb + cap_e)));
    }
  }
  for (; i < tab.size(); ++i)
    out.push_back(make_int4(tab[i].x, tab[i].y, off[tab[i].x], off[tab[i].y]));
  return out;
}

// PageRank + eigenvector blocks: as make_cc_table, except that a chunk
// entry names its row's long-row slot (rows in `lrow`) instead of the row.
static std::vector<int4> make_prec_table(const int32_t* off, int nrows, int cap_e, int cap_v,
                                         std::vector<int32_t>* lrow) {
  std::vector<int4> tab = make_cc_table(off, nrows, cap_e, cap_v);
  lrow->clear();
  for (int4& e : tab) {
    if (e.y >= 0) break;  // chunk entries come first
    if (e.y == -1) lrow->push_back(e.x);
    e.x = (int)lrow->size() - 1;
  }
  return tab;
}

// PageRank destination blocks: whole-row blocks as above, except that a
// row longer than cap_e becomes ceil(len/cap_e) chunk entries (listed
// first) sharing one long-row slot.
static std::vector<int4> make_pr_table(const int32_t* off, int nrows, int cap_e, int cap_v,
                                       std::vector<int32_t>* chunks) {
  std::vector<int4> longs, rest;
  chunks->clear();
  int r = 0;
  while (r < nrows) {
    const int64_t d = (int64_t)off[r + 1] - off[r];
    if (d > cap_e) {
      const int slot = (int)chunks->size();
      const int nc = (int)((d + cap_e - 1) / cap_e);
      chunks->push_back(nc);
      for (int c = 0; c < nc; ++c) longs.push_back(make_int4(r, r + 1, slot, c));
      ++r;
      continue;
    }
    int e = r;
    int64_t sum = 0;
    while (e < nrows && e - r < cap_v) {
      const int64_t de = (int64_t)off[e + 1] - off[e];
      if (de > cap_e || sum + de > cap_e) break;
      sum += de;
      ++e;
    }
    rest.push_back(make_int4(r, e, -1, 0));
    r = e;
  }
  longs.insert(longs.end(), rest.begin(), rest.end());
  return longs;
}

// Graph-level selector features: log2 n, log2 E, E/n, log2(1 + max deg),
// coefficient of variation of the degrees; and the algorithm id.
static FeatConst feat_const(const int32_t* deg, int32_t n, int64_t edges, float alg) {
  FeatConst c{};
  double sum = 0.0, sq = 0.0;
  int32_t mx = 0;
  for (int32_t v = 0; v < n; ++v) {
    sum += deg[v];
    sq += (double)deg[v] * deg[v];
    mx = std::max(mx, deg[v]);
  }
  const double mean = sum / n, var = std::max(0.0, sq / n - mean * mean);
  c.g[0] = (float)std::log2((double)n);
  c.g[1] = (float)std::log2((double)std::max<int64_t>(edges, 1));
  c.g[2] = (float)((double)edges / n);
  c.g[3] = (float)std::log2(1.0 + mx);
  c.g[4] = mean > 0.0 ? (float)(std::sqrt(var) / mean) : 0.0f;
  c.alg = alg;
  return c;
}

static gi_status upload(const void* h, void* d, size_t bytes) {
  if (bytes == 0) return GI_OK;
  HIP_TRY(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice));
  return GI_OK;
}

// Segments of the in-adjacency by source range (section 2, cache
// partitioning; configApplyNumSSG).  Rows keep only destinations with at
// least one in-edge from the segment.
static gi_status build_segments(gi_graph* g, int p, int strategy) {
  const int32_t n = g->n;
  HIP_TRY(hipDeviceSynchronize());
  free_list(g->seg_allocs);
  g->segs.clear();
  g->pr_acc = nullptr;
  g->seg_rows = nullptr;
  g->seg_p = 0;
  std::vector<int64_t> bound((size_t)p + 1, 0);
  if (strategy == GI_SEG_FIXED_VERTEX_COUNT) {
    const int64_t per = ((int64_t)n + p - 1) / p;
    for (int i = 0; i <= p; ++i) bound[(size_t)i] = std::min<int64_t>(n, per * i);
  } else {  // edge-aware: equal shares of out-edges (the edges each segment's sources own)
    const int64_t total = g->m;
    int64_t acc = 0;
    int seg = 1;
    for (int32_t u = 0; u < n && seg < p; ++u) {
      acc += g->h_outdeg[(size_t)u];
      while (seg < p && acc * p >= total * seg) bound[(size_t)seg++] = u + 1;
    }
    for (; seg < p; ++seg) bound[(size_t)seg] = n;
    bound[(size_t)p] = n;
  }
  const int32_t* off = g->h_in_off.data();
  const int32_t* idx = g->h_in_idx.data();
  g->segs.assign((size_t)p, SegDev());
  // host arrays of a wave of segments are built by worker threads, one
  // segment each, then uploaded in segment order
  struct HostSeg {
    std::vector<int32_t> soff, sidx, sdst, chunks;
    std::vector<int4> tab;
    bool failed = false;
  };
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  for (int w0 = 0; w0 < p; w0 += nth) {
    const int w1 = std::min(p, w0 + nth);
    std::vector<HostSeg> hs((size_t)(w1 - w0));
    auto build_one = [&](int i) {
      HostSeg& h = hs[(size_t)(i - w0)];
      const int32_t lo = (int32_t)bound[(size_t)i], hi = (int32_t)bound[(size_t)i + 1];
      h.soff.push_back(0);
      for (int32_t v = 0; v < n; ++v) {
        const int32_t* rb = idx + off[v];
        const int32_t* re = idx + off[v + 1];
        const int32_t* a = std::lower_bound(rb, re, lo);
        const int32_t* z = std::lower_bound(a, re, hi);
        if (a == z) continue;
        h.sidx.insert(h.sidx.end(), a, z);
        h.sdst.push_back(v);
        h.soff.push_back((int32_t)h.sidx.size());
      }
      h.tab = make_pr_table(h.soff.data(), (int)h.sdst.size(), g->pr_cap_e, g->pr_cap_v,
                            &h.chunks);
    };
    auto work = [&](int i) {
      try {
        build_one(i);
      } catch (...) {
        hs[(size_t)(i - w0)].failed = true;
      }
    };
    std::vector<std::thread> pool;
    for (int i = w0 + 1; i < w1; ++i) pool.emplace_back(work, i);
    work(w0);
    for (auto& th : pool) th.join();
    for (const HostSeg& h : hs)
      if (h.failed) return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed (segments)");
    for (int i = w0; i < w1; ++i) {
      const HostSeg& h = hs[(size_t)(i - w0)];
      SegDev& sg = g->segs[(size_t)i];
      sg.nrows = (int)h.sdst.size();
      sg.nnz = (int64_t)h.sidx.size();
      sg.ntab = (int)h.tab.size();
      gi_status st;
      if ((st = dev_alloc(g, g->seg_allocs, &sg.off, h.soff.size())) != GI_OK) return st;
      if ((st = dev_alloc(g, g->seg_allocs, &sg.idx, h.sidx.size())) != GI_OK) return st;
      if ((st = dev_alloc(g, g->seg_allocs, &sg.dst, h.sdst.size())) != GI_OK) return st;
      if ((st = dev_alloc(g, g->seg_allocs, &sg.table, h.tab.size())) != GI_OK) return st;
      if ((st = upload(h.soff.data(), sg.off, h.soff.size() * 4)) != GI_OK) return st;
      if ((st = upload(h.sidx.data(), sg.idx, h.sidx.size() * 4)) != GI_OK) return st;
      if ((st = upload(h.sdst.data(), sg.dst, h.sdst.size() * 4)) != GI_OK) return st;
      if ((st = upload(h.tab.data(), sg.table, h.tab.size() * sizeof(int4))) != GI_OK) return st;
    }
  }
  // one partial-sum buffer per segment (the concurrent form needs them all;
  // the sequential form uses the first)
  gi_status st = dev_alloc(g, g->seg_allocs, &g->pr_acc, (size_t)n * (size_t)p);
  if (st != GI_OK) return st;
  HIP_TRY(hipMemset(g->pr_acc, 0, sizeof(double) * (size_t)n * (size_t)p));
  std::vector<PrRows> rows;
  for (const SegDev& sg : g->segs)
    rows.push_back(PrRows{sg.table, sg.ntab, sg.off, sg.idx, sg.dst, nullptr, nullptr, nullptr});
  if ((st = dev_alloc(g, g->seg_allocs, &g->seg_rows, rows.size())) != GI_OK) return st;
  if ((st = upload(rows.data(), g->seg_rows, sizeof(PrRows) * rows.size())) != GI_OK) return st;
  g->seg_p = p;
  g->seg_strategy = strategy;
  g->seg_cap = g->pr_cap_e;
  return GI_OK;
}

// The schedule's segments, built when a segmented PageRank first needs them
// (a schedule change alone builds nothing, so alternating schedules between
// algorithms costs nothing).
static gi_status ensure_pr_segments(gi_graph* g, int p, int strategy) {
  if (!g->segs.empty() && g->seg_p == p && g->seg_strategy == strategy &&
      g->seg_cap == g->pr_cap_e)
    return GI_OK;
  return build_segments(g, p, strategy);
}

// The BFS pull's copy of the in-rows: each row ordered by decreasing source
// out-degree, ties by id, so it starts with the probe (in_probe) and goes on
// with the next most connected sources, the ones most likely to be on the
// frontier.  Same rows, same edges; only the order of a pull's scan changes
// (and with it which frontier in-neighbour becomes the parent).
static gi_status ensure_bfs_rows(gi_graph* g) {
  if (g->bfs_idx) return GI_OK;
  const int32_t n = g->n;
  const size_t m = (size_t)g->m;
  std::vector<int32_t> idx(g->h_in_idx.begin(), g->h_in_idx.begin() + (ptrdiff_t)m);
  const int32_t* io = g->h_in_off.data();
  const int32_t* od = g->h_outdeg.data();
  const unsigned nth = host_workers();
  const bool ok = run_workers([&](unsigned t) {
    for (int32_t v = worker_row(n, t, nth); v < worker_row(n, t + 1, nth); ++v)
      std::sort(idx.data() + io[v], idx.data() + io[v + 1], [od](int32_t a, int32_t b) {
        return od[a] != od[b] ? od[a] > od[b] : a < b;
      });
  });
  if (!ok) return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed (BFS in-rows)");
  int32_t* d = nullptr;
  gi_status st = dev_alloc(g, g->bfsr_allocs, &d, std::max<size_t>(1, m));
  if (st == GI_OK) st = upload(idx.data(), d, 4 * m);
  if (st != GI_OK) {
    free_list(g->bfsr_allocs);
    return st;
  }
  g->bfs_idx = d;
  return GI_OK;
}

// Degree-ordered copy of the in-adjacency (PageRank, vertex_order =
// GI_ORDER_OUT_DEGREE): new ids by decreasing out-degree, ties by id; row r
// holds the new ids of the in-neighbours of old_id[r], sorted.
static gi_status ensure_pr_order(gi_graph* g) {
  if (g->ord_off) return GI_OK;
  const int32_t n = g->n;
  const int64_t m = g->m;
  std::vector<int32_t> old_id((size_t)n), new_id((size_t)n), deg((size_t)n);
  {
    // counting sort by out-degree, highest first, stable in the old id
    std::vector<int64_t> start((size_t)g->max_out + 2, 0);
    for (int32_t v = 0; v < n; ++v) ++start[(size_t)(g->max_out - g->h_outdeg[(size_t)v]) + 1];
    for (size_t b = 1; b < start.size(); ++b) start[b] += start[b - 1];
    for (int32_t v = 0; v < n; ++v) {
      const int64_t r = start[(size_t)(g->max_out - g->h_outdeg[(size_t)v])]++;
      old_id[(size_t)r] = v;
      new_id[(size_t)v] = (int32_t)r;
    }
  }
  int32_t nsrc = 0;
  for (int32_t r = 0; r < n; ++r) {
    deg[(size_t)r] = g->h_outdeg[(size_t)old_id[(size_t)r]];
    if (deg[(size_t)r] > 0) nsrc = r + 1;
  }
  std::vector<int32_t>& off = g->h_ord_off;
  off.assign((size_t)n + 1, 0);
  for (int32_t r = 0; r < n; ++r) {
    const int32_t v = old_id[(size_t)r];
    off[(size_t)r + 1] = off[(size_t)r] + (g->h_in_off[(size_t)v + 1] - g->h_in_off[(size_t)v]);
  }
  std::vector<int32_t> idx((size_t)m);
  const unsigned nth = host_workers();
  const bool ok = run_workers([&](unsigned t) {
    const int32_t lo = worker_row(n, t, nth), hi = worker_row(n, t + 1, nth);
    for (int32_t r = lo; r < hi; ++r) {
      const int32_t v = old_id[(size_t)r];
      int32_t* dst = idx.data() + off[(size_t)r];
      const int32_t b = g->h_in_off[(size_t)v], e = g->h_in_off[(size_t)v + 1];
      for (int32_t k = b; k < e; ++k) dst[k - b] = new_id[(size_t)g->h_in_idx[(size_t)k]];
      std::sort(dst, dst + (e - b));
    }
  });
  if (!ok) return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed (ordered in-adjacency)");
  gi_status st;
  if ((st = dev_alloc(g, g->ord_allocs, &g->ord_off, (size_t)n + 1)) != GI_OK ||
      (st = dev_alloc(g, g->ord_allocs, &g->ord_idx, std::max<size_t>(1, (size_t)m))) != GI_OK ||
      (st = dev_alloc(g, g->ord_allocs, &g->ord_outdeg, (size_t)n)) != GI_OK ||
      (st = dev_alloc(g, g->ord_allocs, &g->ord_old, (size_t)n)) != GI_OK) {
    free_list(g->ord_allocs);
    g->ord_off = nullptr;
    return st;
  }
  if ((st = upload(off.data(), g->ord_off, 4 * ((size_t)n + 1))) != GI_OK ||
      (st = upload(idx.data(), g->ord_idx, 4 * (size_t)m)) != GI_OK ||
      (st = upload(deg.data(), g->ord_outdeg, 4 * (size_t)n)) != GI_OK ||
      (st = upload(old_id.data(), g->ord_old, 4 * (size_t)n)) != GI_OK) {
    free_list(g->ord_allocs);
    g->ord_off = nullptr;
    return st;
  }
  g->ord_nsrc = nsrc;
  return GI_OK;
}

// Merge-path tiles of T items over the ordered in-adjacency (n row ends and
// m edges; the end of row r is item off[r + 1] + r).  Tile t starts at the
// row r holding item t T and the edge t T - r.  A row with edges in one tile
// and its end (or more edges) in a later one gets a split slot.
static gi_status ensure_pr_order_tiles(gi_graph* g, int T) {
  if (g->ord_tiles && g->ord_T == T) return GI_OK;
  HIP_TRY(hipDeviceSynchronize());
  free_list(g->ordt_allocs);
  g->ord_tiles = nullptr;
  const int32_t n = g->n;
  const int64_t items = (int64_t)n + g->m;
  const int64_t nt64 = (items + T - 1) / T;
  if (nt64 > INT32_MAX - 1) return fail(GI_ERR_OVERFLOW, "too many PageRank tiles");
  const int nt = (int)nt64;
  const int32_t* off = g->h_ord_off.data();
  std::vector<int2> tiles((size_t)nt + 1);
  for (int t = 0; t < nt; ++t) {
    const int64_t d = (int64_t)t * T;
    // rows whose end item lies before d
    int32_t lo = 0, hi = n;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      if ((int64_t)off[(size_t)mid + 1] + mid < d) lo = mid + 1;
      else hi = mid;
    }
    tiles[(size_t)t] = make_int2(lo, (int32_t)(d - lo));
  }
  tiles[(size_t)nt] = make_int2(n, (int32_t)g->m);
  std::vector<int2> tslot((size_t)nt, make_int2(-1, -1));
  std::vector<int32_t> srow;
  for (int t = 0; t < nt; ++t) {
    const int32_t r0 = tiles[(size_t)t].x, e0 = tiles[(size_t)t].y;
    const int32_t r1 = tiles[(size_t)t + 1].x, e1 = tiles[(size_t)t + 1].y;
    if (r0 < n && off[(size_t)r0] < e0) {
      if (srow.empty() || srow.back() != r0)
        return fail(GI_ERR_DEVICE, "PageRank tiles: inconsistent split row");
      tslot[(size_t)t].x = (int32_t)srow.size() - 1;
    }
    if (r1 < n && off[(size_t)r1] < e1) {
      if (srow.empty() || srow.back() != r1) srow.push_back(r1);
      tslot[(size_t)t].y = (int32_t)srow.size() - 1;
    }
  }
  const size_t ns = std::max<size_t>(1, srow.size());
  gi_status st;
  if ((st = dev_alloc(g, g->ordt_allocs, &g->ord_tiles, tiles.size())) != GI_OK ||
      (st = dev_alloc(g, g->ordt_allocs, &g->ord_tslot, tslot.size())) != GI_OK ||
      (st = dev_alloc(g, g->ordt_allocs, &g->ord_srow, ns)) != GI_OK ||
      (st = dev_alloc(g, g->ordt_allocs, &g->ord_sacc, ns)) != GI_OK) {
    free_list(g->ordt_allocs);
    g->ord_tiles = nullptr;
    return st;
  }
  if ((st = upload(tiles.data(), g->ord_tiles, sizeof(int2) * tiles.size())) != GI_OK ||
      (st = upload(tslot.data(), g->ord_tslot, sizeof(int2) * tslot.size())) != GI_OK ||
      (st = upload(srow.data(), g->ord_srow, 4 * srow.size())) != GI_OK) {
    free_list(g->ordt_allocs);
    g->ord_tiles = nullptr;
    return st;
  }
  HIP_TRY(hipMemset(g->ord_sacc, 0, sizeof(double) * ns));
  g->ord_ntiles = nt;
  g->ord_nslots = (int)srow.size();
  g->ord_T = T;
  return GI_OK;
}

static gi_status apply_schedule(gi_graph* g, const gi_schedule& s) {
  // only the PageRank block layout owns device tables here (segments are
  // built on first use): any other change is free
  if (g->pr_table && s.pull_block_edges == g->sched.pull_block_edges) {
    g->sched = s;
    return GI_OK;
  }
  HIP_TRY(hipDeviceSynchronize());
  free_list(g->sched_allocs);
  free_list(g->seg_allocs);
  g->segs.clear();
  g->seg_p = 0;
  g->pr_acc = nullptr;
  g->seg_rows = nullptr;
  g->pr_table = nullptr;
  g->sched = s;
  if (s.pull_block_edges > 0) {
    g->pr_cap_e = s.pull_block_edges;
  } else {
    // about 2048 destination blocks (eight per CU): the power of two in
    // [256, 2048] nearest above m / 2048 edges per block
    int cap = 256;
    while (cap < 2048 && (int64_t)cap * 2048 < g->m) cap *= 2;
    g->pr_cap_e = cap;
  }
  g->pr_cap_v = std::min(g->pr_cap_e, 1024);
  std::vector<int32_t> chunks;
  std::vector<int4> tab = make_pr_table(g->h_in_off.data(), g->n, g->pr_cap_e, g->pr_cap_v,
                                        &chunks);
  g->pr_ntab = (int)tab.size();
  gi_status st = dev_alloc(g, g->sched_allocs, &g->pr_table, tab.size());
  if (st != GI_OK) return st;
  if ((st = upload(tab.data(), g->pr_table, tab.size() * sizeof(int4))) != GI_OK) return st;
  g->pr_nlong = (int)chunks.size();
  const size_t nl = std::max<size_t>(1, chunks.size());
  if ((st = dev_alloc(g, g->sched_allocs, &g->lr_acc, nl)) != GI_OK) return st;
  if ((st = dev_alloc(g, g->sched_allocs, &g->lr_cnt, nl)) != GI_OK) return st;
  if ((st = dev_alloc(g, g->sched_allocs, &g->lr_chunks, nl)) != GI_OK) return st;
  HIP_TRY(hipMemset(g->lr_acc, 0, sizeof(double) * nl));
  HIP_TRY(hipMemset(g->lr_cnt, 0, sizeof(unsigned) * nl));
  if ((st = upload(chunks.data(), g->lr_chunks, 4 * chunks.size())) != GI_OK) return st;
  return GI_OK;
}

extern "C" gi_status gi_schedule_init(gi_schedule* s) {
  if (!s) return fail(GI_ERR_INVALID_ARG, "NULL schedule");
  std::memset(s, 0, sizeof *s);
  s->direction = GI_DIR_DENSE_PULL_SPARSE_PUSH;
  s->dense_frontier = GI_FRONTIER_BITVECTOR;
  s->num_segments = 1;
  s->segment_strategy = GI_SEG_FIXED_VERTEX_COUNT;
  s->hybrid_divisor = 20;
  s->steps_per_sync = 0;
  s->pull_block_edges = 0;
  s->block_threads = 0;
  s->sssp_delta = 0;
  return GI_OK;
}

static gi_status validate_schedule(const gi_graph* g, const gi_schedule* s) {
  if (s->direction < GI_DIR_SPARSE_PUSH || s->direction > GI_DIR_LEARNED)
    return fail(GI_ERR_UNSUPPORTED, "direction %d not offered", s->direction);
  if (s->dense_frontier != GI_FRONTIER_BITVECTOR && s->dense_frontier != GI_FRONTIER_BOOLMAP)
    return fail(GI_ERR_UNSUPPORTED, "dense frontier kind %d not offered", s->dense_frontier);
  if (s->num_segments < 1 || s->num_segments > 4096)
    return fail(GI_ERR_UNSUPPORTED, "num_segments %d outside [1, 4096]", s->num_segments);
  if (s->segment_strategy != GI_SEG_FIXED_VERTEX_COUNT &&
      s->segment_strategy != GI_SEG_EDGE_AWARE_VERTEX_COUNT)
    return fail(GI_ERR_UNSUPPORTED, "segment strategy %d not offered", s->segment_strategy);
  if (s->hybrid_divisor < 1) return fail(GI_ERR_UNSUPPORTED, "hybrid_divisor must be >= 1");
  if (s->steps_per_sync < 0 || s->steps_per_sync > 4096)
    return fail(GI_ERR_UNSUPPORTED, "steps_per_sync outside [0, 4096]");
  if (s->pull_block_edges != 0 && (s->pull_block_edges < 64 || s->pull_block_edges > 8192))
    return fail(GI_ERR_UNSUPPORTED, "pull_block_edges outside [64, 8192]");
  if (s->segments_concurrent != 0 && s->segments_concurrent != 1)
    return fail(GI_ERR_UNSUPPORTED, "segments_concurrent must be 0 or 1");
  if (s->cc_adjacency < GI_CC_ADJ_AUTO || s->cc_adjacency > GI_CC_ADJ_DIRECT)
    return fail(GI_ERR_UNSUPPORTED, "cc_adjacency %d not offered", s->cc_adjacency);
  if (s->vertex_order != GI_ORDER_GIVEN && s->vertex_order != GI_ORDER_OUT_DEGREE)
    return fail(GI_ERR_UNSUPPORTED, "vertex_order %d not offered", s->vertex_order);
  if (s->vertex_order == GI_ORDER_OUT_DEGREE) {
    if (s->num_segments != 1)
      return fail(GI_ERR_UNSUPPORTED, "vertex_order OUT_DEGREE pulls unsegmented (num_segments 1)");
    if (s->block_threads != 0 && s->block_threads != 256 && s->block_threads != 512 &&
        s->block_threads != 1024)
      return fail(GI_ERR_UNSUPPORTED,
                  "block_threads must be 0, 256, 512 or 1024 with vertex_order OUT_DEGREE");
    if (s->pull_items_per_thread != 0 && s->pull_items_per_thread != 4 &&
        s->pull_items_per_thread != 8 && s->pull_items_per_thread != 16)
      return fail(GI_ERR_UNSUPPORTED, "pull_items_per_thread must be 0, 4, 8 or 16");
    if (s->pull_items_per_thread == 16 && s->block_threads == 1024)
      return fail(GI_ERR_UNSUPPORTED, "pull_items_per_thread 16 needs block_threads <= 512");
    if (s->pull_hot_sources < -1)
      return fail(GI_ERR_UNSUPPORTED, "pull_hot_sources must be -1, 0 or a count");
  } else {
    if (s->block_threads != 0 && s->block_threads != 64 && s->block_threads != 128 &&
        s->block_threads != 256 && s->block_threads != 512)
      return fail(GI_ERR_UNSUPPORTED, "block_threads must be 0, 64, 128, 256 or 512");
    if (s->pull_items_per_thread != 0 || s->pull_hot_sources != 0)
      return fail(GI_ERR_UNSUPPORTED,
                  "pull_items_per_thread and pull_hot_sources need vertex_order OUT_DEGREE");
  }
  if (s->reserved[0] != 0 || s->reserved[1] != 0)
    return fail(GI_ERR_UNSUPPORTED, "reserved schedule fields must be 0");
  (void)g;
  return GI_OK;
}

extern "C" gi_status gi_set_schedule(gi_graph* g, const gi_schedule* s) {
  if (!g || !s) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  gi_status st = validate_schedule(g, s);
  if (st != GI_OK) return st;
  return apply_schedule(g, *s);
}

extern "C" gi_status gi_get_schedule(const gi_graph* g, gi_schedule* s) {
  if (!g || !s) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  *s = g->sched;
  return GI_OK;
}

extern "C" int32_t gi_hybrid_choose_dense(int64_t nf, int64_t degsum, int64_t edges, int32_t divisor) {
  return hybrid_dense(nf, degsum, edges, divisor < 1 ? 1 : divisor) ? 1 : 0;
}

// ---------------------------------------------------------- lifecycle ----

extern "C" gi_status gi_graph_destroy(gi_graph* g) {
  if (!g) return GI_OK;
  (void)hipDeviceSynchronize();
  free_list(g->sched_allocs);
  free_list(g->seg_allocs);
  free_list(g->ccseg_allocs);
  free_list(g->ordt_allocs);
  free_list(g->ord_allocs);
  free_list(g->bfsr_allocs);
  free_list(g->allocs);
  for (void* q : {(void*)g->sel_p, (void*)g->sel_wb, (void*)g->sel_io}) dmem_free(q);
  if (g->hflags) (void)hipHostFree(g->hflags);
  if (g->prg_exec) (void)hipGraphExecDestroy(g->prg_exec);
  if (g->prg_graph) (void)hipGraphDestroy(g->prg_graph);
  if (g->prg_evw) (void)hipEventDestroy(g->prg_evw);
  if (g->prg_stream) (void)hipStreamDestroy(g->prg_stream);
  for (hipEvent_t e : g->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : g->evb)
    if (e) (void)hipEventDestroy(e);
  for (StepEvents& t : g->tev) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.main);
    (void)hipEventDestroy(t.end);
  }
  delete g;
  return GI_OK;
}

// Slots of a chunked expansion (frontier loops): at least kMinChunk slots
// each, at most kParts of them below the largest chunk size.
static size_t expand_chunks(size_t m) {
  return std::max((2 * m) / (size_t)expand_chunk_size(), (size_t)kParts) + 2;
}

// Bytes of the arrays gi_graph_create_ex places in a caller's workspace, each
// rounded up to 256 bytes, for a graph with `nhubs` vertices of out-degree
// above kHubDeg.  Must list exactly the G_ALLOC calls of create_graph.
static size_t core_bytes(int32_t n, int64_t m, bool weighted, size_t nhubs) {
  const size_t N = (size_t)n, M = (size_t)m, W = (N + 63) / 64;
  const size_t sizes[] = {
      4 * (N + 1), 4 * M, 4 * (N + 1), 4 * M, 4 * N, 4 * N,  // CSR, CSC, degrees
      4 * N, 4 * std::max<size_t>(1, nhubs),                 // probe, hubs
      weighted ? 4 * M : 0, weighted ? 4 * M : 0,            // weights
      8 * W, 64 * W, 8 * W, 64 * W, 8 * W, 8 * W,            // frontiers, visited, far
      4 * N, 4 * (N + 1), 4 * (N + 1),                       // labels, contributions
      sizeof(Part) * kParts, sizeof(Blk) * kMaxCount, 8 * (size_t)kMaxCount,
      4 * N, 8 * (N + 1), 4 * expand_chunks(M), sizeof(Control)};
  size_t total = 0;
  for (size_t b : sizes)
    if (b) total += arena_round(b);
  return total;
}

extern "C" gi_status gi_graph_workspace_size(int32_t n, int64_t m, int32_t weighted,
                                             size_t* bytes) {
  if (!bytes) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (n < 1) return fail(GI_ERR_INVALID_ARG, "n must be >= 1 (got %d)", n);
  if (n > INT32_MAX - 64) return fail(GI_ERR_OVERFLOW, "n too large");
  if (m < 0) return fail(GI_ERR_INVALID_ARG, "negative edge count");
  if (m > INT32_MAX) return fail(GI_ERR_OVERFLOW, "m = %lld exceeds 2^31-1", (long long)m);
  // at most m / (kHubDeg + 1) vertices have more than kHubDeg out-edges
  const size_t hub_bound = std::min<size_t>((size_t)n, (size_t)m / (kHubDeg + 1));
  *bytes = core_bytes(n, m, weighted != 0, hub_bound);
  return GI_OK;
}

static gi_status create_graph(int32_t n, int64_t m, const int32_t* out_off,
                              const int32_t* out_idx, const uint32_t* out_w,
                              const int32_t* in_off, const int32_t* in_idx,
                              const uint32_t* in_w, void* workspace, size_t ws_bytes,
                              hipStream_t stream, gi_graph** out);

extern "C" gi_status gi_graph_create(int32_t n, int64_t m, const int32_t* out_off,
                                     const int32_t* out_idx, const uint32_t* out_w,
                                     const int32_t* in_off, const int32_t* in_idx,
                                     const uint32_t* in_w, gi_graph** out) {
  return create_graph(n, m, out_off, out_idx, out_w, in_off, in_idx, in_w, nullptr, 0, nullptr,
                      out);
}

extern "C" gi_status gi_graph_create_ex(int32_t n, int64_t m, const int32_t* out_off,
                                        const int32_t* out_idx, const uint32_t* out_w,
                                        const int32_t* in_off, const int32_t* in_idx,
                                        const uint32_t* in_w, int32_t ptr_kind, void* workspace,
                                        size_t workspace_bytes, void* stream, gi_graph** out) {
  if (!out) return fail(GI_ERR_INVALID_ARG, "NULL output handle");
  *out = nullptr;
  if (ptr_kind != GI_PTR_HOST && ptr_kind != GI_PTR_DEVICE)
    return fail(GI_ERR_INVALID_ARG, "ptr_kind %d is neither GI_PTR_HOST nor GI_PTR_DEVICE",
                ptr_kind);
  if (workspace && ((uintptr_t)workspace % kArenaAlign) != 0)
    return fail(GI_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kArenaAlign);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ptr_kind == GI_PTR_HOST)
    return create_graph(n, m, out_off, out_idx, out_w, in_off, in_idx, in_w, workspace,
                        workspace_bytes, s, out);
  // device arrays: staged to the host once (validation and the schedule
  // tables are built there), in the caller's stream order
  if (n < 1) return fail(GI_ERR_INVALID_ARG, "n must be >= 1 (got %d)", n);
  if (n > INT32_MAX - 64) return fail(GI_ERR_OVERFLOW, "n too large");
  if (m < 0) return fail(GI_ERR_INVALID_ARG, "negative edge count");
  if (m > INT32_MAX) return fail(GI_ERR_OVERFLOW, "m = %lld exceeds 2^31-1", (long long)m);
  if (!out_off || (m > 0 && !out_idx)) return fail(GI_ERR_INVALID_ARG, "out-adjacency: NULL array");
  if ((!in_off && in_idx) || (in_off && m > 0 && !in_idx))
    return fail(GI_ERR_INVALID_ARG, "in_off and in_idx must both be given or both be NULL");
  std::vector<int32_t> h_oo, h_oi, h_io, h_ii;
  std::vector<uint32_t> h_ow, h_iw;
  try {
    h_oo.resize((size_t)n + 1);
    h_oi.resize((size_t)m);
    if (out_w) h_ow.resize((size_t)m);
    if (in_off) {
      h_io.resize((size_t)n + 1);
      h_ii.resize((size_t)m);
      if (in_w) h_iw.resize((size_t)m);
    }
  } catch (...) {
    return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  auto d2h = [&](void* h, const void* d, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s) : hipSuccess;
  };
  const size_t N = (size_t)n, M = (size_t)m;
  HIP_TRY(d2h(h_oo.data(), out_off, 4 * (N + 1)));
  HIP_TRY(d2h(h_oi.data(), out_idx, 4 * M));
  if (out_w) HIP_TRY(d2h(h_ow.data(), out_w, 4 * M));
  if (in_off) {
    HIP_TRY(d2h(h_io.data(), in_off, 4 * (N + 1)));
    HIP_TRY(d2h(h_ii.data(), in_idx, 4 * M));
    if (in_w) HIP_TRY(d2h(h_iw.data(), in_w, 4 * M));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return create_graph(n, m, h_oo.data(), h_oi.data(), out_w ? h_ow.data() : nullptr,
                      in_off ? h_io.data() : nullptr, in_off ? h_ii.data() : nullptr,
                      in_w ? h_iw.data() : nullptr, workspace, workspace_bytes, s, out);
}

static gi_status create_graph(int32_t n, int64_t m, const int32_t* out_off,
                              const int32_t* out_idx, const uint32_t* out_w,
                              const int32_t* in_off, const int32_t* in_idx,
                              const uint32_t* in_w, void* workspace, size_t ws_bytes,
                              hipStream_t stream, gi_graph** out) {
  if (!out) return fail(GI_ERR_INVALID_ARG, "NULL output handle");
  *out = nullptr;
  if (n < 1) return fail(GI_ERR_INVALID_ARG, "n must be >= 1 (got %d)", n);
  if (n > INT32_MAX - 64) return fail(GI_ERR_OVERFLOW, "n too large");
  if (m < 0) return fail(GI_ERR_INVALID_ARG, "negative edge count");
  if (m > INT32_MAX) return fail(GI_ERR_OVERFLOW, "m = %lld exceeds 2^31-1", (long long)m);
  gi_status st = check_adjacency(n, m, out_off, out_idx, "out-adjacency");
  if (st != GI_OK) return st;
  if ((!in_off && in_idx) || (in_off && m > 0 && !in_idx))
    return fail(GI_ERR_INVALID_ARG, "in_off and in_idx must both be given or both be NULL");
  if (in_w && !in_off) return fail(GI_ERR_INVALID_ARG, "in_w given without in-adjacency");
  if (in_off && (out_w != nullptr) != (in_w != nullptr))
    return fail(GI_ERR_INVALID_ARG, "weights must be given for both directions or neither");

  gi_graph* g = new (std::nothrow) gi_graph();
  if (!g) return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed");
  g->n = n;
  g->m = m;
  g->weighted = out_w != nullptr;
  g->arena.base = static_cast<char*>(workspace);
  g->arena.size = workspace ? ws_bytes : 0;
  // in-adjacency: given, or transposed here from the out-adjacency
  std::vector<int32_t> t_idx;
  std::vector<uint32_t> t_w;
  try {
    g->h_in_off.resize((size_t)n + 1);
    g->h_outdeg.resize((size_t)n);
    if (in_off) {
      st = check_adjacency(n, m, in_off, in_idx, "in-adjacency");
      if (st != GI_OK) {
        delete g;
        return st;
      }
      // every in-edge u->v must be an out-edge of u (with degrees equal below,
      // the two adjacencies then hold the same edge set); workers check row
      // ranges and report their first bad in-edge (position, kind)
      const unsigned nth = host_workers();
      std::vector<int64_t> bad_k(nth, -1);
      std::vector<int> bad_kind(nth, 0);
      run_workers([&](unsigned t) {
        for (int32_t v = worker_row(n, t, nth); v < worker_row(n, t + 1, nth); ++v)
          for (int32_t k = in_off[v]; k < in_off[v + 1]; ++k) {
            const int32_t u = in_idx[k];
            const int32_t* b = out_idx + out_off[u];
            const int32_t* e = out_idx + out_off[u + 1];
            const int32_t* f = std::lower_bound(b, e, v);
            const int kind = (f == e || *f != v) ? 1
                             : (in_w && out_w && in_w[k] != out_w[f - out_idx]) ? 2 : 0;
            if (kind) {
              bad_k[t] = k;
              bad_kind[t] = kind;
              return;
            }
          }
      });
      for (unsigned t = 0; t < nth; ++t) {
        if (!bad_kind[t]) continue;
        const int64_t k = bad_k[t];
        const int32_t v = (int32_t)(std::upper_bound(in_off, in_off + n + 1, (int32_t)k) - in_off - 1);
        const int32_t u = in_idx[k];
        delete g;
        if (bad_kind[t] == 1)
          return fail(GI_ERR_INVALID_ARG, "in-edge %d->%d is not an out-edge", u, v);
        return fail(GI_ERR_INVALID_ARG, "weight of %d->%d differs between adjacencies", u, v);
      }
      std::memcpy(g->h_in_off.data(), in_off, sizeof(int32_t) * ((size_t)n + 1));
      g->h_in_idx.assign(in_idx, in_idx + m);
    } else {
      std::vector<int32_t> cnt((size_t)n + 1, 0);
      for (int64_t k = 0; k < m; ++k) cnt[(size_t)out_idx[k] + 1]++;
      for (int32_t v = 0; v < n; ++v) cnt[(size_t)v + 1] += cnt[(size_t)v];
      std::memcpy(g->h_in_off.data(), cnt.data(), sizeof(int32_t) * ((size_t)n + 1));
      g->h_in_idx.resize((size_t)m);
      if (out_w) t_w.resize((size_t)m);
      for (int32_t u = 0; u < n; ++u)  // ascending u keeps CSC rows sorted
        for (int32_t k = out_off[u]; k < out_off[u + 1]; ++k) {
          const int32_t pos = cnt[(size_t)out_idx[k]]++;
          g->h_in_idx[(size_t)pos] = u;
          if (out_w) t_w[(size_t)pos] = out_w[k];
        }
    }
  } catch (...) {
    delete g;
    return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  // in-degrees of the two adjacencies must agree (CSC is the transpose)
  {
    std::vector<int32_t> indeg((size_t)n, 0);
    const unsigned nth = host_workers();
    run_workers([&](unsigned t) {
      const int32_t r0 = worker_row(n, t, nth), r1 = worker_row(n, t + 1, nth);
      for (int64_t k = 0; k < m; ++k) {
        const int32_t v = out_idx[k];
        if (v >= r0 && v < r1) indeg[(size_t)v]++;
      }
    });
    for (int32_t v = 0; v < n; ++v) {
      if (indeg[(size_t)v] != g->h_in_off[(size_t)v + 1] - g->h_in_off[(size_t)v]) {
        delete g;
        return fail(GI_ERR_INVALID_ARG, "in-adjacency is not the transpose (in-degree of %d)", v);
      }
      g->max_in = std::max(g->max_in, indeg[(size_t)v]);
    }
  }
  g->h_out_off.assign(out_off, out_off + (size_t)n + 1);
  std::vector<int32_t> h_udeg((size_t)n);
  for (int32_t v = 0; v < n; ++v) {
    g->h_outdeg[(size_t)v] = out_off[v + 1] - out_off[v];
    g->max_out = std::max(g->max_out, g->h_outdeg[(size_t)v]);
    h_udeg[(size_t)v] = g->h_outdeg[(size_t)v] + (g->h_in_off[(size_t)v + 1] - g->h_in_off[(size_t)v]);
  }
  g->fc_bfs = feat_const(g->h_outdeg.data(), n, m, 0.0f);
  g->fc_cc = feat_const(h_udeg.data(), n, 2 * m, 0.5f);
  g->fc_pr = feat_const(g->h_outdeg.data(), n, m, 1.0f);
  (void)hipGetDevice(&g->device);
  const size_t N = (size_t)n, M = (size_t)m, W = (N + 63) / 64;
#define G_ALLOC(ptr, cnt)                                             \
  do {                                                                \
    if ((st = dev_alloc(g, g->allocs, &(ptr), (cnt), true)) != GI_OK) { \
      gi_graph_destroy(g);                                            \
      return st;                                                      \
    }                                                                 \
  } while (0)
// copies in the caller's stream order; each waits for its own completion
// (some host arrays are scoped to a block below)
#define G_UP(h, d, bytes)                                             \
  do {                                                                \
    if ((bytes) > 0 &&                                                \
        (hipMemcpyAsync((d), (h), (bytes), hipMemcpyHostToDevice, stream) != hipSuccess || \
         hipStreamSynchronize(stream) != hipSuccess)) {               \
      (void)hipGetLastError();                                        \
      gi_graph_destroy(g);                                            \
      return fail(GI_ERR_DEVICE, "host-to-device copy of %zu bytes failed", (size_t)(bytes)); \
    }                                                                 \
  } while (0)
  if (g->arena.base) {
    size_t nh = 0;
    for (size_t v = 0; v < N; ++v) nh += g->h_outdeg[v] > kHubDeg;
    const size_t need = core_bytes(n, m, out_w != nullptr, nh);
    if (g->arena.size < need) {
      gi_graph_destroy(g);
      return fail(GI_ERR_INVALID_ARG, "workspace of %zu bytes, the graph needs %zu "
                  "(gi_graph_workspace_size)", g->arena.size, need);
    }
  }
  G_ALLOC(g->out_off, N + 1);
  G_ALLOC(g->out_idx, M);
  G_ALLOC(g->in_off, N + 1);
  G_ALLOC(g->in_idx, M);
  G_ALLOC(g->outdeg, N);
  G_ALLOC(g->udeg, N);
  G_UP(out_off, g->out_off, 4 * (N + 1));
  G_UP(out_idx, g->out_idx, 4 * M);
  G_UP(g->h_in_off.data(), g->in_off, 4 * (N + 1));
  G_UP(g->h_in_idx.data(), g->in_idx, 4 * M);
  G_UP(g->h_outdeg.data(), g->outdeg, 4 * N);
  G_UP(h_udeg.data(), g->udeg, 4 * N);
  {
    // first in-neighbour a BFS pull tests: the one of largest out-degree
    // (smallest id among equals).  Such hubs are reached early, so in the
    // large pull levels this one test usually finds a parent without
    // touching the in-row.
    std::vector<int32_t> probe(N, -1);
    const int32_t* io = g->h_in_off.data();
    const int32_t* ii = g->h_in_idx.data();
    const int32_t* od = g->h_outdeg.data();
    const unsigned nth = host_workers();
    run_workers([&](unsigned t) {
      for (int32_t v = worker_row(n, t, nth); v < worker_row(n, t + 1, nth); ++v) {
        int best = -1, bd = -1;
        for (int32_t e = io[v]; e < io[v + 1]; ++e)
          if (od[ii[e]] > bd) {
            bd = od[ii[e]];
            best = ii[e];
          }
        probe[(size_t)v] = best;
      }
    });
    G_ALLOC(g->in_probe, N);
    G_UP(probe.data(), g->in_probe, 4 * N);
    std::vector<int32_t> hubs;
    for (size_t v = 0; v < N; ++v)
      if (od[v] > kHubDeg) hubs.push_back((int32_t)v);
    g->nhubs = (int)hubs.size();
    G_ALLOC(g->hubs, std::max<size_t>(1, hubs.size()));
    if (!hubs.empty()) G_UP(hubs.data(), g->hubs, 4 * hubs.size());
  }
  if (out_w) {
    G_ALLOC(g->out_w, M);
    G_ALLOC(g->in_w, M);
    G_UP(out_w, g->out_w, 4 * M);
    G_UP(in_off ? in_w : t_w.data(), g->in_w, 4 * M);
  }
  // frontier-loop workspace
  // chunks of at least kMinChunk slots, at most kParts of them below the
  // largest chunk size
  const size_t nchunk = expand_chunks(M);
  for (int k = 0; k < 2; ++k) {
    G_ALLOC(g->fbv[k], W);
    G_ALLOC(g->fbm[k], W * 64);
  }
  G_ALLOC(g->vis, W);
  G_ALLOC(g->far, W);
  G_ALLOC(g->lab, N);
  // one slot past n: the ordered PageRank pull sends the stores of lanes
  // without a row there, so that every lane issues the same stores
  G_ALLOC(g->contrib[0], N + 1);
  G_ALLOC(g->contrib[1], N + 1);
  G_ALLOC(g->part, kParts);
  G_ALLOC(g->blk, kMaxCount);
  G_ALLOC(g->fmin, kMaxCount);
  G_ALLOC(g->ids, N);
  G_ALLOC(g->excl, N + 1);
  G_ALLOC(g->chunk_item, nchunk);
  G_ALLOC(g->ctl, 1);
  {
    // count/write workgroups own >= 256 bitvector words each (at most
    // kMaxCount workgroups); step kernels always run kParts workgroups
    Engine& e = g->eng;
    e.n = n;
    e.cgrid = (int)std::max<size_t>(1, std::min<size_t>(kMaxCount, (W + 255) / 256));
    e.tw = (int)((W + e.cgrid - 1) / e.cgrid);
    e.blk = g->blk;
    e.ids = g->ids;
    e.excl = g->excl;
    e.chunk_item = g->chunk_item;
    e.chunk_cap = (long long)nchunk;
    e.ctl = g->ctl;
  }
#undef G_ALLOC
#undef G_UP

  if (hipHostMalloc((void**)&g->hflags, sizeof(HostFlags),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&g->dflags, g->hflags, 0) != hipSuccess) {
    (void)hipGetLastError();
    gi_graph_destroy(g);
    return fail(GI_ERR_OUT_OF_MEMORY, "pinned host flags allocation failed");
  }
  std::memset(g->hflags, 0, sizeof(HostFlags));
  for (hipEvent_t* e : {&g->ev[0], &g->ev[1], &g->evb[0], &g->evb[1]}) {
    if (hipEventCreate(e) != hipSuccess) {
      (void)hipGetLastError();
      *e = nullptr;
      gi_graph_destroy(g);
      return fail(GI_ERR_DEVICE, "hipEventCreate failed");
    }
  }
  gi_schedule s;
  gi_schedule_init(&s);
  if ((st = apply_schedule(g, s)) != GI_OK) {
    gi_graph_destroy(g);
    return st;
  }
  *out = g;
  return GI_OK;
}

extern "C" gi_status gi_graph_info(const gi_graph* g, int32_t* n, int64_t* m, int32_t* max_out,
                                   int32_t* max_in) {
  if (!g) return fail(GI_ERR_INVALID_ARG, "NULL graph");
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (max_out) *max_out = g->max_out;
  if (max_in) *max_in = g->max_in;
  return GI_OK;
}

extern "C" gi_status gi_graph_copy_in_adjacency(const gi_graph* g, int32_t* in_off, int32_t* in_idx,
                                                uint32_t* in_w) {
  if (!g || !in_off || (g->m > 0 && !in_idx)) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (in_w && !g->weighted) return fail(GI_ERR_INVALID_ARG, "graph has no weights");
  HIP_TRY(hipMemcpy(in_off, g->in_off, 4 * ((size_t)g->n + 1), hipMemcpyDeviceToHost));
  if (g->m > 0) HIP_TRY(hipMemcpy(in_idx, g->in_idx, 4 * (size_t)g->m, hipMemcpyDeviceToHost));
  if (in_w && g->m > 0) HIP_TRY(hipMemcpy(in_w, g->in_w, 4 * (size_t)g->m, hipMemcpyDeviceToHost));
  return GI_OK;
}

// ------------------------------------------------------- helpers -----

static DevGraph dev_graph(const gi_graph* g) {
  DevGraph d;
  d.n = g->n;
  d.m = g->m;
  d.out_off = g->out_off;
  d.out_idx = g->out_idx;
  d.out_w = g->out_w;
  d.in_off = g->in_off;
  d.in_idx = g->in_idx;
  d.in_w = g->in_w;
  d.outdeg = g->outdeg;
  d.udeg = g->udeg;
  d.in_probe = g->in_probe;
  d.bfs_idx = g->bfs_idx;
  return d;
}

static DenseSet frontier_set(const gi_graph* g, int k) {
  DenseSet d;
  const bool bm = g->sched.dense_frontier == GI_FRONTIER_BOOLMAP;
  d.bv = bm ? nullptr : g->fbv[k & 1];
  d.bm = bm ? g->fbm[k & 1] : nullptr;
  return d;
}

// Copy the control block and the step log of the last frontier loop (one
// copy) into g->stats.
// Events of step k when per-step timing is on (nullptr otherwise, or past
// the trace capacity).  Events are created on first use and kept.
static const StepEvents* step_events(gi_graph* g, long long k) {
  if (!g->step_timing || k >= kMaxLog || g->timing_failed) return nullptr;
  while ((long long)g->tev.size() <= k) {
    StepEvents t{nullptr, nullptr, nullptr};
    // timing-only events: no system-scope cache writeback at each record
    const unsigned fl = hipEventDisableSystemFence;
    if (hipEventCreateWithFlags(&t.start, fl) != hipSuccess ||
        hipEventCreateWithFlags(&t.main, fl) != hipSuccess ||
        hipEventCreateWithFlags(&t.end, fl) != hipSuccess) {
      (void)hipGetLastError();
      for (hipEvent_t e : {t.start, t.main, t.end})
        if (e) (void)hipEventDestroy(e);
      g->timing_failed = true;
      return nullptr;
    }
    g->tev.push_back(t);
  }
  g->tev_count = std::max(g->tev_count, (int)k + 1);
  return &g->tev[(size_t)k];
}

static gi_status read_loop_stats(gi_graph* g, int alg) {
  const volatile HostFlags* h = g->hflags;
  gi_run_stats& r = g->stats;
  r.algorithm = alg;
  r.steps = h->steps;
  r.dense_steps = h->dense_steps;
  r.edges_examined = (int64_t)h->edges_examined;
  r.trace_len = std::min(r.steps, GI_MAX_TRACE);
  g->last_steps[alg] = r.steps;
  for (int i = 0; i < r.trace_len; ++i) {
    r.step_direction[i] = (int8_t)(h->log[i].dir % kLogSegmented);
    r.step_segmented[i] = (int8_t)(h->log[i].dir / kLogSegmented);
    r.step_frontier[i] = h->log[i].frontier;
    r.step_degree_sum[i] = h->log[i].degsum;
    r.step_edges[i] = h->log[i].edges;
  }
  return GI_OK;
}

// GPU time between the two timing events of the last run.
static gi_status read_kernel_ms(gi_graph* g, int launches) {
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, g->ev[0], g->ev[1]));
  g->stats.kernel_ms = ms;
  g->stats.launches = launches;
  g->stats_pending = 0;
  return GI_OK;
}

// Wait for the graph's last enqueued run (its end event) and read its time
// if a call returned before its work finished.
static gi_status finish_pending(gi_graph* g) {
  HIP_TRY(hipEventSynchronize(g->ev[1]));
  if (g->stats_pending) return read_kernel_ms(g, g->stats_pending);
  return GI_OK;
}

extern "C" gi_status gi_sync_status(gi_graph* g) {
  if (!g) return fail(GI_ERR_INVALID_ARG, "NULL graph");
  gi_status st = finish_pending(g);
  if (st != GI_OK) return st;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GI_ERR_DEVICE, "device error: %s", hipGetErrorString(e));
  return GI_OK;
}

// Enqueue steps in batches until the device reports completion through the
// pinned host flags.  `step(k)` enqueues step k and returns the number of
// kernels it launched (negative on a launch error).  The first batch is
// sized from the previous run of the same algorithm, so a run of the usual
// length needs one host synchronisation; longer runs continue with two
// batches in flight, so the stream never drains while the host looks at the
// flags.  Steps enqueued after completion see the finished state and return
// at once.
template <class StepFn>
static gi_status run_frontier_loop(gi_graph* g, hipStream_t s, int alg, int dflt,
                                   long long max_steps, StepFn step, const char* what) {
  int launches = 0;
  long long k = 0;
  g->tev_count = 0;
  const int fixed = g->sched.steps_per_sync;
  const int first = fixed > 0 ? fixed
                              : (g->last_steps[alg] > 0 ? std::min(g->last_steps[alg] + 1, kMaxLog)
                                                        : dflt);
  const int batch = fixed > 0 ? fixed : dflt;
  long long kmark[2] = {0, 0};  // steps enqueued when each batch event was recorded
  auto enqueue = [&](int nb, int j) -> gi_status {
    for (int b = 0; b < nb; ++b, ++k) {
      const int nl = step(k);
      if (nl < 0) {
        hipError_t e = hipGetLastError();
        return fail(GI_ERR_DEVICE, "%s: kernel launch failed: %s", what, hipGetErrorString(e));
      }
      launches += nl;
    }
    HIP_TRY(hipEventRecord(g->evb[j], s));
    kmark[j] = k;
    return GI_OK;
  };
  // Waits for batch event j; *done once the device reported completion.
  auto finished = [&](int j, bool* done) -> gi_status {
    HIP_TRY(hipEventSynchronize(g->evb[j]));
    const volatile HostFlags* f = g->hflags;
    if (f->error) return fail(GI_ERR_DEVICE, "%s: internal size check failed", what);
    *done = f->done != 0;
    if (!*done && kmark[j] > max_steps) return fail(GI_ERR_DEVICE, "%s did not terminate", what);
    return GI_OK;
  };
  HIP_TRY(hipEventRecord(g->ev[0], s));
  gi_status st = enqueue(first, 0);
  bool done = false;
  if (st == GI_OK) st = finished(0, &done);
  if (st == GI_OK && !done) {
    st = enqueue(batch, 0);
    for (int i = 1; st == GI_OK; ++i) {
      if ((st = enqueue(batch, i & 1)) != GI_OK) break;
      if ((st = finished((i - 1) & 1, &done)) != GI_OK || done) break;
    }
  }
  HIP_TRY(hipEventRecord(g->ev[1], s));
  HIP_TRY(hipEventSynchronize(g->ev[1]));
  if (st != GI_OK) return st;
  if (g->timing_failed) return fail(GI_ERR_DEVICE, "%s: could not create timing events", what);
  return read_kernel_ms(g, launches);
}

// Reset the control block and the pinned flags before a run.
static gi_status start_run(gi_graph* g, unsigned long long delta, hipStream_t s) {
  HIP_TRY(hipStreamSynchronize(s));
  std::memset((void*)g->hflags, 0, offsetof(HostFlags, log));
  LAUNCH_TRY(launch_ctl_init(g->ctl, g->dflags, delta, s));
  return GI_OK;
}


// ---------------------------------------------------------- algorithms ----

static SelDev sel_dev(const gi_graph* g) {
  SelDev d;
  d.p = g->sel_p;
  d.wb = g->sel_wb;
  d.mu = g->sel_p ? g->sel_p + kParams : nullptr;
  d.isd = g->sel_p ? g->sel_p + kParams + kFeat : nullptr;
  d.lo = g->sel_p ? g->sel_p + kParams + 2 * kFeat : nullptr;
  d.hi = g->sel_p ? g->sel_p + kParams + 3 * kFeat : nullptr;
  return d;
}

static DecideArgs decide_args(const gi_graph* g, int alg) {
  DecideArgs d;
  d.part = g->part;
  d.ctl = g->ctl;
  d.direction = g->sched.direction;
  d.divisor = g->sched.hybrid_divisor;
  d.forced_dir = -1;
  d.edges = alg == ALG_CC ? 2 * g->m : g->m;
  d.is_bfs = alg == ALG_BFS;
  d.max_steps = 0;
  d.fc = alg == ALG_CC ? g->fc_cc : g->fc_bfs;
  d.sel = sel_dev(g);
  d.seg_pull = 0;
  return d;
}

static gi_status check_learned(const gi_graph* g) {
  if (g->sched.direction == GI_DIR_LEARNED && !g->sel_p)
    return fail(GI_ERR_INVALID_ARG, "learned direction without an attached selector");
  return GI_OK;
}

// Segment count used when the segmented schedule is chosen without one:
// contrib segments of at most 2 MiB (half of one XCD's L2).
static int auto_segments(const gi_graph* g) {
  const long long bytes = 4LL * g->n;
  return (int)std::max<long long>(2, (bytes + (2LL << 20) - 1) / (2LL << 20));
}

// The 12 selector features of a PageRank iteration (every vertex active).
static void pr_features(const gi_graph* g, float* x) {
  for (int i = 0; i < 5; ++i) x[i] = g->fc_pr.g[i];
  x[5] = 1.0f;
  x[6] = 1.0f;
  x[7] = 1.0f;
  x[8] = std::log2(1.0f + (float)g->n);
  x[9] = std::log2(1.0f + (float)g->m);
  x[10] = 1.0f;
  x[11] = g->fc_pr.alg;
}

// 20-iteration (or `iters`) DensePull PageRank, unsegmented or over the
// graph's segments.
// Launch shape of the ordered pull: threads, items per thread, LDS sources
// and workgroups.
struct PrOrdShape {
  int bt, u, hot, grid;
};

static gi_status pr_ord_shape(gi_graph* g, PrOrdShape* sh) {
  sh->bt = g->sched.block_threads > 0 ? g->sched.block_threads : 256;
  sh->u = g->sched.pull_items_per_thread > 0 ? g->sched.pull_items_per_thread : 8;
  if (!g->ncu) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&g->ncu, hipDeviceAttributeMultiprocessorCount, dev));
  }
  int maxlds = 0, dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // LDS of the kernel besides the hot sources: per wave, the tile's row
  // offsets, gathered contributions and FP64 row sums
  const long long fixed = 4LL * (sh->bt / 64) * (4LL * 64 * sh->u + 2);
  long long cap = ((long long)maxlds - fixed) / 4;
  // never more than the sources that are gathered at all (rounded up to 64),
  // nor past the end of the contribution array
  const long long useful = ((long long)g->ord_nsrc + 63) / 64 * 64;
  cap = std::min<long long>(cap, std::min<long long>(useful, (long long)g->n / 4 * 4));
  cap = std::max<long long>(0, cap / 64 * 64);
  long long hot = g->sched.pull_hot_sources;
  if (hot < 0) {
    // the most that one workgroup per CU leaves (LDS is per CU; the
    // workgroup's waves share the hot sources, so one large workgroup
    // beats several with smaller copies)
    hot = cap;
  }
  hot = std::min<long long>(std::max<long long>(0, hot) / 64 * 64, cap);
  sh->hot = (int)hot;
  const int per = pr_ord_occupancy(sh->hot, sh->bt, sh->u);
  if (per <= 0) return fail(GI_ERR_DEVICE, "occupancy query for the ordered PageRank pull failed");
  sh->grid = per * g->ncu;
  return GI_OK;
}

// DensePull PageRank over the degree-ordered in-adjacency (pr_order.hip).
namespace gi {
// Writes a run's results computed in the degree-ordered numbering back under
// the caller's ids (pagerank.hip): oa[old_id[r]] = ta[r] (when ta is set),
// ob[old_id[r]] = tb[r].
int launch_prec_remap(int n, const int32_t* old_id, const float* ta, float* oa, const float* tb,
                      float* ob, hipStream_t s);
}  // namespace gi

// The ordered run's launches: contributions from the ranks' initial value,
// then per iteration the pass and the split rows' finish (the last
// iteration writes the ranks).  With `events`, each iteration is bracketed
// by its step-timing events when step timing is on.  Returns nonzero on a
// launch error.
static int pr_ord_enqueue(gi_graph* g, const PrOrdArgs& a, const PrOrdShape& sh, int iters,
                          float* ranks, hipStream_t s, bool events) {
  if (launch_pr_init(g->n, g->ord_outdeg, g->contrib[0], ranks, iters == 0, s)) return -1;
  for (int k = 0; k < iters; ++k) {
    const bool last = k == iters - 1;
    const StepEvents* te = events ? step_events(g, k) : nullptr;
    if (te && (hipEventRecord(te->start, s) != hipSuccess ||
               hipEventRecord(te->main, s) != hipSuccess))
      return -1;
    if (launch_pr_ord(a, sh.bt, sh.u, sh.grid, g->contrib[k & 1], g->contrib[(k + 1) & 1],
                      last ? ranks : nullptr, s) ||
        launch_pr_ord_split(a, g->contrib[(k + 1) & 1], last ? ranks : nullptr, s))
      return -1;
    if (te && hipEventRecord(te->end, s) != hipSuccess) return -1;
  }
  return 0;
}

static void pr_drop_graph(gi_graph* g) {
  // a replay may still run on the graph's stream
  if (g->prg_exec && g->prg_stream) (void)hipStreamSynchronize(g->prg_stream);
  if (g->prg_exec) (void)hipGraphExecDestroy(g->prg_exec);
  if (g->prg_graph) (void)hipGraphDestroy(g->prg_graph);
  g->prg_exec = nullptr;
  g->prg_graph = nullptr;
}

// Captures the ordered run on the graph's own stream (a fill kernel and the
// passes only: no memset nodes) and instantiates it.
static gi_status pr_ord_capture(gi_graph* g, const PrOrdArgs& a, const PrOrdShape& sh, int iters,
                                float* ranks) {
  if (!g->prg_stream) {
    HIP_TRY(hipStreamCreateWithFlags(&g->prg_stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g->prg_evw, hipEventDisableTiming));
  }
  HIP_TRY(hipStreamBeginCapture(g->prg_stream, hipStreamCaptureModeThreadLocal));
  const int lr = pr_ord_enqueue(g, a, sh, iters, ranks, g->prg_stream, false);
  hipGraph_t gcap = nullptr;
  const hipError_t ce = hipStreamEndCapture(g->prg_stream, &gcap);
  if (lr != 0 || ce != hipSuccess) {
    if (gcap) (void)hipGraphDestroy(gcap);
    (void)hipGetLastError();
    return fail(GI_ERR_DEVICE, "PageRank graph capture failed");
  }
  g->prg_graph = gcap;
  if (hipGraphInstantiate(&g->prg_exec, g->prg_graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    pr_drop_graph(g);
    return fail(GI_ERR_DEVICE, "PageRank graph instantiation failed");
  }
  return GI_OK;
}

static gi_status pr_run_ordered(gi_graph* g, int32_t iters, float damping, float* ranks,
                                hipStream_t s) {
  gi_status st = ensure_pr_order(g);
  if (st != GI_OK) return st;
  PrOrdShape sh;
  if ((st = pr_ord_shape(g, &sh)) != GI_OK) return st;
  if ((st = ensure_pr_order_tiles(g, 64 * sh.u)) != GI_OK) return st;
  PrOrdArgs a{};
  a.off = g->ord_off;
  a.idx = g->ord_idx;
  a.tiles = g->ord_tiles;
  a.tslot = g->ord_tslot;
  a.srow = g->ord_srow;
  a.sacc = g->ord_sacc;
  a.nslots = g->ord_nslots;
  a.outdeg = g->ord_outdeg;
  a.old_id = g->ord_old;
  a.n = g->n;
  a.m = (int)g->m;
  a.ntiles = g->ord_ntiles;
  a.hot = sh.hot;
  a.alpha = (double)damping;
  a.base = (1.0 - (double)damping) / (double)g->n;
  const int launches = 1 + iters * (a.nslots > 0 ? 2 : 1);
  g->tev_count = 0;
  // a call that repeats the previous call's arguments replays the run as a
  // HIP graph (no per-step timing events in it); any other call runs the
  // launches directly and remembers its arguments
  gi_graph::PrGraphKey key;
  key.ranks = ranks;
  key.iters = iters;
  key.damping = damping;
  key.bt = sh.bt;
  key.u = sh.u;
  key.hot = sh.hot;
  key.grid = sh.grid;
  key.ntiles = a.ntiles;
  key.nslots = a.nslots;
  key.tiles = a.tiles;
  key.idx = a.idx;
  const bool replay = !g->step_timing && iters > 0 && key == g->prg_key;
  if (!(key == g->prg_key)) {
    pr_drop_graph(g);
    g->prg_key = key;
  }
  if (replay) {
    if (!g->prg_exec && (st = pr_ord_capture(g, a, sh, iters, ranks)) != GI_OK) return st;
    HIP_TRY(hipEventRecord(g->prg_evw, s));
    HIP_TRY(hipStreamWaitEvent(g->prg_stream, g->prg_evw, 0));
    HIP_TRY(hipEventRecord(g->ev[0], g->prg_stream));
    HIP_TRY(hipGraphLaunch(g->prg_exec, g->prg_stream));
    HIP_TRY(hipEventRecord(g->ev[1], g->prg_stream));
    HIP_TRY(hipStreamWaitEvent(s, g->ev[1], 0));  // the caller's later work follows the run
  } else {
    HIP_TRY(hipEventRecord(g->ev[0], s));
    LAUNCH_TRY(pr_ord_enqueue(g, a, sh, iters, ranks, s, true));
    HIP_TRY(hipEventRecord(g->ev[1], s));
  }
  if (g->timing_failed) return fail(GI_ERR_DEVICE, "PageRank: could not create timing events");
  // returns after enqueue: the run's time is read when it is asked for
  g->stats_pending = launches;
  g->last_stream = s;
  gi_run_stats& rs = g->stats;
  rs.algorithm = ALG_PR;
  rs.steps = iters;
  rs.dense_steps = iters;
  rs.edges_examined = (int64_t)iters * g->m;
  rs.trace_len = std::min(iters, GI_MAX_TRACE);
  for (int k = 0; k < rs.trace_len; ++k) {
    rs.step_direction[k] = GI_DIR_DENSE_PULL;
    rs.step_segmented[k] = 0;
    rs.step_frontier[k] = g->n;
    rs.step_degree_sum[k] = g->m;
    rs.step_edges[k] = g->m;
  }
  return GI_OK;
}

static gi_status pr_run(gi_graph* g, int32_t iters, float damping, float* ranks, hipStream_t s,
                        bool segmented) {
  PrVertex pv;
  pv.outdeg = g->outdeg;
  pv.alpha = (double)damping;
  pv.base = (1.0 - (double)damping) / (double)g->n;
  const int bt = g->sched.block_threads > 0 ? g->sched.block_threads : 256;
  int launches = 1;
  HIP_TRY(hipEventRecord(g->ev[0], s));
  LAUNCH_TRY(launch_pr_init(g->n, g->outdeg, g->contrib[0], ranks, iters == 0, s));
  g->tev_count = 0;
  for (int k = 0; k < iters; ++k) {
    const bool last = k == iters - 1;
    float* cin = g->contrib[k & 1];
    float* cout = g->contrib[(k + 1) & 1];
    const StepEvents* te = step_events(g, k);
    if (te) {
      HIP_TRY(hipEventRecord(te->start, s));
      HIP_TRY(hipEventRecord(te->main, s));
    }
    if (!segmented) {
      PrRows r{g->pr_table, g->pr_ntab, g->in_off, g->in_idx, nullptr, g->lr_acc, g->lr_cnt,
               g->lr_chunks};
      LAUNCH_TRY(launch_pr_rows(r, g->pr_cap_e, g->pr_cap_v, bt, 0, cin, 0, pv, cout,
                                last ? ranks : nullptr, nullptr, s));
      ++launches;
    } else if (g->sched.segments_concurrent && g->segs.size() > 1) {
      const int p = (int)g->segs.size();
      LAUNCH_TRY(launch_pr_seg_concurrent(g->seg_rows, p, g->pr_cap_e, g->pr_cap_v, bt, cin, pv,
                                          g->pr_acc, g->n, s));
      LAUNCH_TRY(launch_pr_seg_final_multi(g->n, p, pv, g->pr_acc, cout, last ? ranks : nullptr,
                                           s));
      launches += 2;
    } else {
      for (const SegDev& sg : g->segs) {
        PrRows r{sg.table, sg.ntab, sg.off, sg.idx, sg.dst, nullptr, nullptr, nullptr};
        LAUNCH_TRY(launch_pr_rows(r, g->pr_cap_e, g->pr_cap_v, bt, 0, cin, 1, pv, nullptr,
                                  nullptr, g->pr_acc, s));
        ++launches;
      }
      LAUNCH_TRY(launch_pr_seg_final(g->n, pv, g->pr_acc, cout, last ? ranks : nullptr, s));
      ++launches;
    }
    if (te) HIP_TRY(hipEventRecord(te->end, s));
  }
  HIP_TRY(hipEventRecord(g->ev[1], s));
  if (g->timing_failed) return fail(GI_ERR_DEVICE, "PageRank: could not create timing events");
  // returns after enqueue: the run's time is read when it is asked for
  g->stats_pending = launches;
  g->last_stream = s;
  gi_run_stats& st = g->stats;
  st.algorithm = ALG_PR;
  st.steps = iters;
  st.dense_steps = iters;
  st.edges_examined = (int64_t)iters * g->m;
  st.trace_len = std::min(iters, GI_MAX_TRACE);
  for (int k = 0; k < st.trace_len; ++k) {
    st.step_direction[k] = GI_DIR_DENSE_PULL;
    st.step_segmented[k] = segmented ? 1 : 0;
    st.step_frontier[k] = g->n;
    st.step_degree_sum[k] = g->m;
    st.step_edges[k] = g->m;
  }
  return GI_OK;
}

// The automatic segments (2 MiB of contributions each) for a segmented
// choice when the schedule itself has one segment; rebuilt when the graph
// holds segments of another count from an earlier schedule.
static gi_status ensure_segments(gi_graph* g) {
  return ensure_pr_segments(g, auto_segments(g), GI_SEG_FIXED_VERTEX_COUNT);
}

extern "C" gi_status gi_pagerank(gi_graph* g, int32_t iters, float damping, float* ranks,
                                 void* stream) {
  if (!g || !ranks) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (iters < 0) return fail(GI_ERR_INVALID_ARG, "iters must be >= 0");
  if (!(damping >= 0.0f && damping <= 1.0f)) return fail(GI_ERR_INVALID_ARG, "damping outside [0,1]");
  gi_status st = check_learned(g);
  if (st != GI_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool segmented = g->sched.num_segments > 1;
  if (segmented && g->sched.direction != GI_DIR_LEARNED &&
      (st = ensure_pr_segments(g, g->sched.num_segments, g->sched.segment_strategy)) != GI_OK)
    return st;
  if (g->sched.direction == GI_DIR_LEARNED) {
    // one inference for the whole run: every iteration meets the same state
    float io[kFeat + kOut];
    pr_features(g, io);
    HIP_TRY(hipMemcpyAsync(g->sel_io, io, sizeof(float) * kFeat, hipMemcpyHostToDevice, s));
    LAUNCH_TRY(launch_mlp_predict(sel_dev(g), g->sel_io, 1, true, g->sel_io + kFeat, s));
    HIP_TRY(hipMemcpyAsync(io + kFeat, g->sel_io + kFeat, sizeof(float) * kOut,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    segmented = io[kFeat + 2] - io[kFeat + 3] > kLearnedMargin;
    // the choice is the direction; the layout is the schedule's: its
    // segments for the segmented pull (else the automatic count), its
    // vertex order for the unsegmented one
    if (segmented) {
      st = g->sched.num_segments > 1
               ? ensure_pr_segments(g, g->sched.num_segments, g->sched.segment_strategy)
               : ensure_segments(g);
      if (st != GI_OK) return st;
    } else if (g->sched.vertex_order == GI_ORDER_OUT_DEGREE) {
      return pr_run_ordered(g, iters, damping, ranks, s);
    }
  }
  if (g->sched.vertex_order == GI_ORDER_OUT_DEGREE && g->sched.direction != GI_DIR_LEARNED)
    return pr_run_ordered(g, iters, damping, ranks, s);
  return pr_run(g, iters, damping, ranks, s, segmented);
}


extern "C" gi_status gi_bfs(gi_graph* g, int32_t src, int32_t* level, int32_t* parent, void* stream) {
  if (!g || !level) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (src < 0 || src >= g->n) return fail(GI_ERR_INVALID_ARG, "source %d outside [0, %d)", src, g->n);
  hipStream_t s = static_cast<hipStream_t>(stream);
  gi_status st = check_learned(g);
  if (st != GI_OK) return st;
  const int dir = g->sched.direction;
  if (dir == GI_DIR_DENSE_PULL || dir == GI_DIR_DENSE_PULL_SPARSE_PUSH || dir == GI_DIR_LEARNED) {
    st = ensure_bfs_rows(g);
    if (st != GI_OK) return st;
  }
  st = start_run(g, 0, s);
  if (st != GI_OK) return st;
  BfsArgs b;
  b.g = dev_graph(g);
  b.level = level;
  b.parent = parent;
  b.cur = frontier_set(g, 0);
  b.next = frontier_set(g, 1);
  b.vis = g->vis;
  b.part = g->part;
  b.ctl = g->ctl;
  LAUNCH_TRY(launch_bfs_init(b, src, frontier_set(g, 0), frontier_set(g, 1), s));
  const DecideArgs d = decide_args(g, ALG_BFS);
  st = run_frontier_loop(
      g, s, ALG_BFS, 8, (long long)g->n + 2,
      [&](long long k) {
        BfsArgs bk = b;
        bk.cur = frontier_set(g, (int)(k & 1));
        bk.next = frontier_set(g, (int)((k + 1) & 1));
        const FrontierArgs f = frontier_args(g->eng, bk.cur, bk.next, g->outdeg, nullptr, nullptr);
        return enqueue_bfs_step(g->eng, f, d, bk, step_events(g, k), s) ? -1 : 4;
      },
      "BFS");
  if (st != GI_OK) return st;
  return read_loop_stats(g, ALG_BFS);
}

// Whether CC reads the CSR and CSC rows directly (no symmetric copy).
static bool cc_direct(const gi_graph* g) {
  if (g->sched.cc_adjacency == GI_CC_ADJ_DIRECT) return true;
  if (g->sched.cc_adjacency == GI_CC_ADJ_SYMMETRIC) return false;
  return 2 * g->m > (int64_t)INT32_MAX;
}

// Destination blocks of the CSR and CSC rows for the direct CC pull, built
// on first use.
static gi_status ensure_cc_direct(gi_graph* g) {
  if (g->ccd_out_table) return GI_OK;
  std::vector<int32_t> out_off((size_t)g->n + 1, 0);
  for (size_t v = 0; v < (size_t)g->n; ++v) out_off[v + 1] = out_off[v] + g->h_outdeg[v];
  std::vector<int4> to = make_cc_table(out_off.data(), g->n, kCcCapE, kCcCapV);
  std::vector<int4> ti = make_cc_table(g->h_in_off.data(), g->n, kCcCapE, kCcCapV);
  gi_status st;
  int4 *dto = nullptr, *dti = nullptr;
  if ((st = dev_alloc(g, g->allocs, &dto, std::max<size_t>(1, to.size()))) != GI_OK) return st;
  if ((st = dev_alloc(g, g->allocs, &dti, std::max<size_t>(1, ti.size()))) != GI_OK) return st;
  if (!to.empty() && (st = upload(to.data(), dto, to.size() * sizeof(int4))) != GI_OK) return st;
  if (!ti.empty() && (st = upload(ti.data(), dti, ti.size() * sizeof(int4))) != GI_OK) return st;
  g->ccd_out_table = dto;
  g->ccd_in_table = dti;
  g->ccd_out_ntab = (int)to.size();
  g->ccd_in_ntab = (int)ti.size();
  return GI_OK;
}

// Symmetric adjacency for CC, built on the device on first use.
static gi_status ensure_sym(gi_graph* g, hipStream_t s) {
  if (g->sym_idx) return GI_OK;
  const size_t N = (size_t)g->n;
  // 2m entries under int32 offsets: larger graphs take the direct form
  if (2 * g->m > (int64_t)INT32_MAX)
    return fail(GI_ERR_OVERFLOW,
                "the symmetric adjacency (2m = %lld entries) exceeds 32-bit offsets; "
                "schedule cc_adjacency AUTO or DIRECT reads the rows directly",
                (long long)(2 * g->m));
  std::vector<int32_t> off(N + 1, 0);
  for (size_t v = 0; v < N; ++v)
    off[v + 1] = off[v] + g->h_outdeg[v] + (g->h_in_off[v + 1] - g->h_in_off[v]);
  std::vector<int4> tab = make_cc_table(off.data(), g->n, kCcCapE, kCcCapV);
  gi_status st;
  if ((st = dev_alloc(g, g->allocs, &g->sym_off, N + 1)) != GI_OK) return st;
  if ((st = dev_alloc(g, g->allocs, &g->sym_idx, (size_t)off[N])) != GI_OK) return st;
  if ((st = dev_alloc(g, g->allocs, &g->sym_table, tab.size())) != GI_OK) return st;
  if ((st = upload(off.data(), g->sym_off, 4 * (N + 1))) != GI_OK) return st;
  if ((st = upload(tab.data(), g->sym_table, tab.size() * sizeof(int4))) != GI_OK) return st;
  g->sym_ntab = (int)tab.size();
  LAUNCH_TRY(launch_build_sym(dev_graph(g), g->sym_off, g->sym_idx, s));
  HIP_TRY(hipStreamSynchronize(s));
  return GI_OK;
}

// Source segments for the segmented CC pull (configApplyNumSSG applied to
// CC): p ranges of equal vertex count, or of equal out+in degree sums
// (edge-aware); segment x keeps, for every vertex with a neighbour (out- or
// in-) in range x, those neighbours, out-row first.  Built on first use on
// the host from the CSR and CSC rows, so it needs no symmetric copy; each
// segment's entries must fit 32-bit offsets.
static gi_status ensure_cc_segments(gi_graph* g, int p, int strategy, hipStream_t s) {
  if (g->ccsegs && g->ccseg_p == p && g->ccseg_strategy == strategy) return GI_OK;
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipDeviceSynchronize());
  free_list(g->ccseg_allocs);
  g->ccsegs = nullptr;
  g->cc_segmin = nullptr;
  g->ccseg_p = 0;
  const int32_t n = g->n;
  const size_t N = (size_t)n;
  const int32_t* ooff = g->h_out_off.data();
  const int32_t* ioff = g->h_in_off.data();
  const int32_t* iidx = g->h_in_idx.data();
  std::vector<int32_t> oidx((size_t)g->m);
  if (!oidx.empty())
    HIP_TRY(hipMemcpy(oidx.data(), g->out_idx, 4 * oidx.size(), hipMemcpyDeviceToHost));
  auto udeg = [&](size_t v) -> int64_t {
    return (int64_t)(ooff[v + 1] - ooff[v]) + (int64_t)(ioff[v + 1] - ioff[v]);
  };
  // segment of each vertex
  std::vector<int32_t> segof(N);
  {
    const int64_t total = 2 * g->m;
    int64_t acc = 0;
    int x = 0;
    const int64_t per = ((int64_t)n + p - 1) / p;
    for (int32_t v = 0; v < n; ++v) {
      if (strategy == GI_SEG_FIXED_VERTEX_COUNT) {
        x = (int)(v / per);
      } else {
        while (x < p - 1 && acc * p >= total * (x + 1)) ++x;
        acc += udeg((size_t)v);
      }
      segof[(size_t)v] = x;
    }
  }
  std::vector<std::vector<int32_t>> soff((size_t)p, std::vector<int32_t>(1, 0)), sidx((size_t)p),
      sdst((size_t)p);
  std::vector<int32_t> cnt((size_t)p, 0), touched;
  for (int32_t v = 0; v < n; ++v) {
    const int32_t ob = ooff[v], oe = ooff[v + 1], ib = ioff[v], ie = ioff[v + 1];
    if (ob == oe && ib == ie) continue;
    touched.clear();
    auto count = [&](int32_t u) {
      const int32_t x = segof[(size_t)u];
      if (cnt[(size_t)x]++ == 0) touched.push_back(x);
    };
    for (int32_t j = ob; j < oe; ++j) count(oidx[(size_t)j]);
    for (int32_t j = ib; j < ie; ++j) count(iidx[(size_t)j]);
    std::sort(touched.begin(), touched.end());
    for (int32_t x : touched) {
      std::vector<int32_t>& so = soff[(size_t)x];
      if ((int64_t)so.back() + cnt[(size_t)x] > (int64_t)INT32_MAX)
        return fail(GI_ERR_OVERFLOW, "CC segment %d exceeds 2^31-1 entries; use more segments", x);
      sdst[(size_t)x].push_back(v);
      so.push_back(so.back() + cnt[(size_t)x]);
      cnt[(size_t)x] = 0;
    }
    for (int32_t j = ob; j < oe; ++j) {
      const int32_t u = oidx[(size_t)j];
      sidx[(size_t)segof[(size_t)u]].push_back(u);
    }
    for (int32_t j = ib; j < ie; ++j) {
      const int32_t u = iidx[(size_t)j];
      sidx[(size_t)segof[(size_t)u]].push_back(u);
    }
  }
  std::vector<int32_t>().swap(oidx);
  std::vector<CcSeg> hs((size_t)p);
  gi_status st;
  for (int x = 0; x < p; ++x) {
    std::vector<int4> tab = make_cc_table(soff[(size_t)x].data(), (int)sdst[(size_t)x].size(),
                                          kCcCapE, kCcCapV);
    int32_t *doff = nullptr, *didx = nullptr, *ddst = nullptr;
    int4* dtab = nullptr;
    if ((st = dev_alloc(g, g->ccseg_allocs, &doff, soff[(size_t)x].size())) != GI_OK) return st;
    if ((st = dev_alloc(g, g->ccseg_allocs, &didx, std::max<size_t>(1, sidx[(size_t)x].size()))) != GI_OK) return st;
    if ((st = dev_alloc(g, g->ccseg_allocs, &ddst, std::max<size_t>(1, sdst[(size_t)x].size()))) != GI_OK) return st;
    if ((st = dev_alloc(g, g->ccseg_allocs, &dtab, std::max<size_t>(1, tab.size()))) != GI_OK) return st;
    if ((st = upload(soff[(size_t)x].data(), doff, 4 * soff[(size_t)x].size())) != GI_OK) return st;
    if (!sidx[(size_t)x].empty() &&
        (st = upload(sidx[(size_t)x].data(), didx, 4 * sidx[(size_t)x].size())) != GI_OK)
      return st;
    if (!sdst[(size_t)x].empty() &&
        (st = upload(sdst[(size_t)x].data(), ddst, 4 * sdst[(size_t)x].size())) != GI_OK)
      return st;
    if (!tab.empty() && (st = upload(tab.data(), dtab, sizeof(int4) * tab.size())) != GI_OK)
      return st;
    hs[(size_t)x] = CcSeg{RowBlocks{dtab, (int)tab.size(), doff, didx}, ddst};
  }
  if ((st = dev_alloc(g, g->ccseg_allocs, &g->ccsegs, (size_t)p)) != GI_OK) return st;
  if ((st = upload(hs.data(), g->ccsegs, sizeof(CcSeg) * (size_t)p)) != GI_OK) return st;
  if ((st = dev_alloc(g, g->ccseg_allocs, &g->cc_segmin, (size_t)p * N)) != GI_OK) return st;
  HIP_TRY(hipMemset(g->cc_segmin, 0xff, sizeof(uint32_t) * (size_t)p * N));
  g->ccseg_p = p;
  g->ccseg_strategy = strategy;
  return GI_OK;
}

extern "C" gi_status gi_cc(gi_graph* g, int32_t* label, void* stream) {
  if (!g || !label) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  gi_status st = check_learned(g);
  if (st != GI_OK) return st;
  const bool direct = cc_direct(g);
  st = direct ? ensure_cc_direct(g) : ensure_sym(g, s);
  if (st != GI_OK) return st;
  // segments: the schedule's; the learned choice's S3 pulls over them too,
  // or over the automatic count (2 MiB of labels each) when the schedule
  // has none
  const bool learned = g->sched.direction == GI_DIR_LEARNED;
  int seg_pull = 0;
  if (learned) {
    const bool own = g->sched.num_segments > 1;
    if ((st = ensure_cc_segments(g, own ? std::min(g->sched.num_segments, kParts) : auto_segments(g),
                                 own ? g->sched.segment_strategy : GI_SEG_FIXED_VERTEX_COUNT, s)) !=
        GI_OK)
      return st;
    seg_pull = 2;
  } else if (g->sched.num_segments > 1) {
    // every segment needs at least one of the step kernel's kParts workgroups
    const int p = std::min(g->sched.num_segments, kParts);
    if ((st = ensure_cc_segments(g, p, g->sched.segment_strategy, s)) != GI_OK) return st;
    seg_pull = 1;
  }
  if ((st = start_run(g, 0, s)) != GI_OK) return st;
  int32_t* labs[2] = {label, g->lab};
  CcArgs c;
  c.g = dev_graph(g);
  c.cur = labs[0];
  c.nxt = labs[1];
  c.fr = frontier_set(g, 0);
  c.next = frontier_set(g, 1);
  c.direct = direct ? 1 : 0;
  if (direct) {
    c.sym_off = nullptr;
    c.sym_idx = nullptr;
    c.rows = RowBlocks{g->ccd_out_table, g->ccd_out_ntab, g->out_off, g->out_idx};
    c.rows_in = RowBlocks{g->ccd_in_table, g->ccd_in_ntab, g->in_off, g->in_idx};
  } else {
    c.sym_off = g->sym_off;
    c.sym_idx = g->sym_idx;
    c.rows = RowBlocks{g->sym_table, g->sym_ntab, g->sym_off, g->sym_idx};
    c.rows_in = RowBlocks{nullptr, 0, nullptr, nullptr};
  }
  c.segs = nullptr;
  c.nseg = 1;
  c.seg_min = nullptr;
  if (seg_pull) {
    c.segs = g->ccsegs;
    c.nseg = g->ccseg_p;
    c.seg_min = g->cc_segmin;
  }
  c.part = g->part;
  c.ctl = g->ctl;
  LAUNCH_TRY(launch_cc_init(c, frontier_set(g, 0), frontier_set(g, 1), labs[1], s));
  DecideArgs d = decide_args(g, ALG_CC);
  d.seg_pull = seg_pull;
  st = run_frontier_loop(
      g, s, ALG_CC, 8, (long long)g->n + 2,
      [&](long long k) {
        CcArgs ck = c;
        ck.cur = labs[k & 1];
        ck.nxt = labs[(k + 1) & 1];
        ck.fr = frontier_set(g, (int)(k & 1));
        ck.next = frontier_set(g, (int)((k + 1) & 1));
        const FrontierArgs f = frontier_args(g->eng, ck.fr, ck.next, g->udeg, ck.cur, ck.nxt);
        return enqueue_cc_step(g->eng, f, d, ck, step_events(g, k), s) ? -1 : 4;
      },
      "CC");
  if (st != GI_OK) return st;
  st = read_loop_stats(g, ALG_CC);
  if (st != GI_OK) return st;
  // after `steps` rounds the labels sit in labs[steps & 1]
  if (g->stats.steps & 1) {
    HIP_TRY(hipMemcpyAsync(label, g->lab, 4 * (size_t)g->n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return GI_OK;
}

extern "C" gi_status gi_sssp(gi_graph* g, int32_t src, uint32_t* dist, void* stream) {
  if (!g || !dist) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (!g->weighted) return fail(GI_ERR_INVALID_ARG, "graph has no edge weights");
  if (src < 0 || src >= g->n) return fail(GI_ERR_INVALID_ARG, "source %d outside [0, %d)", src, g->n);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned long long delta = g->sched.sssp_delta > 0 ? g->sched.sssp_delta : 512u;
  gi_status st = start_run(g, delta, s);
  if (st != GI_OK) return st;
  SsspArgs a;
  a.g = dev_graph(g);
  a.dist = dist;
  a.cur = DenseSet{g->fbv[0], nullptr};
  a.next = DenseSet{g->fbv[1], nullptr};
  a.far = DenseSet{g->far, nullptr};
  a.delta = delta;
  a.fmin = g->fmin;
  a.part = g->part;
  a.ctl = g->ctl;
  LAUNCH_TRY(launch_sssp_init(a, src, s));
  st = run_frontier_loop(
      g, s, ALG_SSSP, 64, 64LL * g->n + 1024,
      [&](long long k) {
        SsspArgs ak = a;
        ak.cur = DenseSet{g->fbv[k & 1], nullptr};
        ak.next = DenseSet{g->fbv[(k + 1) & 1], nullptr};
        const FrontierArgs f = frontier_args(g->eng, ak.cur, ak.next, g->outdeg, nullptr, nullptr);
        return enqueue_sssp_step(g->eng, f, ak, step_events(g, k), s) ? -1 : 5;
      },
      "SSSP");
  if (st != GI_OK) return st;
  if (((const volatile HostFlags*)g->hflags)->overflow) return fail(GI_ERR_OVERFLOW, "a distance reached UINT32_MAX");
  st = read_loop_stats(g, ALG_SSSP);
  g->stats.dense_steps = 0;
  return st;
}

extern "C" gi_status gi_prdelta(gi_graph* g, int32_t rounds, double damping, double epsilon,
                                double* ranks, void* stream) {
  if (!g || !ranks) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (rounds < 0) return fail(GI_ERR_INVALID_ARG, "rounds must be >= 0");
  if (!(damping >= 0.0 && damping <= 1.0)) return fail(GI_ERR_INVALID_ARG, "damping outside [0,1]");
  if (!(epsilon >= 0.0) || !std::isfinite(epsilon))
    return fail(GI_ERR_INVALID_ARG, "epsilon must be finite and >= 0");
  if (g->sched.direction == GI_DIR_LEARNED)
    return fail(GI_ERR_UNSUPPORTED, "PageRankDelta has no learned direction");
  hipStream_t s = static_cast<hipStream_t>(stream);
  gi_status st;
  if (!g->prd && (st = dev_alloc(g, g->allocs, &g->prd, 3 * (size_t)g->n)) != GI_OK) return st;
  if ((st = start_run(g, 0, s)) != GI_OK) return st;
  PrdArgs a;
  a.g = dev_graph(g);
  a.delta = g->prd;
  a.contrib = g->prd + g->n;
  a.dsum = g->prd + 2 * (size_t)g->n;
  a.rank = ranks;
  a.cur = DenseSet{g->fbv[0], nullptr};
  a.next = DenseSet{g->fbv[1], nullptr};
  a.rows = PrRows{g->pr_table, g->pr_ntab, g->in_off, g->in_idx, nullptr, g->lr_acc, g->lr_cnt,
                  g->lr_chunks};
  a.cap_e = g->pr_cap_e;
  a.alpha = damping;
  a.base = (1.0 - damping) / (double)g->n;
  a.inv_n = 1.0 / (double)g->n;
  a.eps = epsilon;
  a.part = g->part;
  a.ctl = g->ctl;
  LAUNCH_TRY(launch_prd_init(a, s));
  if (rounds == 0) {
    HIP_TRY(hipStreamSynchronize(s));
    g->stats = gi_run_stats{};
    g->stats.algorithm = ALG_PRD;
    return GI_OK;
  }
  DecideArgs d = decide_args(g, ALG_BFS);
  d.is_bfs = 0;
  d.fc = g->fc_pr;
  d.max_steps = rounds;
  st = run_frontier_loop(
      g, s, ALG_PRD, 8, (long long)rounds + 2,
      [&](long long k) {
        PrdArgs ak = a;
        ak.cur = DenseSet{g->fbv[k & 1], nullptr};
        ak.next = DenseSet{g->fbv[(k + 1) & 1], nullptr};
        const FrontierArgs f = frontier_args(g->eng, ak.cur, ak.next, g->outdeg, nullptr, nullptr);
        return enqueue_prd_step(g->eng, f, d, ak, step_events(g, k), s) ? -1 : 5;
      },
      "PageRankDelta");
  if (st != GI_OK) return st;
  return read_loop_stats(g, ALG_PRD);
}

extern "C" gi_status gi_bc(gi_graph* g, int32_t src, double* dependency, double* sigma,
                           void* stream) {
  if (!g || !dependency) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (src < 0 || src >= g->n) return fail(GI_ERR_INVALID_ARG, "source %d outside [0, %d)", src, g->n);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t N = (size_t)g->n;
  // sigma, fs, bw double[n]; bounds u64[n + 2]; level, order int32[n]
  const size_t bytes = 8 * 3 * N + 8 * (N + 2) + 4 * 2 * N;
  gi_status st;
  if (!g->bc) {
    uint8_t* p = nullptr;
    if ((st = dev_alloc(g, g->allocs, &p, bytes)) != GI_OK) return st;
    g->bc = p;
    std::vector<int4> tab = make_cc_table(g->h_in_off.data(), g->n, kCcCapE, kCcCapV);
    if ((st = dev_alloc(g, g->allocs, &g->bc_tab, std::max<size_t>(1, tab.size()))) != GI_OK)
      return st;
    if (!tab.empty() && (st = upload(tab.data(), g->bc_tab, tab.size() * sizeof(int4))) != GI_OK)
      return st;
    g->bc_ntab = (int)tab.size();
  }
  uint8_t* base = static_cast<uint8_t*>(g->bc);
  BcArgs a;
  a.g = dev_graph(g);
  a.src = src;
  a.sigma = reinterpret_cast<double*>(base);
  a.fs = reinterpret_cast<double*>(base + 8 * N);
  a.bw = reinterpret_cast<double*>(base + 16 * N);
  a.bounds = reinterpret_cast<unsigned long long*>(base + 24 * N);
  a.level = reinterpret_cast<int32_t*>(base + 24 * N + 8 * (N + 2));
  a.order = reinterpret_cast<int32_t*>(base + 28 * N + 8 * (N + 2));
  if (sigma) a.sigma = sigma;
  a.delta = dependency;
  a.in_rows = RowBlocks{g->bc_tab, g->bc_ntab, g->in_off, g->in_idx};
  a.divisor = g->sched.hybrid_divisor;
  a.ctl = g->ctl;
  if ((st = start_run(g, 0, s)) != GI_OK) return st;
  LAUNCH_TRY(launch_bc_init(a, s));
  st = run_frontier_loop(
      g, s, ALG_BC, 8, (long long)g->n + 2,
      [&](long long k) { return enqueue_bc_forward(a, step_events(g, k), s) ? -1 : 4; },
      "betweenness");
  if (st != GI_OK) return st;
  if ((st = read_loop_stats(g, ALG_BC)) != GI_OK) return st;
  const int levels = ((const volatile HostFlags*)g->hflags)->steps;
  std::vector<unsigned long long> bd((size_t)levels + 1);
  HIP_TRY(hipMemcpy(bd.data(), a.bounds, 8 * bd.size(), hipMemcpyDeviceToHost));
  // deepest level first: each level's dependencies come from the next one's
  for (int L = levels - 1; L >= 0; --L)
    LAUNCH_TRY(enqueue_bc_backward_level(a, (long long)bd[(size_t)L], (long long)bd[(size_t)L + 1],
                                         L, s));
  HIP_TRY(hipStreamSynchronize(s));
  return GI_OK;
}

extern "C" gi_status gi_pagerank_eigenvector(gi_graph* g, int32_t iters, float damping,
                                             float* ranks, float* eigen, int32_t fused,
                                             void* stream) {
  if (!g || !ranks || !eigen) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (iters < 0) return fail(GI_ERR_INVALID_ARG, "iters must be >= 0");
  if (!(damping >= 0.0f && damping <= 1.0f)) return fail(GI_ERR_INVALID_ARG, "damping outside [0,1]");
  if (fused != 0 && fused != 1) return fail(GI_ERR_INVALID_ARG, "fused must be 0 or 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t N = (size_t)g->n;
  gi_status st;
  if (!g->prec_tab) {
    std::vector<int32_t> lrow;
    std::vector<int4> tab = make_prec_table(g->h_in_off.data(), g->n, kPrEcCapE, kPrEcCapV, &lrow);
    g->prec_nlong = (int)lrow.size();
    if ((st = dev_alloc(g, g->allocs, &g->prec_lrow, std::max<size_t>(1, lrow.size()))) != GI_OK) return st;
    if ((st = dev_alloc(g, g->allocs, &g->prec_lacc, 2 * std::max<size_t>(1, lrow.size()))) != GI_OK) return st;
    if (!lrow.empty() &&
        (st = upload(lrow.data(), g->prec_lrow, lrow.size() * sizeof(int32_t))) != GI_OK)
      return st;
    HIP_TRY(hipMemset(g->prec_lacc, 0, sizeof(double) * 2 * std::max<size_t>(1, lrow.size())));
    if ((st = dev_alloc(g, g->allocs, &g->prec_tab, tab.size())) != GI_OK) return st;
    if ((st = upload(tab.data(), g->prec_tab, tab.size() * sizeof(int4))) != GI_OK) return st;
    g->prec_ntab = (int)tab.size();
    if ((st = dev_alloc(g, g->allocs, &g->prec_aos, 2 * N)) != GI_OK) return st;
    if ((st = dev_alloc(g, g->allocs, &g->prec_y, 2 * N)) != GI_OK) return st;
  }
  if (g->prec_norm_cap < iters + 1) {
    const int cap = std::max(iters + 1, 64);
    if ((st = dev_alloc(g, g->allocs, &g->prec_norm, (size_t)cap)) != GI_OK) return st;
    g->prec_norm_cap = cap;
  }
  // the fused pass over the degree-ordered in-adjacency (vertex_order =
  // GI_ORDER_OUT_DEGREE): the same kernel over the ordered rows, pairs and
  // out-degrees in the new numbering, results returned to the caller's ids
  const bool ordered = fused && g->sched.vertex_order == GI_ORDER_OUT_DEGREE;
  if (ordered) {
    if ((st = ensure_pr_order(g)) != GI_OK) return st;
    if (!g->preco_tab) {
      std::vector<int32_t> lrow;
      std::vector<int4> tab =
          make_prec_table(g->h_ord_off.data(), g->n, kPrEcCapE, kPrEcCapV, &lrow);
      const size_t nl = std::max<size_t>(1, lrow.size());
      int32_t* d_lrow = nullptr;
      double* d_lacc = nullptr;
      int4* d_tab = nullptr;
      float* d_tmp = nullptr;
      if ((st = dev_alloc(g, g->ord_allocs, &d_lrow, nl)) != GI_OK ||
          (st = dev_alloc(g, g->ord_allocs, &d_lacc, 2 * nl)) != GI_OK ||
          (st = dev_alloc(g, g->ord_allocs, &d_tab, std::max<size_t>(1, tab.size()))) != GI_OK ||
          (st = dev_alloc(g, g->ord_allocs, &d_tmp, 2 * N)) != GI_OK)
        return st;
      if (!lrow.empty() && (st = upload(lrow.data(), d_lrow, lrow.size() * sizeof(int32_t))) != GI_OK)
        return st;
      HIP_TRY(hipMemset(d_lacc, 0, sizeof(double) * 2 * nl));
      if (!tab.empty() && (st = upload(tab.data(), d_tab, tab.size() * sizeof(int4))) != GI_OK)
        return st;
      g->preco_lrow = d_lrow;
      g->preco_lacc = d_lacc;
      g->preco_tmp = d_tmp;
      g->preco_nlong = (int)lrow.size();
      g->preco_ntab = (int)tab.size();
      g->preco_tab = d_tab;
    }
  }
  const int32_t* outdeg = ordered ? g->ord_outdeg : g->outdeg;
  PrVertex pv;
  pv.outdeg = outdeg;
  pv.alpha = (double)damping;
  pv.base = (1.0 - (double)damping) / (double)g->n;
  PrEcArgs a;
  if (ordered) {
    a.rb = RowBlocks{g->preco_tab, g->preco_ntab, g->ord_off, g->ord_idx};
    a.lacc = g->preco_lacc;
    a.lrow = g->preco_lrow;
    a.nlong = g->preco_nlong;
  } else {
    a.rb = RowBlocks{g->prec_tab, g->prec_ntab, g->in_off, g->in_idx};
    a.lacc = g->prec_lacc;
    a.lrow = g->prec_lrow;
    a.nlong = g->prec_nlong;
  }
  a.pv = pv;
  float* ranks_out = ordered ? g->preco_tmp : ranks;  // last iteration's ranks
  float* eigen_out = ordered ? g->preco_tmp + N : eigen;
  int launches = 0;
  HIP_TRY(hipEventRecord(g->ev[0], s));
  if (fused) {
    LAUNCH_TRY(launch_prec_init(g->n, outdeg, g->prec_aos, nullptr, g->prec_norm, iters + 1, s));
  } else {
    LAUNCH_TRY(launch_pr_init(g->n, g->outdeg, g->contrib[0], ranks, iters == 0, s));
    LAUNCH_TRY(launch_prec_init(g->n, g->outdeg, nullptr, g->prec_y, g->prec_norm, iters + 1, s));
    ++launches;
  }
  ++launches;
  if (fused && iters == 0) LAUNCH_TRY(launch_pr_init(g->n, g->outdeg, g->contrib[0], ranks, true, s));
  g->tev_count = 0;
  const int bt = g->sched.block_threads > 0 ? g->sched.block_threads : 256;
  for (int k = 0; k < iters; ++k) {
    const bool last = k == iters - 1;
    const StepEvents* te = step_events(g, k);
    if (te) {
      HIP_TRY(hipEventRecord(te->start, s));
      HIP_TRY(hipEventRecord(te->main, s));
    }
    a.norm2_prev = g->prec_norm + k;
    a.norm2_next = g->prec_norm + k + 1;
    if (fused) {
      a.aos_in = g->prec_aos + (k & 1) * N;
      a.aos_out = g->prec_aos + ((k + 1) & 1) * N;
      a.ranks = last ? ranks_out : nullptr;
      LAUNCH_TRY(launch_prec_rows(a, true, s));
      launches += a.nlong > 0 ? 2 : 1;
    } else {
      PrRows r{g->pr_table, g->pr_ntab, g->in_off, g->in_idx, nullptr, g->lr_acc, g->lr_cnt,
               g->lr_chunks};
      LAUNCH_TRY(launch_pr_rows(r, g->pr_cap_e, g->pr_cap_v, bt, 0, g->contrib[k & 1], 0, pv,
                                g->contrib[(k + 1) & 1], last ? ranks : nullptr, nullptr, s));
      a.y_in = g->prec_y + (k & 1) * N;
      a.y_out = g->prec_y + ((k + 1) & 1) * N;
      a.ranks = nullptr;
      LAUNCH_TRY(launch_prec_rows(a, false, s));
      launches += a.nlong > 0 ? 3 : 2;
    }
    if (te) HIP_TRY(hipEventRecord(te->end, s));
  }
  LAUNCH_TRY(launch_ec_final(g->n, fused ? nullptr : g->prec_y + (iters & 1) * N,
                             fused ? g->prec_aos + (iters & 1) * N : nullptr,
                             g->prec_norm + iters, eigen_out, s));
  ++launches;
  if (ordered) {
    // with no iteration the ranks are x_0, already written under caller ids
    LAUNCH_TRY(launch_prec_remap(g->n, g->ord_old, iters > 0 ? ranks_out : nullptr, ranks,
                                 eigen_out, eigen, s));
    ++launches;
  }
  HIP_TRY(hipEventRecord(g->ev[1], s));
  HIP_TRY(hipStreamSynchronize(s));
  if (g->timing_failed) return fail(GI_ERR_DEVICE, "could not create timing events");
  if ((st = read_kernel_ms(g, launches)) != GI_OK) return st;
  gi_run_stats& rs = g->stats;
  rs.algorithm = 6;
  rs.steps = iters;
  rs.dense_steps = iters;
  rs.edges_examined = (int64_t)iters * g->m * (fused ? 1 : 2);
  rs.trace_len = 0;
  return GI_OK;
}

// Reading a run's statistics waits for the run if its call returned after
// enqueue (the handle's timing state is updated then, hence the cast).
extern "C" gi_status gi_get_run_stats(const gi_graph* g, gi_run_stats* out) {
  if (!g || !out) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (g->stats_pending) {
    gi_status st = finish_pending(const_cast<gi_graph*>(g));
    if (st != GI_OK) return st;
  }
  *out = g->stats;
  return GI_OK;
}

extern "C" gi_status gi_set_step_timing(gi_graph* g, int32_t enable) {
  if (!g) return fail(GI_ERR_INVALID_ARG, "NULL graph");
  if (enable != 0 && enable != 1) return fail(GI_ERR_INVALID_ARG, "enable must be 0 or 1");
  g->step_timing = enable;
  g->timing_failed = false;
  g->tev_count = 0;
  return GI_OK;
}

extern "C" gi_status gi_get_step_times(const gi_graph* g, float* step_ms, float* main_ms,
                                       int32_t cap, int32_t* count) {
  if (!g || !count || cap < 0 || (cap > 0 && (!step_ms || !main_ms)))
    return fail(GI_ERR_INVALID_ARG, "bad step-time arguments");
  if (g->stats_pending) {
    gi_status st = finish_pending(const_cast<gi_graph*>(g));
    if (st != GI_OK) return st;
  }
  const int nk = std::min(g->tev_count, (int)cap);
  for (int k = 0; k < nk; ++k) {
    const StepEvents& t = g->tev[(size_t)k];
    HIP_TRY(hipEventElapsedTime(&step_ms[k], t.start, t.end));
    HIP_TRY(hipEventElapsedTime(&main_ms[k], t.main, t.end));
  }
  *count = g->tev_count;
  return GI_OK;
}

// ------------------------------------------------- frontier primitives ----

extern "C" gi_status gi_frontier_sparse_to_bitvec(int32_t n, const int32_t* ids, int32_t count,
                                                  uint64_t* bv, void* stream) {
  if (n < 1 || count < 0 || count > n || !bv || (count > 0 && !ids))
    return fail(GI_ERR_INVALID_ARG, "bad frontier arguments");
  LAUNCH_TRY(launch_sparse_to_bitvec(n, ids, count, bv, static_cast<hipStream_t>(stream)));
  return GI_OK;
}

extern "C" gi_status gi_frontier_bitvec_to_sparse(int32_t n, const uint64_t* bv, int32_t* ids,
                                                  int32_t* count_dev, void* stream) {
  if (n < 1 || !bv || !ids || !count_dev) return fail(GI_ERR_INVALID_ARG, "bad frontier arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t* scratch = nullptr;
  const size_t W = ((size_t)n + 63) / 64;
  HIP_TRY(hipMallocAsync((void**)&scratch, 4 * (W + 1), s));
  const int rc = launch_bitvec_to_sparse(n, bv, ids, count_dev, scratch, s);
  HIP_TRY(hipFreeAsync(scratch, s));
  if (rc != 0) return fail(GI_ERR_DEVICE, "bitvector compaction launch failed");
  return GI_OK;
}

// Scratch of the allocation-free conversion: one count per bitvector word,
// in a file-scope device array of fixed size.  Every GPU the library runs
// on holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address): it looks up each device's address once with
// hipGetSymbolAddress and passes that.
static __device__ __align__(256) int32_t scratch[GI_NOALLOC_MAX_WORDS];

static std::mutex g_noalloc_mu;
static int32_t* g_noalloc_ptr[GI_NOALLOC_MAX_DEVICES] = {};

static gi_status noalloc_scratch(int32_t** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= GI_NOALLOC_MAX_DEVICES)
    return fail(GI_ERR_UNSUPPORTED, "device %d beyond the %d the allocation-free calls serve", dev,
                GI_NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(GI_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch");
    g_noalloc_ptr[dev] = static_cast<int32_t*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return GI_OK;
}

extern "C" gi_status gi_frontier_bitvec_to_sparse_noalloc(int32_t n, const uint64_t* bv,
                                                          int32_t* ids, int32_t* count_dev,
                                                          void* stream) {
  if (n < 1 || !bv || !ids || !count_dev) return fail(GI_ERR_INVALID_ARG, "bad frontier arguments");
  const int64_t W = ((int64_t)n + 63) / 64;
  if (W > GI_NOALLOC_MAX_WORDS)
    return fail(GI_ERR_UNSUPPORTED,
                "n = %d needs %lld bitvector words; the allocation-free conversion holds at most "
                "%d (n <= %lld)",
                n, (long long)W, GI_NOALLOC_MAX_WORDS, 64LL * GI_NOALLOC_MAX_WORDS);
  int32_t* sc = nullptr;
  gi_status st = noalloc_scratch(&sc);
  if (st != GI_OK) return st;
  // every word count is written before it is read: nothing to clear
  if (launch_bitvec_to_sparse(n, bv, ids, count_dev, sc, static_cast<hipStream_t>(stream)) != 0)
    return fail(GI_ERR_DEVICE, "bitvector compaction launch failed");
  return GI_OK;
}

extern "C" gi_status gi_frontier_bitvec_to_boolmap(int32_t n, const uint64_t* bv, uint8_t* bm,
                                                   void* stream) {
  if (n < 1 || !bv || !bm) return fail(GI_ERR_INVALID_ARG, "bad frontier arguments");
  LAUNCH_TRY(launch_bitvec_to_boolmap(n, bv, bm, static_cast<hipStream_t>(stream)));
  return GI_OK;
}

extern "C" gi_status gi_frontier_boolmap_to_bitvec(int32_t n, const uint8_t* bm, uint64_t* bv,
                                                   void* stream) {
  if (n < 1 || !bv || !bm) return fail(GI_ERR_INVALID_ARG, "bad frontier arguments");
  LAUNCH_TRY(launch_boolmap_to_bitvec(n, bm, bv, static_cast<hipStream_t>(stream)));
  return GI_OK;
}

extern "C" gi_status gi_frontier_degree_sum(const gi_graph* g, const int32_t* ids, int32_t count,
                                            int64_t* out, void* stream) {
  if (!g || !out || count < 0 || (count > 0 && !ids))
    return fail(GI_ERR_INVALID_ARG, "bad frontier arguments");
  LAUNCH_TRY(launch_degree_sum(g->outdeg, ids, count, out, static_cast<hipStream_t>(stream)));
  return GI_OK;
}

// ------------------------------------------------------------- selector ----

struct gi_selector {
  std::vector<float> p;   // host copy of the parameters
  std::vector<float> mu, sd;
  std::vector<float> lo, hi;  // inference clamps each feature to [lo, hi]
  float* d_p = nullptr;   // parameters, then mu[12], isd[12], lo[12], hi[12]
  float* d_m1 = nullptr;  // Adam moments
  float* d_m2 = nullptr;
  float* d_grad = nullptr;
  uint16_t* d_wb = nullptr;
  long long adam_t = 0;
};

// splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) as a counter-based stream.
static uint64_t sel_mix(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

static uint16_t f32_to_bf16(float f) {  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Push the host parameters and standardisation to the device copies.
static gi_status sel_upload(gi_selector* s) {
  std::vector<float> buf(s->p);
  for (int i = 0; i < kFeat; ++i) buf.push_back(s->mu[(size_t)i]);
  for (int i = 0; i < kFeat; ++i) buf.push_back(1.0f / s->sd[(size_t)i]);
  for (int i = 0; i < kFeat; ++i) buf.push_back(s->lo[(size_t)i]);
  for (int i = 0; i < kFeat; ++i) buf.push_back(s->hi[(size_t)i]);
  HIP_TRY(hipMemcpy(s->d_p, buf.data(), sizeof(float) * buf.size(), hipMemcpyHostToDevice));
  std::vector<uint16_t> wb((size_t)kParams);
  for (int i = 0; i < kParams; ++i) wb[(size_t)i] = f32_to_bf16(s->p[(size_t)i]);
  HIP_TRY(hipMemcpy(s->d_wb, wb.data(), 2 * wb.size(), hipMemcpyHostToDevice));
  return GI_OK;
}

static gi_status sel_reset_moments(gi_selector* s) {
  HIP_TRY(hipMemset(s->d_m1, 0, sizeof(float) * kParams));
  HIP_TRY(hipMemset(s->d_m2, 0, sizeof(float) * kParams));
  s->adam_t = 0;
  return GI_OK;
}

extern "C" gi_status gi_selector_destroy(gi_selector* s) {
  if (!s) return GI_OK;
  for (void* q : {(void*)s->d_p, (void*)s->d_m1, (void*)s->d_m2, (void*)s->d_grad, (void*)s->d_wb})
    if (q) dmem_free(q);
  delete s;
  return GI_OK;
}

extern "C" gi_status gi_selector_create(uint64_t seed, gi_selector** out) {
  if (!out) return fail(GI_ERR_INVALID_ARG, "NULL output handle");
  *out = nullptr;
  gi_selector* s = new (std::nothrow) gi_selector();
  if (!s) return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->p.assign((size_t)kParams, 0.0f);
  s->mu.assign((size_t)kFeat, 0.0f);
  s->sd.assign((size_t)kFeat, 1.0f);
  s->lo.assign((size_t)kFeat, -FLT_MAX);
  s->hi.assign((size_t)kFeat, FLT_MAX);
  // He-uniform weights: U(-b, b), b = sqrt(6 / fan_in); zero biases
  auto fill = [&](int off, int count, int fan_in) {
    const double b = std::sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) {
      const double u = (double)(sel_mix(seed * 0x100000001B3ull + (uint64_t)(off + i)) >> 11) *
                       (1.0 / 9007199254740992.0);
      s->p[(size_t)(off + i)] = (float)((2.0 * u - 1.0) * b);
    }
  };
  fill(kOffW1, kFeat * kHid, kFeat);
  fill(kOffW2, kHid * kHid, kHid);
  fill(kOffW3, kHid * kOut, kHid);
  if (dmem_get((void**)&s->d_p, sizeof(float) * kSelBuf) != hipSuccess ||
      dmem_get((void**)&s->d_m1, sizeof(float) * kParams) != hipSuccess ||
      dmem_get((void**)&s->d_m2, sizeof(float) * kParams) != hipSuccess ||
      dmem_get((void**)&s->d_grad, sizeof(float) * kParams) != hipSuccess ||
      dmem_get((void**)&s->d_wb, 2 * (size_t)kParams) != hipSuccess) {
    (void)hipGetLastError();
    gi_selector_destroy(s);
    return fail(GI_ERR_OUT_OF_MEMORY, "selector device allocation failed");
  }
  gi_status st = sel_upload(s);
  if (st == GI_OK) st = sel_reset_moments(s);
  if (st != GI_OK) {
    gi_selector_destroy(s);
    return st;
  }
  *out = s;
  return GI_OK;
}

extern "C" gi_status gi_selector_get_params(const gi_selector* s, float* params, float* mu,
                                            float* sd) {
  if (!s) return fail(GI_ERR_INVALID_ARG, "NULL selector");
  if (params) std::memcpy(params, s->p.data(), sizeof(float) * kParams);
  if (mu) std::memcpy(mu, s->mu.data(), sizeof(float) * kFeat);
  if (sd) std::memcpy(sd, s->sd.data(), sizeof(float) * kFeat);
  return GI_OK;
}

extern "C" gi_status gi_selector_set_params(gi_selector* s, const float* params, const float* mu,
                                            const float* sd) {
  if (!s) return fail(GI_ERR_INVALID_ARG, "NULL selector");
  if (sd)
    for (int i = 0; i < kFeat; ++i)
      if (!(sd[i] > 0.0f)) return fail(GI_ERR_INVALID_ARG, "sd[%d] must be > 0", i);
  if (params) std::memcpy(s->p.data(), params, sizeof(float) * kParams);
  if (mu) std::memcpy(s->mu.data(), mu, sizeof(float) * kFeat);
  if (sd) std::memcpy(s->sd.data(), sd, sizeof(float) * kFeat);
  gi_status st = sel_upload(s);
  return st != GI_OK ? st : sel_reset_moments(s);
}

extern "C" gi_status gi_selector_get_range(const gi_selector* s, float* lo, float* hi) {
  if (!s) return fail(GI_ERR_INVALID_ARG, "NULL selector");
  if (lo) std::memcpy(lo, s->lo.data(), sizeof(float) * kFeat);
  if (hi) std::memcpy(hi, s->hi.data(), sizeof(float) * kFeat);
  return GI_OK;
}

extern "C" gi_status gi_selector_set_range(gi_selector* s, const float* lo, const float* hi) {
  if (!s) return fail(GI_ERR_INVALID_ARG, "NULL selector");
  for (int i = 0; i < kFeat; ++i) {
    const float a = lo ? lo[i] : s->lo[(size_t)i], b = hi ? hi[i] : s->hi[(size_t)i];
    if (std::isnan(a) || std::isnan(b) || a > b)
      return fail(GI_ERR_INVALID_ARG, "feature %d: range [%g, %g] is empty or NaN", i, a, b);
  }
  if (lo) std::memcpy(s->lo.data(), lo, sizeof(float) * kFeat);
  if (hi) std::memcpy(s->hi.data(), hi, sizeof(float) * kFeat);
  return sel_upload(s);
}

// Device copies of training records, released on scope exit.
struct DevRecords {
  float* x = nullptr;
  float* y = nullptr;
  uint8_t* v = nullptr;
  int32_t* order = nullptr;
  float* loss = nullptr;
  ~DevRecords() {
    for (void* q : {(void*)x, (void*)y, (void*)v, (void*)order, (void*)loss})
      if (q) dmem_free(q);
  }
};

static gi_status sel_records(DevRecords& r, const float* feats, const float* log_ms,
                             const uint8_t* valid, int64_t count, const std::vector<int32_t>& order,
                             int loss_len) {
  const size_t n = (size_t)count;
  if (dmem_get((void**)&r.x, sizeof(float) * n * kFeat) != hipSuccess ||
      dmem_get((void**)&r.y, sizeof(float) * n * kOut) != hipSuccess ||
      dmem_get((void**)&r.v, n * kOut) != hipSuccess ||
      dmem_get((void**)&r.order, sizeof(int32_t) * n) != hipSuccess ||
      dmem_get((void**)&r.loss, sizeof(float) * (size_t)std::max(loss_len, 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GI_ERR_OUT_OF_MEMORY, "selector record allocation failed");
  }
  HIP_TRY(hipMemcpy(r.x, feats, sizeof(float) * n * kFeat, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(r.y, log_ms, sizeof(float) * n * kOut, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(r.v, valid, n * kOut, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(r.order, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  return GI_OK;
}

static gi_status sel_check_records(const float* feats, const float* log_ms, const uint8_t* valid,
                                   int64_t count) {
  if (!feats || !log_ms || !valid || count < 1 || count > INT32_MAX)
    return fail(GI_ERR_INVALID_ARG, "bad selector records");
  for (int64_t r = 0; r < count; ++r) {
    int any = 0;
    for (int q = 0; q < kOut; ++q) {
      if (valid[r * kOut + q]) {
        any = 1;
        if (!std::isfinite(log_ms[r * kOut + q]))
          return fail(GI_ERR_INVALID_ARG, "record %lld: non-finite target", (long long)r);
      }
    }
    if (!any) return fail(GI_ERR_INVALID_ARG, "record %lld has no valid schedule", (long long)r);
    for (int f = 0; f < kFeat; ++f)
      if (!std::isfinite(feats[r * kFeat + f]))
        return fail(GI_ERR_INVALID_ARG, "record %lld: non-finite feature", (long long)r);
  }
  return GI_OK;
}

static TrainArgs train_args(gi_selector* s, const DevRecords& r, int n, int epochs, float lr,
                            int apply) {
  TrainArgs a;
  a.p = s->d_p;
  a.m1 = s->d_m1;
  a.m2 = s->d_m2;
  a.grad = s->d_grad;
  a.x = r.x;
  a.y = r.y;
  a.valid = r.v;
  a.order = r.order;
  a.n = n;
  a.mu = s->d_p + kParams;
  a.isd = s->d_p + kParams + kFeat;
  a.epochs = epochs;
  a.lr = lr;
  a.beta1 = 0.9f;
  a.beta2 = 0.999f;
  a.eps = 1e-8f;
  a.apply = apply;
  a.t0 = s->adam_t;
  a.loss = r.loss;
  return a;
}

extern "C" gi_status gi_selector_train(gi_selector* s, const float* feats, const float* log_ms,
                                       const uint8_t* valid, int64_t count, int32_t epochs,
                                       float lr, uint64_t seed, int32_t standardise, float* loss) {
  if (!s) return fail(GI_ERR_INVALID_ARG, "NULL selector");
  if (epochs < 1 || !(lr > 0.0f)) return fail(GI_ERR_INVALID_ARG, "epochs >= 1 and lr > 0 required");
  gi_status st = sel_check_records(feats, log_ms, valid, count);
  if (st != GI_OK) return st;
  if (standardise) {
    for (int f = 0; f < kFeat; ++f) {
      double sum = 0.0, sq = 0.0;
      for (int64_t r = 0; r < count; ++r) {
        const double x = feats[r * kFeat + f];
        sum += x;
        sq += x * x;
      }
      const double mean = sum / count, var = std::max(0.0, sq / count - mean * mean);
      s->mu[(size_t)f] = (float)mean;
      s->sd[(size_t)f] = var > 1e-12 ? (float)std::sqrt(var) : 1.0f;
      float lo = feats[f], hi = feats[f];
      for (int64_t r = 1; r < count; ++r) {
        lo = std::min(lo, feats[r * kFeat + f]);
        hi = std::max(hi, feats[r * kFeat + f]);
      }
      s->lo[(size_t)f] = lo;
      s->hi[(size_t)f] = hi;
    }
    if ((st = sel_upload(s)) != GI_OK) return st;
  }
  // seeded Fisher-Yates order (the same every epoch)
  std::vector<int32_t> order((size_t)count);
  for (int64_t i = 0; i < count; ++i) order[(size_t)i] = (int32_t)i;
  for (int64_t i = count - 1; i > 0; --i) {
    const uint64_t j = sel_mix(seed ^ (0xD1B54A32D192ED03ull * (uint64_t)i)) % (uint64_t)(i + 1);
    std::swap(order[(size_t)i], order[(size_t)j]);
  }
  DevRecords r;
  if ((st = sel_records(r, feats, log_ms, valid, count, order, epochs)) != GI_OK) return st;
  const TrainArgs a = train_args(s, r, (int)count, epochs, lr, 1);
  LAUNCH_TRY(launch_mlp_train(a, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  s->adam_t += (long long)epochs * ((count + 31) / 32);
  HIP_TRY(hipMemcpy(s->p.data(), s->d_p, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  if (loss) HIP_TRY(hipMemcpy(loss, r.loss, sizeof(float) * (size_t)epochs, hipMemcpyDeviceToHost));
  // refresh the bf16 copy from the trained weights
  return sel_upload(s);
}

extern "C" gi_status gi_selector_gradient(gi_selector* s, const float* feats, const float* log_ms,
                                          const uint8_t* valid, int32_t count, float* grad,
                                          float* loss) {
  if (!s || !grad) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  if (count < 1 || count > 32) return fail(GI_ERR_INVALID_ARG, "count must be in [1, 32]");
  gi_status st = sel_check_records(feats, log_ms, valid, count);
  if (st != GI_OK) return st;
  std::vector<int32_t> order((size_t)count);
  for (int i = 0; i < count; ++i) order[(size_t)i] = i;
  DevRecords r;
  if ((st = sel_records(r, feats, log_ms, valid, count, order, 1)) != GI_OK) return st;
  const TrainArgs a = train_args(s, r, count, 1, 0.0f, 0);
  LAUNCH_TRY(launch_mlp_train(a, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(grad, s->d_grad, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  if (loss) HIP_TRY(hipMemcpy(loss, r.loss, sizeof(float), hipMemcpyDeviceToHost));
  return GI_OK;
}

extern "C" gi_status gi_selector_predict(const gi_selector* s, const float* feats, int64_t count,
                                         int32_t bf16, float* out) {
  if (!s || !feats || !out || count < 0) return fail(GI_ERR_INVALID_ARG, "bad arguments");
  if (count == 0) return GI_OK;
  float* dx = nullptr;
  float* dy = nullptr;
  if (dmem_get((void**)&dx, sizeof(float) * (size_t)count * kFeat) != hipSuccess ||
      dmem_get((void**)&dy, sizeof(float) * (size_t)count * kOut) != hipSuccess) {
    (void)hipGetLastError();
    if (dx) dmem_free(dx);
    return fail(GI_ERR_OUT_OF_MEMORY, "prediction buffers");
  }
  SelDev d;
  d.p = s->d_p;
  d.wb = s->d_wb;
  d.mu = s->d_p + kParams;
  d.isd = s->d_p + kParams + kFeat;
  d.lo = s->d_p + kParams + 2 * kFeat;
  d.hi = s->d_p + kParams + 3 * kFeat;
  gi_status st = GI_OK;
  if (hipMemcpy(dx, feats, sizeof(float) * (size_t)count * kFeat, hipMemcpyHostToDevice) != hipSuccess)
    st = fail(GI_ERR_DEVICE, "copy of features failed");
  else if (launch_mlp_predict(d, dx, count, bf16 != 0, dy, nullptr) != 0)
    st = fail(GI_ERR_DEVICE, "prediction launch failed: %s", hipGetErrorString(hipGetLastError()));
  else if (hipMemcpy(out, dy, sizeof(float) * (size_t)count * kOut, hipMemcpyDeviceToHost) != hipSuccess)
    st = fail(GI_ERR_DEVICE, "copy of predictions failed");
  dmem_free(dx);
  dmem_free(dy);
  return st;
}

extern "C" gi_status gi_selector_attach(gi_graph* g, const gi_selector* s) {
  if (!g) return fail(GI_ERR_INVALID_ARG, "NULL graph");
  HIP_TRY(hipDeviceSynchronize());
  for (void* q : {(void*)g->sel_p, (void*)g->sel_wb, (void*)g->sel_io})
    if (q) dmem_free(q);
  g->sel_p = nullptr;
  g->sel_wb = nullptr;
  g->sel_io = nullptr;
  if (!s) return GI_OK;
  if (dmem_get((void**)&g->sel_p, sizeof(float) * kSelBuf) != hipSuccess ||
      dmem_get((void**)&g->sel_wb, 2 * (size_t)kParams) != hipSuccess ||
      dmem_get((void**)&g->sel_io, sizeof(float) * (kFeat + kOut)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GI_ERR_OUT_OF_MEMORY, "selector copy allocation failed");
  }
  HIP_TRY(hipMemcpy(g->sel_p, s->d_p, sizeof(float) * kSelBuf,
                    hipMemcpyDeviceToDevice));
  HIP_TRY(hipMemcpy(g->sel_wb, s->d_wb, 2 * (size_t)kParams, hipMemcpyDeviceToDevice));
  return GI_OK;
}

extern "C" gi_status gi_get_step_features(const gi_graph* g, float* feats, int32_t cap,
                                          int32_t* count) {
  if (!g || !count || cap < 0 || (cap > 0 && !feats))
    return fail(GI_ERR_INVALID_ARG, "bad step-feature arguments");
  const int alg = g->stats.algorithm;
  const int k = (alg == ALG_BFS || alg == ALG_CC) ? std::min(g->stats.trace_len, kMaxLog) : 0;
  const volatile HostFlags* h = g->hflags;
  for (int i = 0; i < std::min(k, (int)cap); ++i)
    for (int f = 0; f < kFeat; ++f) feats[(size_t)i * kFeat + f] = h->feat[i][f];
  *count = k;
  return GI_OK;
}

extern "C" gi_status gi_trace_exhaustive(gi_graph* g, int32_t algorithm, int32_t src, float* feats,
                                         float* step_ms, uint8_t* valid, int32_t cap,
                                         int32_t* count) {
  if (!g || !count || cap < 0 || (cap > 0 && (!feats || !step_ms || !valid)))
    return fail(GI_ERR_INVALID_ARG, "bad trace arguments");
  if (algorithm != GI_ALG_PAGERANK && algorithm != GI_ALG_BFS && algorithm != GI_ALG_CC)
    return fail(GI_ERR_INVALID_ARG, "algorithm %d has no schedule choice", algorithm);
  if (algorithm == GI_ALG_BFS && (src < 0 || src >= g->n))
    return fail(GI_ERR_INVALID_ARG, "source %d outside [0, %d)", src, g->n);
  int32_t* out = nullptr;
  if (dmem_get((void**)&out, sizeof(float) * (size_t)g->n) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GI_ERR_OUT_OF_MEMORY, "trace output buffer");
  }
  const gi_schedule saved = g->sched;
  const int saved_timing = g->step_timing;
  g->step_timing = 1;
  g->timing_failed = false;
  gi_status st = GI_OK;
  int steps = -1;
  std::vector<int32_t> fr0;
  std::vector<float> t((size_t)kMaxLog * kOut, 0.0f);
  std::vector<uint8_t> ok((size_t)kMaxLog * kOut, 0);
  std::vector<float> x((size_t)kMaxLog * kFeat, 0.0f);
  // PageRank: S2, S3; BFS: S0..S2; CC: S0..S3.  S3 pulls over the
  // schedule's source segments (the automatic count when it has none), and
  // PageRank's S2 follows the schedule's vertex order: the same layout the
  // learned choice runs on
  const int nsched = algorithm == GI_ALG_PAGERANK ? 2 : algorithm == GI_ALG_CC ? 4 : 3;
  for (int q = 0; q < nsched && st == GI_OK; ++q) {
    const int sched = algorithm == GI_ALG_PAGERANK ? 2 + q : q;  // S index
    if (algorithm == GI_ALG_CC && sched == 3) {
      g->sched.direction = GI_DIR_DENSE_PULL;
      g->sched.dense_frontier = GI_FRONTIER_BITVECTOR;
      if (saved.num_segments <= 1) {
        g->sched.num_segments = auto_segments(g);
        g->sched.segment_strategy = GI_SEG_FIXED_VERTEX_COUNT;
      }
      st = gi_cc(g, out, nullptr);
      g->sched.num_segments = saved.num_segments;
      g->sched.segment_strategy = saved.segment_strategy;
    } else if (algorithm == GI_ALG_PAGERANK) {
      g->sched.direction = GI_DIR_DENSE_PULL;
      const bool seg = sched == 3;
      if (seg && (st = saved.num_segments > 1 ? ensure_pr_segments(g, saved.num_segments,
                                                                   saved.segment_strategy)
                                              : ensure_segments(g)) != GI_OK)
        break;
      st = !seg && saved.vertex_order == GI_ORDER_OUT_DEGREE
               ? pr_run_ordered(g, 20, 0.85f, reinterpret_cast<float*>(out), nullptr)
               : pr_run(g, 20, 0.85f, reinterpret_cast<float*>(out), nullptr, seg);
      if (st == GI_OK) st = finish_pending(g);  // the run returned after enqueue
    } else {
      g->sched.direction = sched;  // GI_DIR_SPARSE_PUSH, DENSE_PUSH, DENSE_PULL
      g->sched.dense_frontier = GI_FRONTIER_BITVECTOR;
      g->sched.num_segments = 1;
      st = algorithm == GI_ALG_BFS ? gi_bfs(g, src, out, nullptr, nullptr) : gi_cc(g, out, nullptr);
      g->sched.num_segments = saved.num_segments;
    }
    if (st != GI_OK) break;
    const gi_run_stats& rs = g->stats;
    const int k = std::min(rs.trace_len, kMaxLog);
    if (q == 0) {
      steps = k;
      fr0.assign(rs.step_frontier, rs.step_frontier + k);
      if (algorithm == GI_ALG_PAGERANK) {
        for (int i = 0; i < k; ++i) pr_features(g, &x[(size_t)i * kFeat]);
      } else {
        const volatile HostFlags* h = g->hflags;
        for (int i = 0; i < k; ++i)
          for (int f = 0; f < kFeat; ++f) x[(size_t)i * kFeat + f] = h->feat[i][f];
      }
    } else if (k != steps || !std::equal(fr0.begin(), fr0.end(), rs.step_frontier)) {
      st = fail(GI_ERR_DEVICE, "frontier sequence differs between schedules");
      break;
    }
    const int ne = std::min(g->tev_count, k);
    for (int i = 0; i < ne; ++i) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, g->tev[(size_t)i].start, g->tev[(size_t)i].end) != hipSuccess) {
        st = fail(GI_ERR_DEVICE, "event timing failed");
        break;
      }
      t[(size_t)i * kOut + sched] = ms;
      ok[(size_t)i * kOut + sched] = 1;
    }
  }
  g->sched = saved;
  g->step_timing = saved_timing;
  dmem_free(out);
  if (st != GI_OK) return st;
  const int k = std::max(steps, 0);
  for (int i = 0; i < std::min(k, (int)cap); ++i) {
    std::memcpy(&feats[(size_t)i * kFeat], &x[(size_t)i * kFeat], sizeof(float) * kFeat);
    std::memcpy(&step_ms[(size_t)i * kOut], &t[(size_t)i * kOut], sizeof(float) * kOut);
    std::memcpy(&valid[(size_t)i * kOut], &ok[(size_t)i * kOut], kOut);
  }
  *count = k;
  return GI_OK;
}

// ---------------------------------------------------------------- batch ----

struct gi_batch {
  std::vector<gi_graph*> graphs;
  std::vector<gi_task> tasks;
  std::vector<int> k;        // workgroups per task
  std::vector<double> est;   // estimated time per task (ms, or a size proxy before tuning)
  int max_grid = 0;          // resident workgroups of the batch kernel
  int grid = 0;
  int bt = 256;              // threads per workgroup
  int algs = kBatchAll;      // algorithms among the tasks (selects the kernel build)
  int trace_cap = 0;         // per-task step records (gi_batch_set_trace)
  long long* d_trace = nullptr;
  bool bt_pinned = false;    // set by gi_batch_set_threads: the autotuner keeps it
  bool xcd_local = true;     // place each task's workgroups on one XCD when they fit
  int xcd_barrier = 1;       // one-XCD task barriers where a task's workgroups share an L2
  int cus = 0;
  size_t lds = 0;
  int cap_e = 0;
  long long spin_limit = 0;
  int clock_khz = 100000;
  BatchGraph* d_graphs = nullptr;
  BatchTask* d_tasks = nullptr;
  TaskCtl* d_ctl = nullptr;
  int2* d_items = nullptr;
  int* d_wg_off = nullptr;
  int* d_err = nullptr;
  std::vector<BatchTask> h_tasks;
  // per graph: the batch's own PageRank destination blocks (block size
  // chosen per graph by the autotuner; the graph's own schedule untouched)
  struct PrLayout {
    int cap_e = 0, cap_v = 0, ntab = 0, nlong = 0;
    int4* table = nullptr;
    int32_t* chunks = nullptr;
  };
  std::vector<PrLayout> lay;
  std::vector<int> lr_max;   // per graph: long-row slots at the smallest block size
  std::vector<void*> work;
  hipStream_t gstream = nullptr;
  hipGraph_t hg = nullptr;
  hipGraphExec_t hx = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t evw = nullptr;  // orders the batch's stream after the caller's
  bool launched = false;     // gi_batch_launch done, gi_batch_wait not yet
  float last_ms = 0.0f;
};

static void batch_drop_graph(gi_batch* b) {
  if (b->hx) (void)hipGraphExecDestroy(b->hx);
  if (b->hg) (void)hipGraphDestroy(b->hg);
  b->hx = nullptr;
  b->hg = nullptr;
}

static void batch_free_layout(gi_batch::PrLayout* l) {
  if (l->table) dmem_free(l->table);
  if (l->chunks) dmem_free(l->chunks);
  l->table = nullptr;
  l->chunks = nullptr;
}

extern "C" gi_status gi_batch_destroy(gi_batch* b) {
  if (!b) return GI_OK;
  (void)hipDeviceSynchronize();
  batch_drop_graph(b);
  for (gi_batch::PrLayout& l : b->lay) batch_free_layout(&l);
  for (void* q : b->work) dmem_free(q);
  for (void* q : {(void*)b->d_graphs, (void*)b->d_tasks, (void*)b->d_ctl, (void*)b->d_items,
                  (void*)b->d_wg_off, (void*)b->d_err, (void*)b->d_trace})
    if (q) dmem_free(q);
  for (hipEvent_t e : b->ev)
    if (e) (void)hipEventDestroy(e);
  if (b->evw) (void)hipEventDestroy(b->evw);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  delete b;
  return GI_OK;
}

template <typename T>
static gi_status batch_alloc(gi_batch* b, T** p, size_t count) {
  void* q = nullptr;
  if (dmem_get(&q, std::max<size_t>(1, count * sizeof(T))) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GI_ERR_OUT_OF_MEMORY, "batch workspace allocation failed");
  }
  b->work.push_back(q);
  *p = static_cast<T*>(q);
  return GI_OK;
}

// PageRank block sizes (edges per destination block) the autotuner tries for
// a graph's PageRank tasks; a batch's long-row slots are sized for the
// smallest.
static const int kBatchCaps[] = {256, 512, 1024, 2048, 4096};
constexpr int kBatchCapMin = 256, kBatchCapMax = 4096;

// The batch's destination blocks of graph i at cap_e edges per block.
static gi_status batch_set_layout(gi_batch* b, size_t i, int cap_e) {
  gi_batch::PrLayout& l = b->lay[i];
  if (l.table && l.cap_e == cap_e) return GI_OK;
  const gi_graph* g = b->graphs[i];
  std::vector<int32_t> chunks;
  const int cap_v = std::min(cap_e, 1024);
  const std::vector<int4> tab = make_pr_table(g->h_in_off.data(), g->n, cap_e, cap_v, &chunks);
  if ((int)chunks.size() > b->lr_max[i] || cap_e > b->cap_e)
    return fail(GI_ERR_INVALID_ARG, "PageRank block size %d outside the batch's range", cap_e);
  HIP_TRY(hipDeviceSynchronize());  // no launch reads the old blocks any more
  batch_free_layout(&l);
  if (dmem_get((void**)&l.table, sizeof(int4) * std::max<size_t>(1, tab.size())) != hipSuccess ||
      dmem_get((void**)&l.chunks, sizeof(int32_t) * std::max<size_t>(1, chunks.size())) !=
          hipSuccess) {
    (void)hipGetLastError();
    batch_free_layout(&l);
    return fail(GI_ERR_OUT_OF_MEMORY, "batch PageRank blocks");
  }
  HIP_TRY(hipMemcpy(l.table, tab.data(), sizeof(int4) * tab.size(), hipMemcpyHostToDevice));
  if (!chunks.empty())
    HIP_TRY(hipMemcpy(l.chunks, chunks.data(), sizeof(int32_t) * chunks.size(),
                      hipMemcpyHostToDevice));
  l.cap_e = cap_e;
  l.cap_v = cap_v;
  l.ntab = (int)tab.size();
  l.nlong = (int)chunks.size();
  return GI_OK;
}

// Workgroup size: the resident grid follows from the kernel's occupancy at
// that size (at most 8 workgroups per CU).
static gi_status batch_set_bt(gi_batch* b, int bt) {
  if (!batch_threads_ok(bt)) return fail(GI_ERR_INVALID_ARG, "threads must be 256, 512 or 1024");
  const int occ = batch_occupancy(bt, b->lds, b->algs);
  if (occ < 1) return fail(GI_ERR_DEVICE, "batch kernel does not fit on a compute unit");
  b->bt = bt;
  b->max_grid = b->cus * std::min(occ, 8);
  return GI_OK;
}

static BatchGraph batch_graph(const gi_graph* g, const gi_batch::PrLayout& l) {
  BatchGraph d;
  d.n = g->n;
  d.m = g->m;
  d.out_off = g->out_off;
  d.out_idx = g->out_idx;
  d.in_off = g->in_off;
  d.in_idx = g->in_idx;
  d.outdeg = g->outdeg;
  d.out_w = g->out_w;
  d.in_probe = g->in_probe;
  d.bfs_idx = g->bfs_idx;
  d.hubs = g->hubs;
  d.nhubs = g->nhubs;
  d.pr_table = l.table;
  d.pr_ntab = l.ntab;
  d.pr_cap_e = l.cap_e;
  d.lr_chunks = l.chunks;
  d.n_long = l.nlong;
  return d;
}

// Workgroup lists: tasks in decreasing estimated time; a task of k
// workgroups goes to the aligned block of pow2ceil(k) workgroups whose first
// k have the least maximum load, and those k then all carry that maximum
// plus the task's time, so a task's workgroups reach it together instead of
// one waiting behind another's earlier work.  Every list follows the one
// task order.
//
// XCD placement: workgroups are dispatched to the 8 XCDs round-robin by
// index, so the plan works on logical slots l = x * (G / 8) + j that map to
// workgroup j * 8 + x, and a block is placed inside one XCD's range when the
// task fits in it.  A task's workgroups then share one L2: its frontier and
// visited bitvectors stay cached there instead of competing with every
// other task's in all eight.  (Placement affects speed only; the barriers
// synchronise at device scope.)
static gi_status batch_plan(gi_batch* b) {
  const int nt = (int)b->tasks.size();
  std::vector<int> order((size_t)nt);
  for (int i = 0; i < nt; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->est[(size_t)x] > b->est[(size_t)y]; });
  int maxk = 1;
  for (int i = 0; i < nt; ++i) maxk = std::max(maxk, b->k[(size_t)i]);
  b->grid = std::min(b->max_grid, std::max(maxk, 1));
  // grow the grid to the resident limit when the work can use it
  long long want = 0;
  for (int i = 0; i < nt; ++i) want += b->k[(size_t)i];
  b->grid = (int)std::min<long long>(b->max_grid, std::max<long long>(b->grid, want));
  constexpr int kXcd = 8;
  if (b->grid >= kXcd && b->grid % kXcd != 0 && b->max_grid % kXcd == 0)
    b->grid = std::min(b->max_grid, (b->grid + kXcd - 1) / kXcd * kXcd);
  const int G = b->grid;
  const bool xcd = b->xcd_local && G >= kXcd && G % kXcd == 0;
  const int per = xcd ? G / kXcd : G;  // logical slots per XCD
  const int pal = per & -per;          // largest power of two dividing per
  std::vector<double> load((size_t)G, 0.0);
  std::vector<std::vector<int2>> lists((size_t)G);  // by logical slot
  for (int t : order) {
    const int k = std::min(b->k[(size_t)t], G);
    b->k[(size_t)t] = k;
    int P = 1;
    while (P < k) P <<= 1;
    int best = 0;
    double best_max = 1e300;
    auto consider = [&](int w0) {
      double mx = 0.0;
      for (int r = 0; r < k; ++r) mx = std::max(mx, load[(size_t)(w0 + r)]);
      if (mx < best_max) {
        best_max = mx;
        best = w0;
      }
    };
    if (k <= per) {
      // inside one XCD's range, starts aligned to min(P, pal) so that a
      // range that is not a power of two still holds its share of blocks
      const int step = std::min(P, pal);
      for (int x = 0; x * per < G; ++x)
        for (int w0 = x * per; w0 + k <= (x + 1) * per; w0 += step) consider(w0);
    } else {
      for (int w0 = 0; w0 + k <= G; w0 += std::min(P, G)) consider(w0);
    }
    for (int r = 0; r < k; ++r) {
      const int w = best + r;
      lists[(size_t)w].push_back(make_int2(t, r));
      load[(size_t)w] = best_max + b->est[(size_t)t];
    }
  }
  std::vector<int> off((size_t)G + 1, 0);
  std::vector<int2> items;
  for (int w = 0; w < G; ++w) {
    // workgroup w runs the list of logical slot (w % 8) * per + w / 8
    const int l = xcd ? (w % kXcd) * per + w / kXcd : w;
    off[(size_t)w] = (int)items.size();
    items.insert(items.end(), lists[(size_t)l].begin(), lists[(size_t)l].end());
  }
  off[(size_t)G] = (int)items.size();
  for (void* q : {(void*)b->d_items, (void*)b->d_wg_off})
    if (q) dmem_free(q);
  b->d_items = nullptr;
  b->d_wg_off = nullptr;
  if (dmem_get((void**)&b->d_items, sizeof(int2) * std::max<size_t>(1, items.size())) != hipSuccess ||
      dmem_get((void**)&b->d_wg_off, sizeof(int) * off.size()) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GI_ERR_OUT_OF_MEMORY, "batch plan allocation failed");
  }
  HIP_TRY(hipMemcpy(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_wg_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice));
  for (int t = 0; t < nt; ++t) b->h_tasks[(size_t)t].k = b->k[(size_t)t];
  HIP_TRY(hipMemcpy(b->d_tasks, b->h_tasks.data(), sizeof(BatchTask) * (size_t)nt,
                    hipMemcpyHostToDevice));
  batch_drop_graph(b);
  return GI_OK;
}

extern "C" gi_status gi_batch_create(gi_graph* const* graphs, int32_t ngraphs, const gi_task* tasks,
                                     int32_t ntasks, gi_batch** out) {
  if (!out) return fail(GI_ERR_INVALID_ARG, "NULL output handle");
  *out = nullptr;
  if (!graphs || ngraphs < 1 || !tasks || ntasks < 1 || ntasks > (1 << 20))
    return fail(GI_ERR_INVALID_ARG, "need graphs and tasks");
  for (int i = 0; i < ngraphs; ++i)
    if (!graphs[i]) return fail(GI_ERR_INVALID_ARG, "graph %d is NULL", i);
  for (int i = 0; i < ntasks; ++i) {
    const gi_task& t = tasks[i];
    if (t.graph < 0 || t.graph >= ngraphs) return fail(GI_ERR_INVALID_ARG, "task %d: bad graph", i);
    if (t.algorithm != GI_ALG_BFS && t.algorithm != GI_ALG_PAGERANK && t.algorithm != GI_ALG_SSSP)
      return fail(GI_ERR_INVALID_ARG, "task %d: algorithm must be BFS, PageRank or SSSP", i);
    if (!t.out) return fail(GI_ERR_INVALID_ARG, "task %d: NULL output", i);
    const gi_graph* g = graphs[t.graph];
    if ((t.algorithm == GI_ALG_BFS || t.algorithm == GI_ALG_SSSP) && (t.src < 0 || t.src >= g->n))
      return fail(GI_ERR_INVALID_ARG, "task %d: source outside the graph", i);
    if (t.algorithm == GI_ALG_SSSP && !g->weighted)
      return fail(GI_ERR_INVALID_ARG, "task %d: SSSP needs a weighted graph", i);
    if (t.algorithm == GI_ALG_PAGERANK &&
        (t.iters < 0 || !(t.damping >= 0.0f && t.damping <= 1.0f)))
      return fail(GI_ERR_INVALID_ARG, "task %d: bad PageRank parameters", i);
    if (t.workgroups < 0 || t.workgroups > 1024)
      return fail(GI_ERR_INVALID_ARG, "task %d: workgroups outside [0, 1024]", i);
    if (t.hybrid_divisor < 0) return fail(GI_ERR_INVALID_ARG, "task %d: hybrid_divisor < 0", i);
  }
  gi_batch* b = new (std::nothrow) gi_batch();
  if (!b) return fail(GI_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->graphs.assign(graphs, graphs + ngraphs);
  b->tasks.assign(tasks, tasks + ntasks);
  b->algs = 0;
  for (int32_t i = 0; i < ntasks; ++i)
    b->algs |= tasks[i].algorithm == GI_ALG_BFS    ? kBatchBfs
               : tasks[i].algorithm == GI_ALG_SSSP ? kBatchSssp
                                                   : kBatchPr;
  auto bail = [&](gi_status st) {
    gi_batch_destroy(b);
    return st;
  };
  // PageRank blocks: the batch's own, at first the graph's block size, any
  // of kBatchCaps after tuning; LDS and long-row slots sized for all of them
  int cap_e = kBatchCapMax;
  std::vector<bool> has_pr((size_t)ngraphs, false);
  for (int32_t i = 0; i < ntasks; ++i)
    if (tasks[i].algorithm == GI_ALG_PAGERANK) has_pr[(size_t)tasks[i].graph] = true;
  b->lay.resize((size_t)ngraphs);
  b->lr_max.assign((size_t)ngraphs, 0);
  for (size_t i = 0; i < (size_t)ngraphs; ++i) {
    const gi_graph* g = b->graphs[i];
    cap_e = std::max(cap_e, g->pr_cap_e);
    const int lo = std::min(kBatchCapMin, g->pr_cap_e);
    int nl = 0;
    for (int32_t v = 0; v < g->n; ++v) nl += g->h_in_off[(size_t)v + 1] - g->h_in_off[(size_t)v] > lo;
    b->lr_max[i] = nl;
  }
  b->cap_e = cap_e;
  b->lds = batch_lds_bytes(cap_e, std::min(cap_e, 1024));
  for (size_t i = 0; i < (size_t)ngraphs; ++i) {
    if (!has_pr[i]) continue;
    gi_status sl = batch_set_layout(b, i, b->graphs[i]->pr_cap_e);
    if (sl != GI_OK) return bail(sl);
  }
  for (int32_t i = 0; i < ntasks; ++i) {
    if (tasks[i].algorithm != GI_ALG_BFS) continue;
    gi_status sb = ensure_bfs_rows(b->graphs[(size_t)tasks[i].graph]);
    if (sb != GI_OK) return bail(sb);
  }
  int dev = 0, cus = 0, rate = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate <= 0)
    rate = 100000;  // kHz
  b->spin_limit = 2000LL * rate;  // two seconds of wall clock
  b->clock_khz = rate;
  b->cus = cus;
  // resident by construction: at most the occupancy (and at most 8 per CU)
  gi_status st = batch_set_bt(b, 256);
  if (st != GI_OK) return bail(st);
  const size_t nt = (size_t)ntasks;
  b->h_tasks.resize(nt);
  b->k.resize(nt);
  b->est.resize(nt);
  for (size_t i = 0; i < nt; ++i) {
    const gi_task& t = b->tasks[i];
    const gi_graph* g = b->graphs[(size_t)t.graph];
    BatchTask& d = b->h_tasks[i];
    d = BatchTask{};
    d.id = (int)i;
    d.alg = t.algorithm == GI_ALG_BFS ? ALG_BFS : t.algorithm == GI_ALG_SSSP ? ALG_SSSP : ALG_PR;
    d.delta = t.sssp_delta > 0 ? t.sssp_delta
                               : (g->sched.sssp_delta > 0 ? g->sched.sssp_delta : 512u);
    d.div = t.hybrid_divisor > 0 ? t.hybrid_divisor : g->sched.hybrid_divisor;
    d.graph = t.graph;
    d.src = t.src;
    d.iters = t.iters;
    d.damping = t.damping;
    d.out = t.out;
    d.parent = t.algorithm == GI_ALG_BFS ? static_cast<int32_t*>(t.parent) : nullptr;
    const size_t W = ((size_t)g->n + 63) / 64;
    if (d.alg == ALG_BFS || d.alg == ALG_SSSP) {
      if ((st = batch_alloc(b, &d.vis, 4 * W)) != GI_OK) return bail(st);
      d.bv0 = d.vis + W;
      d.bv1 = d.vis + 2 * W;
      d.bv2 = d.vis + 3 * W;
      if (d.alg == ALG_SSSP && (st = batch_alloc(b, &d.q, 5 * (size_t)g->n)) != GI_OK)
        return bail(st);
    } else {
      if ((st = batch_alloc(b, &d.c0, 2 * (size_t)g->n)) != GI_OK) return bail(st);
      d.c1 = d.c0 + g->n;
      const size_t nl = (size_t)std::max(1, b->lr_max[(size_t)t.graph]);
      if ((st = batch_alloc(b, &d.lr_acc, nl)) != GI_OK) return bail(st);
      if ((st = batch_alloc(b, &d.lr_cnt, nl)) != GI_OK) return bail(st);
    }
    // default size: one workgroup per 64K edges of work, power of two <= 64
    const double work = (double)std::max<int64_t>(g->m, g->n) * (d.alg == ALG_PR ? std::max(1, t.iters) : 1);
    int k = 1;
    while (k < 64 && (double)k * 65536.0 < (double)std::max<int64_t>(g->m, g->n)) k *= 2;
    b->k[i] = t.workgroups > 0 ? t.workgroups : k;
    b->est[i] = work / b->k[i];
  }
  if (dmem_get((void**)&b->d_graphs, sizeof(BatchGraph) * (size_t)ngraphs) != hipSuccess ||
      dmem_get((void**)&b->d_tasks, sizeof(BatchTask) * nt) != hipSuccess ||
      dmem_get((void**)&b->d_ctl, sizeof(TaskCtl) * nt) != hipSuccess ||
      dmem_get((void**)&b->d_err, sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(GI_ERR_OUT_OF_MEMORY, "batch allocation failed"));
  }
  for (size_t i = 0; i < nt; ++i) b->h_tasks[i].ctl = b->d_ctl + i;
  for (hipEvent_t* e : {&b->ev[0], &b->ev[1]})
    if (hipEventCreate(e) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(GI_ERR_DEVICE, "hipEventCreate failed"));
    }
  if (hipEventCreateWithFlags(&b->evw, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(GI_ERR_DEVICE, "hipEventCreate failed"));
  }
  if (hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(GI_ERR_DEVICE, "stream creation failed"));
  }
  if ((st = batch_plan(b)) != GI_OK) return bail(st);
  *out = b;
  return GI_OK;
}

static BatchArgs batch_args(const gi_batch* b, const int2* items, const int* wg_off) {
  BatchArgs a;
  a.graphs = b->d_graphs;
  a.tasks = b->d_tasks;
  a.items = items;
  a.wg_off = wg_off;
  a.error = b->d_err;
  a.spin_limit = b->spin_limit;
  a.lds_cap_e = b->cap_e;
  a.trace_cap = b->trace_cap;
  a.trace = b->d_trace;
  a.xcd_barrier = b->xcd_barrier;
  a.algs = b->algs;
  return a;
}

static gi_status batch_refresh_graphs(gi_batch* b) {
  std::vector<BatchGraph> hg;
  for (size_t i = 0; i < b->graphs.size(); ++i) hg.push_back(batch_graph(b->graphs[i], b->lay[i]));
  HIP_TRY(hipMemcpy(b->d_graphs, hg.data(), sizeof(BatchGraph) * hg.size(), hipMemcpyHostToDevice));
  return GI_OK;
}

static gi_status batch_check_error(gi_batch* b) {
  int err = 0;
  HIP_TRY(hipMemcpy(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (err == 1) return fail(GI_ERR_DEVICE, "batch barrier wait timed out");
  if (err == 3) return fail(GI_ERR_OVERFLOW, "batch SSSP: a distance reached UINT32_MAX");
  if (err) return fail(GI_ERR_DEVICE, "batch task exceeded its step bound");
  return GI_OK;
}

extern "C" gi_status gi_batch_launch(gi_batch* b, int32_t use_graph, void* stream) {
  if (!b) return fail(GI_ERR_INVALID_ARG, "NULL batch");
  if (b->launched) return fail(GI_ERR_INVALID_ARG, "batch already launched (gi_batch_wait first)");
  gi_status st = batch_refresh_graphs(b);
  if (st != GI_OK) return st;
  const int nt = (int)b->tasks.size();
  const BatchArgs a = batch_args(b, b->d_items, b->d_wg_off);
  if (use_graph) {
    if (!b->hx) {
      HIP_TRY(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal));
      const int lr = launch_batch(a, b->bt, b->grid, b->lds, b->d_ctl, nt, b->gstream);
      hipGraph_t gcap = nullptr;
      const hipError_t ce = hipStreamEndCapture(b->gstream, &gcap);
      if (lr != 0 || ce != hipSuccess) {
        if (gcap) (void)hipGraphDestroy(gcap);
        (void)hipGetLastError();
        return fail(GI_ERR_DEVICE, "batch graph capture failed");
      }
      b->hg = gcap;
      if (hipGraphInstantiate(&b->hx, b->hg, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        batch_drop_graph(b);
        return fail(GI_ERR_DEVICE, "batch graph instantiation failed");
      }
    }
    // the batch's stream waits for the work enqueued on `stream` so far
    HIP_TRY(hipEventRecord(b->evw, static_cast<hipStream_t>(stream)));
    HIP_TRY(hipStreamWaitEvent(b->gstream, b->evw, 0));
    HIP_TRY(hipEventRecord(b->ev[0], b->gstream));
    HIP_TRY(hipGraphLaunch(b->hx, b->gstream));
    HIP_TRY(hipEventRecord(b->ev[1], b->gstream));
  } else {
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipEventRecord(b->ev[0], s));
    LAUNCH_TRY(launch_batch(a, b->bt, b->grid, b->lds, b->d_ctl, nt, s));
    HIP_TRY(hipEventRecord(b->ev[1], s));
  }
  b->launched = true;
  return GI_OK;
}

extern "C" gi_status gi_batch_wait(gi_batch* b) {
  if (!b) return fail(GI_ERR_INVALID_ARG, "NULL batch");
  if (!b->launched) return fail(GI_ERR_INVALID_ARG, "batch not launched");
  b->launched = false;
  HIP_TRY(hipEventSynchronize(b->ev[1]));
  HIP_TRY(hipEventElapsedTime(&b->last_ms, b->ev[0], b->ev[1]));
  return batch_check_error(b);
}

extern "C" gi_status gi_batch_run(gi_batch* b, int32_t use_graph, void* stream) {
  gi_status st = gi_batch_launch(b, use_graph, stream);
  if (st != GI_OK) return st;
  return gi_batch_wait(b);
}

// Time one task alone on k workgroups (median of reps launches).
static gi_status batch_time_task(gi_batch* b, int t, int k, int reps, float* ms) {
  std::vector<int2> items((size_t)k);
  std::vector<int> off((size_t)k + 1);
  for (int r = 0; r < k; ++r) {
    items[(size_t)r] = make_int2(t, r);
    off[(size_t)r] = r;
  }
  off[(size_t)k] = k;
  BatchTask saved = b->h_tasks[(size_t)t];
  b->h_tasks[(size_t)t].k = k;
  HIP_TRY(hipMemcpy(b->d_tasks + t, &b->h_tasks[(size_t)t], sizeof(BatchTask), hipMemcpyHostToDevice));
  int2* di = nullptr;
  int* doff = nullptr;
  gi_status st = GI_OK;
  if (dmem_get((void**)&di, sizeof(int2) * (size_t)k) != hipSuccess ||
      dmem_get((void**)&doff, sizeof(int) * (size_t)(k + 1)) != hipSuccess) {
    (void)hipGetLastError();
    st = fail(GI_ERR_OUT_OF_MEMORY, "tuning buffers");
  }
  if (st == GI_OK && (hipMemcpy(di, items.data(), sizeof(int2) * (size_t)k, hipMemcpyHostToDevice) != hipSuccess ||
                      hipMemcpy(doff, off.data(), sizeof(int) * (size_t)(k + 1), hipMemcpyHostToDevice) != hipSuccess))
    st = fail(GI_ERR_DEVICE, "tuning upload failed");
  std::vector<float> times;
  const BatchArgs a = batch_args(b, di, doff);
  for (int rep = 0; rep < reps && st == GI_OK; ++rep) {
    float x = 0.0f;
    if (hipEventRecord(b->ev[0], nullptr) != hipSuccess ||
        launch_batch(a, b->bt, k, b->lds, b->d_ctl, (int)b->tasks.size(), nullptr) != 0 ||
        hipEventRecord(b->ev[1], nullptr) != hipSuccess ||
        hipEventSynchronize(b->ev[1]) != hipSuccess ||
        hipEventElapsedTime(&x, b->ev[0], b->ev[1]) != hipSuccess) {
      st = fail(GI_ERR_DEVICE, "tuning launch failed: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    if ((st = batch_check_error(b)) != GI_OK) break;
    times.push_back(x);
  }
  if (di) dmem_free(di);
  if (doff) dmem_free(doff);
  b->h_tasks[(size_t)t] = saved;
  if (hipMemcpy(b->d_tasks + t, &saved, sizeof(BatchTask), hipMemcpyHostToDevice) != hipSuccess && st == GI_OK)
    st = fail(GI_ERR_DEVICE, "tuning restore failed");
  if (st != GI_OK) return st;
  std::sort(times.begin(), times.end());
  *ms = times[times.size() / 2];
  return GI_OK;
}

// PageRank block size per graph at the current workgroup size: the graph's
// first PageRank task is timed alone, on its current workgroups, with each
// of kBatchCaps; the fastest stays.  Returns the chosen sizes.
static gi_status batch_tune_layouts(gi_batch* b, int32_t reps, std::vector<int>* caps) {
  gi_status st;
  caps->assign(b->graphs.size(), 0);
  for (size_t i = 0; i < b->graphs.size(); ++i) {
    int q = -1;
    for (size_t t = 0; t < b->tasks.size() && q < 0; ++t)
      if (b->tasks[t].algorithm == GI_ALG_PAGERANK && b->tasks[t].graph == (int32_t)i) q = (int)t;
    if (q < 0) continue;
    float best = 0.0f;
    int best_cap = 0;
    for (int cap : kBatchCaps) {
      if ((st = batch_set_layout(b, i, cap)) != GI_OK) return st;
      if ((st = batch_refresh_graphs(b)) != GI_OK) return st;
      float ms = 0.0f;
      if ((st = batch_time_task(b, q, std::max(1, b->k[(size_t)q]), reps, &ms)) != GI_OK) return st;
      if (best_cap == 0 || ms < best) {
        best = ms;
        best_cap = cap;
      }
    }
    if ((st = batch_set_layout(b, i, best_cap)) != GI_OK) return st;
    (*caps)[i] = best_cap;
  }
  return batch_refresh_graphs(b);
}

// Workgroups per task at the current workgroup size (see gi_batch_autotune).
static gi_status batch_tune_sizes(gi_batch* b, int32_t reps) {
  gi_status st;
  const int nt = (int)b->tasks.size();
  // one representative per (graph, algorithm, iterations) class
  std::vector<int> rep_of((size_t)nt, -1);
  std::vector<int> reps_list;
  for (int t = 0; t < nt; ++t) {
    const gi_task& x = b->tasks[(size_t)t];
    for (int q : reps_list) {
      const gi_task& y = b->tasks[(size_t)q];
      if (x.graph == y.graph && x.algorithm == y.algorithm &&
          (x.algorithm == GI_ALG_BFS ||
           (x.algorithm == GI_ALG_SSSP && x.sssp_delta == y.sssp_delta) ||
           (x.algorithm == GI_ALG_PAGERANK && x.iters == y.iters))) {
        rep_of[(size_t)t] = q;
        break;
      }
    }
    if (rep_of[(size_t)t] < 0) {
      rep_of[(size_t)t] = t;
      reps_list.push_back(t);
    }
  }
  std::vector<int> best_k((size_t)nt, 1), fast_k((size_t)nt, 1);
  std::vector<double> best_t((size_t)nt, 0.0), fast_t((size_t)nt, 0.0);
  for (int q : reps_list) {
    // sizes from the largest down: among the sizes within twice the fastest
    // time, the least workgroup-time (throughput); the sweep stops at the
    // first size slower than that, so a large task is never timed on a
    // handful of workgroups
    int kmax = 1;
    while (kmax * 2 <= std::min(256, b->max_grid)) kmax *= 2;
    double bw = 1e300, bt = 0.0, ft = 1e300;
    int bk = kmax, fk = kmax;
    for (int k = kmax; k >= 1; k /= 2) {
      float ms = 0.0f;
      if ((st = batch_time_task(b, q, k, reps, &ms)) != GI_OK) return st;
      if (ms < ft) {
        ft = ms;
        fk = k;
      }
      if ((double)ms > 2.0 * ft) break;
      if ((double)k * ms < bw) {
        bw = (double)k * ms;
        bk = k;
        bt = ms;
      }
    }
    if (bt > 2.0 * ft) {
      bk = fk;
      bt = ft;
    }
    best_k[(size_t)q] = bk;
    best_t[(size_t)q] = bt;
    fast_k[(size_t)q] = fk;
    fast_t[(size_t)q] = ft;
  }
  double total = 0.0;
  for (int t = 0; t < nt; ++t) {
    if (b->tasks[(size_t)t].workgroups > 0) continue;
    const int q = rep_of[(size_t)t];
    b->k[(size_t)t] = best_k[(size_t)q];
    b->est[(size_t)t] = best_t[(size_t)q];
    total += best_k[(size_t)q] * best_t[(size_t)q];
  }
  // a task longer than the balanced share of the grid sets the makespan:
  // give it its fastest size instead
  const double share = total / std::max(1, b->max_grid);
  for (int t = 0; t < nt; ++t) {
    if (b->tasks[(size_t)t].workgroups > 0) continue;
    const int q = rep_of[(size_t)t];
    if (b->est[(size_t)t] > share && fast_t[(size_t)q] < b->est[(size_t)t]) {
      b->k[(size_t)t] = fast_k[(size_t)q];
      b->est[(size_t)t] = fast_t[(size_t)q];
    }
  }
  return batch_plan(b);
}

// Median time of reps launches of the whole planned batch (stream 0).
static gi_status batch_time_all(gi_batch* b, int reps, float* ms) {
  const BatchArgs a = batch_args(b, b->d_items, b->d_wg_off);
  std::vector<float> times;
  for (int rep = 0; rep < reps; ++rep) {
    float x = 0.0f;
    HIP_TRY(hipEventRecord(b->ev[0], nullptr));
    LAUNCH_TRY(launch_batch(a, b->bt, b->grid, b->lds, b->d_ctl, (int)b->tasks.size(), nullptr));
    HIP_TRY(hipEventRecord(b->ev[1], nullptr));
    HIP_TRY(hipEventSynchronize(b->ev[1]));
    HIP_TRY(hipEventElapsedTime(&x, b->ev[0], b->ev[1]));
    gi_status st = batch_check_error(b);
    if (st != GI_OK) return st;
    times.push_back(x);
  }
  std::sort(times.begin(), times.end());
  *ms = times[times.size() / 2];
  return GI_OK;
}

// Critical-path refinement of a timed plan: the batch ends when its last
// task ends, so the tasks that finish in the last tenth of the run and take
// at least a third of it are resized: first to twice their workgroups (up
// to 256), else to half (a task whose steps are bound by its own barriers
// can finish sooner on fewer workgroups); tasks with fixed workgroups keep
// them.  The plan is rebuilt with every task's measured duration as its
// estimate, and a resize is kept only if the whole batch gets at least 1%
// faster.  At most four rounds.
static gi_status batch_refine_critical(gi_batch* b, int reps) {
  gi_status st;
  const size_t nt = b->tasks.size();
  const int kmax = std::min(256, b->max_grid);
  float ms = 0.0f;
  if ((st = batch_time_all(b, reps, &ms)) != GI_OK) return st;
  for (int round = 0; round < 4; ++round) {
    // durations of the last timed launch of the current plan
    std::vector<TaskCtl> c(nt);
    HIP_TRY(hipMemcpy(c.data(), b->d_ctl, sizeof(TaskCtl) * nt, hipMemcpyDeviceToHost));
    long long t0 = c[0].t_begin, t1 = c[0].t_end;
    for (const TaskCtl& x : c) {
      t0 = std::min(t0, x.t_begin);
      t1 = std::max(t1, x.t_end);
    }
    const double span = (double)(t1 - t0);
    if (!(span > 0.0)) return GI_OK;
    const std::vector<int> k_old = b->k;
    const std::vector<double> est_old = b->est;
    std::vector<double> dur(nt);
    std::vector<char> crit(nt, 0);
    bool any = false;
    for (size_t i = 0; i < nt; ++i) {
      const double d = std::max(0.0, (double)(c[i].t_end - c[i].t_begin));
      dur[i] = d / (double)b->clock_khz;  // ms
      crit[i] = b->tasks[i].workgroups == 0 && (double)(c[i].t_end - t0) > 0.9 * span &&
                d > span / 3.0;
      any = any || crit[i];
    }
    if (!any) return GI_OK;
    bool kept = false;
    for (int dir : {2, -2}) {  // double, else halve
      bool changed = false;
      for (size_t i = 0; i < nt; ++i) {
        b->k[i] = k_old[i];
        b->est[i] = dur[i];
        if (!crit[i]) continue;
        const int k2 = dir > 0 ? std::min(kmax, 2 * k_old[i]) : std::max(1, k_old[i] / 2);
        if (k2 == k_old[i]) continue;
        b->k[i] = k2;
        b->est[i] = dur[i] * (double)k_old[i] / (double)k2;
        changed = true;
      }
      if (!changed) continue;
      float ms2 = 0.0f;
      if ((st = batch_plan(b)) != GI_OK) return st;
      if ((st = batch_time_all(b, reps, &ms2)) != GI_OK) return st;
      if (ms2 < 0.99f * ms) {
        ms = ms2;
        kept = true;
        break;
      }
    }
    if (!kept) {
      b->k = k_old;
      b->est = est_old;
      return batch_plan(b);
    }
  }
  return GI_OK;
}

extern "C" gi_status gi_batch_autotune(gi_batch* b, int32_t reps) {
  if (!b || reps < 1) return fail(GI_ERR_INVALID_ARG, "bad autotune arguments");
  if (b->launched) return fail(GI_ERR_INVALID_ARG, "batch launch in flight (gi_batch_wait first)");
  gi_status st = batch_refresh_graphs(b);
  if (st != GI_OK) return st;
  HIP_TRY(hipDeviceSynchronize());
  const std::vector<int> k0 = b->k;
  const std::vector<double> e0 = b->est;
  int best_bt = b->bt;
  float best_ms = 0.0f;
  std::vector<int> best_k;
  std::vector<double> best_est;
  std::vector<int> best_caps, caps;
  bool best_xcd = true;
  for (int bt : {256, 512, 1024}) {
    if (b->bt_pinned && bt != b->bt) continue;
    b->k = k0;
    b->est = e0;
    if ((st = batch_set_bt(b, bt)) != GI_OK) return st;
    b->xcd_local = true;
    if ((st = batch_tune_layouts(b, reps, &caps)) != GI_OK) return st;
    if ((st = batch_tune_sizes(b, reps)) != GI_OK) return st;
    const std::vector<int> kt = b->k;
    const std::vector<double> et = b->est;
    // the size rule picks per class in isolation; tasks running together
    // also compete, so the whole batch is timed with the chosen sizes capped
    // at 64, 32 and 16 workgroups as well
    for (int cap : {1 << 30, 64, 32, 16}) {
      std::vector<int> kc = kt;
      std::vector<double> ec = et;
      bool changed = cap == (1 << 30);
      for (size_t i = 0; i < kc.size(); ++i) {
        if (b->tasks[i].workgroups > 0 || kc[i] <= cap) continue;
        ec[i] = et[i] * (double)kc[i] / (double)cap;
        kc[i] = cap;
        changed = true;
      }
      if (!changed) continue;
      for (bool xl : {true, false}) {
        b->xcd_local = xl;
        b->k = kc;
        b->est = ec;
        if ((st = batch_plan(b)) != GI_OK) return st;
        const std::vector<int> kp = b->k;  // after the plan's clamp to the grid
        float ms = 0.0f;
        if ((st = batch_time_all(b, reps, &ms)) != GI_OK) return st;
        if (best_k.empty() || ms < best_ms) {
          best_ms = ms;
          best_bt = bt;
          best_xcd = xl;
          best_k = kp;
          best_est = ec;
          best_caps = caps;
        }
      }
    }
  }
  if ((st = batch_set_bt(b, best_bt)) != GI_OK) return st;
  for (size_t i = 0; i < best_caps.size(); ++i)
    if (best_caps[i] > 0 && (st = batch_set_layout(b, i, best_caps[i])) != GI_OK) return st;
  if ((st = batch_refresh_graphs(b)) != GI_OK) return st;
  b->xcd_local = best_xcd;
  b->k = best_k;
  b->est = best_est;
  if ((st = batch_plan(b)) != GI_OK) return st;
  return batch_refine_critical(b, reps);
}

extern "C" gi_status gi_batch_pr_block_edges(const gi_batch* b, int32_t* edges_per_block) {
  if (!b || !edges_per_block) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  for (size_t i = 0; i < b->lay.size(); ++i)
    edges_per_block[i] = b->lay[i].table ? b->lay[i].cap_e : 0;
  return GI_OK;
}

extern "C" gi_status gi_batch_set_threads(gi_batch* b, int32_t threads) {
  if (!b) return fail(GI_ERR_INVALID_ARG, "NULL batch");
  if (b->launched) return fail(GI_ERR_INVALID_ARG, "batch launch in flight (gi_batch_wait first)");
  if (threads == 0) {
    b->bt_pinned = false;
    return GI_OK;
  }
  gi_status st = batch_set_bt(b, threads);
  if (st != GI_OK) return st;
  b->bt_pinned = true;
  return batch_plan(b);
}

extern "C" gi_status gi_batch_set_trace(gi_batch* b, int32_t cap) {
  if (!b || cap < 0 || cap > (1 << 20)) return fail(GI_ERR_INVALID_ARG, "bad trace capacity");
  if (b->launched) return fail(GI_ERR_INVALID_ARG, "batch launch in flight (gi_batch_wait first)");
  HIP_TRY(hipDeviceSynchronize());
  if (b->d_trace) dmem_free(b->d_trace);
  b->d_trace = nullptr;
  b->trace_cap = 0;
  if (cap > 0) {
    const size_t cnt = b->tasks.size() * (size_t)cap * 2;
    if (dmem_get((void**)&b->d_trace, sizeof(long long) * cnt) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GI_ERR_OUT_OF_MEMORY, "trace allocation failed");
    }
    HIP_TRY(hipMemset(b->d_trace, 0, sizeof(long long) * cnt));
    b->trace_cap = cap;
  }
  batch_drop_graph(b);  // the captured launch holds the old arguments
  return GI_OK;
}

extern "C" gi_status gi_batch_get_trace(const gi_batch* b, int32_t task, int64_t* start_ns,
                                        int32_t* pull, int64_t* frontier, int32_t cap,
                                        int32_t* count) {
  if (!b || !count || task < 0 || task >= (int32_t)b->tasks.size() || cap < 0)
    return fail(GI_ERR_INVALID_ARG, "bad trace arguments");
  *count = 0;
  if (b->trace_cap == 0) return GI_OK;
  int levels = 0;
  HIP_TRY(hipMemcpy(&levels, &b->d_ctl[task].levels, sizeof(int), hipMemcpyDeviceToHost));
  const int nrec = std::min(levels + 1, b->trace_cap);
  std::vector<long long> rec((size_t)nrec * 2);
  HIP_TRY(hipMemcpy(rec.data(), b->d_trace + (size_t)task * b->trace_cap * 2,
                    sizeof(long long) * rec.size(), hipMemcpyDeviceToHost));
  const int n = std::min(nrec, cap);
  for (int i = 0; i < n; ++i) {
    if (start_ns)
      start_ns[i] = (int64_t)((double)(rec[2 * i] - rec[0]) * 1e6 / (double)b->clock_khz);
    if (pull) pull[i] = (int32_t)((unsigned long long)rec[2 * i + 1] >> 62);
    if (frontier) frontier[i] = rec[2 * i + 1] & ((1ll << 62) - 1);
  }
  *count = n;
  return GI_OK;
}

extern "C" gi_status gi_batch_set_placement(gi_batch* b, int32_t xcd_local) {
  if (!b || (xcd_local != 0 && xcd_local != 1)) return fail(GI_ERR_INVALID_ARG, "bad placement");
  if (b->launched) return fail(GI_ERR_INVALID_ARG, "batch launch in flight (gi_batch_wait first)");
  b->xcd_local = xcd_local != 0;
  return batch_plan(b);
}

extern "C" gi_status gi_batch_set_barrier_scope(gi_batch* b, int32_t scope) {
  if (!b || (scope != GI_BARRIER_AGENT && scope != GI_BARRIER_XCD))
    return fail(GI_ERR_INVALID_ARG, "bad barrier scope");
  if (b->launched) return fail(GI_ERR_INVALID_ARG, "batch launch in flight (gi_batch_wait first)");
  b->xcd_barrier = scope == GI_BARRIER_XCD ? 1 : 0;
  batch_drop_graph(b);  // the captured launch holds the old arguments
  return GI_OK;
}

extern "C" gi_status gi_batch_get_barrier_scope(const gi_batch* b, int32_t* scope) {
  if (!b || !scope) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  *scope = b->xcd_barrier ? GI_BARRIER_XCD : GI_BARRIER_AGENT;
  return GI_OK;
}

extern "C" gi_status gi_batch_get_placement(const gi_batch* b, int32_t* xcd_local) {
  if (!b || !xcd_local) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  *xcd_local = b->xcd_local ? 1 : 0;
  return GI_OK;
}

extern "C" gi_status gi_batch_get_threads(const gi_batch* b, int32_t* threads) {
  if (!b || !threads) return fail(GI_ERR_INVALID_ARG, "NULL argument");
  *threads = b->bt;
  return GI_OK;
}

extern "C" gi_status gi_batch_task_counters(const gi_batch* b, int64_t* edges, float* barrier_ms) {
  if (!b || (!edges && !barrier_ms)) return fail(GI_ERR_INVALID_ARG, "bad batch counter arguments");
  if (b->launched) return fail(GI_ERR_INVALID_ARG, "batch launch in flight (gi_batch_wait first)");
  const size_t nt = b->tasks.size();
  std::vector<TaskCtl> c(nt);
  HIP_TRY(hipMemcpy(c.data(), b->d_ctl, sizeof(TaskCtl) * nt, hipMemcpyDeviceToHost));
  for (size_t i = 0; i < nt; ++i) {
    if (edges) edges[i] = (int64_t)c[i].relaxed;
    if (barrier_ms)
      barrier_ms[i] = (float)((double)c[i].bar_ticks / (double)std::max(1, b->k[i]) /
                              (double)b->clock_khz);
  }
  return GI_OK;
}

extern "C" gi_status gi_batch_info(const gi_batch* b, float* last_ms, int32_t* grid,
                                   int32_t* workgroups, int32_t* levels, float* task_ms) {
  if (!b) return fail(GI_ERR_INVALID_ARG, "NULL batch");
  if (last_ms) *last_ms = b->last_ms;
  if (grid) *grid = b->grid;
  const size_t nt = b->tasks.size();
  if (workgroups)
    for (size_t i = 0; i < nt; ++i) workgroups[i] = b->k[i];
  if (levels || task_ms) {
    std::vector<TaskCtl> c(nt);
    HIP_TRY(hipMemcpy(c.data(), b->d_ctl, sizeof(TaskCtl) * nt, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < nt; ++i) {
      if (levels) levels[i] = c[i].levels;
      if (task_ms) task_ms[i] = (float)((double)(c[i].t_end - c[i].t_begin) / (double)b->clock_khz);
    }
  }
  return GI_OK;
}
