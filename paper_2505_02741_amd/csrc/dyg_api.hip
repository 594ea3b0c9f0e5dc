// C ABI of libdygrass: context life cycle, host-side validation of the
// initial graphs, device memory management and the per-batch launch sequence.
#include "dygrass.h"
#include "dyg_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

using dyg::AddRec;
using dyg::BatchArgs;
using dyg::BatchCtl;
using dyg::DevGraph;
using dyg::Ent;
using dyg::HashSlot;
using dyg::Row;
using dyg::RowHdr;
using dyg::kInline;
using dyg::kInlineOff;
using dyg::Pair;

namespace {

// Growable device buffer.
// Staging buffers grow to the next power of two (at least 64 KiB): batches of
// varying size then reallocate rarely (freeing device memory waits for the
// device).
size_t grown_size(size_t need) {
  size_t want = size_t(1) << 16;
  while (want < need) want <<= 1;
  return want;
}

struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool ensure(size_t need) {
    if (need <= bytes && p) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    const size_t want = grown_size(need);
    if (hipMalloc(&p, want) != hipSuccess) {
      p = nullptr;
      return false;
    }
    bytes = want;
    return true;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Growable pinned host buffer.
struct HBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool ensure(size_t need) {
    if (need <= bytes && p) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    const size_t want = grown_size(need);
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      return false;
    }
    bytes = want;
    return true;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
};

constexpr uint32_t kMaxWalkersHost = DYG_MAX_WALKERS;

uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Quantised weight: round-half-even(w / w_ref * 2^Q), clamped to [1, 2^32-1].
uint32_t quantize_host(double w, double w_ref, int Q) {
  const double y = std::nearbyint((w / w_ref) * std::ldexp(1.0, Q));
  if (!(y >= 1.0)) return 1u;
  if (y > 4294967295.0) return 4294967295u;
  return static_cast<uint32_t>(y);
}

uint32_t slack_slots(uint32_t len, double slack) {
  const double extra = std::ceil(static_cast<double>(len) * slack);
  return static_cast<uint32_t>(std::max(2.0, extra));
}

// Host image of one adjacency (used at init and by compaction).
struct HostAdj {
  std::vector<Row> rows;
  std::vector<Ent> ent;                 // pool
  std::vector<double> w;                // pool weights
  std::vector<unsigned long long> tree;  // weight tree levels 1.. of long segments
  std::vector<double> rinl;             // 1/w of inline entries, kInline per row
  std::vector<double> winl;             // weights of inline entries, kInline per row
};

// Weight tree of one long segment of len entries (layout in dyg_internal.h):
// level 0 into l0[0 .. round_fan(len)), levels 1.. into tb.
void build_tree_host(const Ent* seg, uint32_t len, unsigned long long* tb) {
  const uint32_t K = dyg::tree_top(len);
  std::vector<unsigned long long> raw(len), up;
  unsigned long long total = 0;
  for (uint32_t i = 0; i < len; ++i) {
    raw[i] = seg[i].qw;
    total += seg[i].qw;
  }
  for (uint32_t l = 0; l <= K; ++l) {  // level 0 is summed but not stored
    const uint32_t n = static_cast<uint32_t>(raw.size());
    unsigned long long* dst = l == 0 ? nullptr : tb + dyg::tree_base(len, l);
    up.assign((n + dyg::kFan - 1) / dyg::kFan, 0ull);
    unsigned long long run = 0;
    for (uint32_t i = 0; i < n; ++i) {
      run += raw[i];
      if (dst) dst[i] = run;
      if (i % dyg::kFan == dyg::kFan - 1 || i == n - 1) {
        up[i / dyg::kFan] = run;
        run = 0;
      }
    }
    if (dst) {
      for (uint32_t i = n; i < dyg::round_fan(n); ++i) dst[i] = dyg::kTreePad;
      if (l == K) dst[dyg::kFan - 1] = total;
    }
    raw.swap(up);
  }
}

// The inline copy of a long segment's top tree block in its row (layout in
// dyg_internal.h), when the top level has at most kInlineTop values.
void inline_top_host(Row& row, uint32_t len, const unsigned long long* tb) {
  if (!dyg::top_inline(len)) return;
  const uint32_t K = dyg::tree_top(len);
  const uint32_t n = dyg::tree_n(len, K);
  const unsigned long long* top = tb + dyg::tree_base(len, K);
  unsigned long long words[kInline];
  std::memcpy(words, row.inl, sizeof(words));
  for (uint32_t j = 0; j + 1 < n; ++j) words[j] = top[j];
  words[kInline - 1] = top[dyg::kFan - 1];
  std::memcpy(row.inl, words, sizeof(words));
}

// Pool slots a long segment of len entries starts at: a multiple of kHubAlign.
uint64_t hub_aligned(uint64_t off) {
  return (off + dyg::kHubAlign - 1) / dyg::kHubAlign * dyg::kHubAlign;
}

}  // namespace

// Working memory of dyg_apply_batch_dev_static: one array in the library's
// code object, so every GPU the library runs on holds its own copy for the
// life of the process.  Host code never uses the array's name as an address
// (on the host it names a stand-in, not device memory): the device address
// of each GPU's copy comes from hipGetSymbolAddress, taken once per device
// at dyg_init with that device current.
constexpr size_t kStaticScratchBytes = DYG_STATIC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

struct StaticScratch {
  std::mutex mu;
  void* addr[kMaxDevices] = {};           // device address of each GPU's copy
  hipError_t status[kMaxDevices] = {};    // result of the address lookup
  bool looked_up[kMaxDevices] = {};
  const dyg_ctx* owner[kMaxDevices] = {};  // context whose batch uses it until dyg_sync
};

StaticScratch& static_scratch() {
  static StaticScratch s;
  return s;
}

// Device address of `dev`'s copy of the array (dev must be current).
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  StaticScratch& s = static_scratch();
  std::lock_guard<std::mutex> lock(s.mu);
  if (!s.looked_up[dev]) {
    void* p = nullptr;
    s.status[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    s.addr[dev] = s.status[dev] == hipSuccess ? p : nullptr;
    s.looked_up[dev] = true;
  }
  return s.addr[dev];
}

}  // namespace

struct dyg_ctx {
  uint32_t n = 0;
  dyg_params params{};
  double w_ref = 1.0;
  int Q = 24;
  bool has_K = false;
  uint64_t uid_base = 0;
  uint64_t batches = 0;
  uint64_t compactions = 0;
  hipStream_t stream = nullptr;
  DevGraph G, H;
  BatchCtl* ctl = nullptr;
  BatchArgs* dargs = nullptr;  // device copy of the current batch's arguments
  // DYG_FLAG_GRAPH: instantiated launch sequences by size class
  std::map<std::tuple<uint64_t, uint64_t, uint64_t, uint32_t, uint32_t, bool, bool, uint32_t, uint32_t>,
           hipGraphExec_t>
      graphs;
  BatchArgs* hargs = nullptr;  // pinned host staging of the same
  BatchCtl* hctl = nullptr;    // pinned copy of ctl, written at the end of each batch
  hipEvent_t done_ev = nullptr;  // recorded after that copy
  const BatchArgs** dargv = nullptr;  // device array {dargs}: a launch of one batch
  uint64_t pool_top[2] = {0, 0};  // host mirror after the last sync
  bool broken = false;
  int pending_status = DYG_OK;
  bool async_inflight = false;
  uint64_t async_nu = 0;
  // DYG_FLAG_TIMING, DYG_FLAG_TIMING_WALK, DYG_FLAG_AUTOTUNE
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // batch begin, walk begin/end, batch end
  bool timed_pending = false;
  uint64_t walk_launches = 0;
  double walk_ms_total = 0.0, walk_ms_last = 0.0, batch_ms_last = 0.0;
  // batch staging
  DBuf iu, iv, iw, du, dv, s, L, ins_qw, ins_rinv, in_h, res, ubytes, wrec, wofs, hadd, hash;
  DBuf fb_list;
  DBuf touched_rows[2], touched_k[2], touched_need[2], add_keep[2], dirty_rows[2], wide_rows[2],
      wmerge[2], dirty_chunk0[2], dirty_small[2];
  DBuf hash2;
  DBuf qcount, qofs, qtile, items, wres;  // batched form
  DBuf tstate, tcount;                     // batched form, head/tail schedule
  uint32_t cus = 256;                      // compute units of the device
  uint32_t walk_blocks_per_cu = 8;         // persistent walk grid = cus x this
  uint32_t refill_min = 1;                 // idle lanes that trigger a refill
  uint32_t updates_per_wave = 4;           // range walk (0 = work queue)
  uint32_t lockstep = 0;                   // batched form walks as the plain form does
  uint32_t tail_lanes = 8;                 // head/tail schedule (0 = off)
  bool has_hubs = false;                   // some row longer than kHub (walk kernel choice)
  double pool_frac[2] = {0.0, 0.0};        // share of G0 / H0 rows held in the pool (walk kernel choice)
  // DYG_FLAG_AUTOTUNE: candidate being tried (-1 = done), best score so far
  int tune_next = -1;
  int tune_best = -1;
  double tune_best_score = 0.0;
  unsigned long long tune_steps0 = 0;
  bool last_graph = false;  // the batch enqueued last ran as a captured graph
  HBuf pin_in, pin_out;
  uint32_t h_lo = 0, h_hi = ~0u;   // H addition slots of the phase 4 in progress (repairs)
  int device = 0;                  // the GPU the context lives on
  void* static_scratch = nullptr;  // that GPU's copy of the static working memory
  bool static_inflight = false;    // the batch in flight uses it
};

namespace {

int fail_hip(hipError_t e) { return e == hipErrorOutOfMemory ? DYG_E_NOMEM : DYG_E_DEVICE; }

void free_graph(DevGraph& X) {
  if (X.rows) (void)hipFree(X.rows);
  if (X.ent) (void)hipFree(X.ent);
  if (X.prinv) (void)hipFree(X.prinv);
  if (X.w) (void)hipFree(X.w);
  if (X.pending) (void)hipFree(X.pending);
  if (X.tree) (void)hipFree(X.tree);
  if (X.mark) (void)hipFree(X.mark);
  if (X.rinl) (void)hipFree(X.rinl);
  if (X.winl) (void)hipFree(X.winl);
  X = DevGraph{};
}

// Upload a host adjacency into freshly allocated device arrays with pool
// capacity `pool_cap` (>= ent.size()).
int upload_graph(DevGraph& X, uint32_t n, const HostAdj& A, uint64_t pool_cap,
                 hipStream_t st) {
  DevGraph Y;
  Y.pool_cap = pool_cap;
  hipError_t e = hipSuccess;
  if ((e = hipMalloc(&Y.rows, sizeof(Row) * std::max<uint64_t>(n, 1))) != hipSuccess ||
      (e = hipMalloc(&Y.ent, sizeof(Pair) * std::max<uint64_t>(pool_cap, 1))) != hipSuccess ||
      (e = hipMalloc(&Y.prinv, sizeof(double) * std::max<uint64_t>(pool_cap, 1))) != hipSuccess ||
      (e = hipMalloc(&Y.w, sizeof(double) * std::max<uint64_t>(pool_cap, 1))) != hipSuccess ||
      (e = hipMalloc(&Y.pending, sizeof(uint32_t) * std::max<uint64_t>(n, 1))) != hipSuccess ||
      (e = hipMalloc(&Y.tree, sizeof(unsigned long long) * (pool_cap / 4 + dyg::kFan))) !=
          hipSuccess ||
      (e = hipMalloc(&Y.mark, sizeof(uint32_t) * std::max<uint64_t>(n, 1))) != hipSuccess ||
      (e = hipMalloc(&Y.rinl, sizeof(double) * kInline * std::max<uint64_t>(n, 1))) !=
          hipSuccess ||
      (e = hipMalloc(&Y.winl, sizeof(double) * kInline * std::max<uint64_t>(n, 1))) !=
          hipSuccess) {
    free_graph(Y);
    return fail_hip(e);
  }
  // pool entries go up as (neighbour, weight) pairs and a 1/w array
  std::vector<Pair> pairs(A.ent.size());
  std::vector<double> prinv(A.ent.size());
  for (size_t i = 0; i < A.ent.size(); ++i) {
    pairs[i] = Pair{A.ent[i].nbr, A.ent[i].qw};
    prinv[i] = A.ent[i].rinv;
  }
  if ((e = hipMemcpyAsync(Y.rows, A.rows.data(), sizeof(Row) * n, hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (!pairs.empty() &&
       (e = hipMemcpyAsync(Y.ent, pairs.data(), sizeof(Pair) * pairs.size(),
                           hipMemcpyHostToDevice, st)) != hipSuccess) ||
      (!prinv.empty() &&
       (e = hipMemcpyAsync(Y.prinv, prinv.data(), sizeof(double) * prinv.size(),
                           hipMemcpyHostToDevice, st)) != hipSuccess) ||
      (!A.w.empty() &&
       (e = hipMemcpyAsync(Y.w, A.w.data(), sizeof(double) * A.w.size(), hipMemcpyHostToDevice,
                           st)) != hipSuccess) ||
      (!A.tree.empty() &&
       (e = hipMemcpyAsync(Y.tree, A.tree.data(), sizeof(unsigned long long) * A.tree.size(),
                           hipMemcpyHostToDevice, st)) != hipSuccess) ||
      (e = hipMemcpyAsync(Y.rinl, A.rinl.data(), sizeof(double) * A.rinl.size(),
                          hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(Y.winl, A.winl.data(), sizeof(double) * A.winl.size(),
                          hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemsetAsync(Y.pending, 0, sizeof(uint32_t) * n, st)) != hipSuccess ||
      (e = hipMemsetAsync(Y.mark, 0, sizeof(uint32_t) * n, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    free_graph(Y);
    return fail_hip(e);
  }
  free_graph(X);
  X = Y;
  return DYG_OK;
}

// Lay out the rows for the given per-row live lists: at most kInline entries
// inside the row, longer lists in a pool segment with slack.
// A long segment (more than kHub entries) starts at a multiple of kHubAlign
// and owns a multiple of kFan slots, as its weight tree needs.
uint32_t segment_cap(uint32_t len, double slack) {
  const uint32_t cap = len + slack_slots(len, slack);
  return len > dyg::kHub ? dyg::round_fan(cap) : (cap + 1u) & ~1u;  // even: two pairs per load
}

void layout(HostAdj& A, uint32_t n, const std::vector<uint64_t>& start,
            const std::vector<Ent>& live_ent, const std::vector<double>& live_w, double slack) {
  A.rows.assign(n, Row{});
  A.rinl.assign(static_cast<size_t>(n) * kInline, 0.0);
  A.winl.assign(static_cast<size_t>(n) * kInline, 0.0);
  A.tree.clear();
  uint64_t total = 0;
  bool hubs = false;
  for (uint32_t u = 0; u < n; ++u) {
    const uint32_t len = static_cast<uint32_t>(start[u + 1] - start[u]);
    if (len <= kInline) continue;
    if (len > dyg::kHub) {
      total = hub_aligned(total);
      hubs = true;
    }
    total += segment_cap(len, slack);
  }
  A.ent.assign(total, Ent{0, 0, 0.0});
  A.w.assign(total, 0.0);
  if (hubs) {
    A.tree.assign(total / 4 + dyg::kFan, dyg::kTreePad);
  }
  uint64_t off = 0;
  for (uint32_t u = 0; u < n; ++u) {
    const uint32_t len = static_cast<uint32_t>(start[u + 1] - start[u]);
    if (len <= kInline) {
      A.rows[u].h = RowHdr{kInlineOff, len, kInline, 0};
      for (uint32_t i = 0; i < len; ++i) {
        const Ent& x = live_ent[start[u] + i];
        A.rows[u].inl[i] = Pair{x.nbr, x.qw};
        A.rinl[static_cast<size_t>(u) * kInline + i] = x.rinv;
        A.winl[static_cast<size_t>(u) * kInline + i] = live_w[start[u] + i];
      }
      continue;
    }
    if (len > dyg::kHub) off = hub_aligned(off);
    const uint32_t cap = segment_cap(len, slack);
    A.rows[u].h = RowHdr{static_cast<uint32_t>(off), len, cap, 0};
    std::copy(live_ent.begin() + start[u], live_ent.begin() + start[u + 1], A.ent.begin() + off);
    std::copy(live_w.begin() + start[u], live_w.begin() + start[u + 1], A.w.begin() + off);
    if (len > dyg::kHub) {
      build_tree_host(&A.ent[off], len, &A.tree[off / 4]);
      inline_top_host(A.rows[u], len, &A.tree[off / 4]);
    }
    off += cap;
  }
}

// Pool capacity for `used` live slots of a graph with n vertices: as much
// again for growth plus room for every vertex to outgrow its inline entries
// (a compaction is a host round trip; HBM is plentiful).
uint64_t pool_capacity_for(uint64_t used, uint32_t n, uint32_t flags) {
  if (flags & DYG_FLAG_LEAN_POOLS) return used + 64;
  return 2 * used + 8ull * n + 65536;
}

// Read one device graph back into per-row live lists.
int download_live(const DevGraph& X, uint32_t n, uint64_t used, std::vector<uint64_t>& start,
                  std::vector<Ent>& live_ent, std::vector<double>& live_w, hipStream_t st) {
  std::vector<Row> rows(n);
  std::vector<Pair> pairs(used);
  std::vector<double> w(used), prinv(used), winl(static_cast<size_t>(n) * kInline),
      rinl(static_cast<size_t>(n) * kInline);
  hipError_t e;
  if ((e = hipMemcpyAsync(rows.data(), X.rows, sizeof(Row) * n, hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(rinl.data(), X.rinl, sizeof(double) * rinl.size(),
                          hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipMemcpyAsync(winl.data(), X.winl, sizeof(double) * winl.size(),
                          hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (used && (e = hipMemcpyAsync(pairs.data(), X.ent, sizeof(Pair) * used,
                                   hipMemcpyDeviceToHost, st)) != hipSuccess) ||
      (used && (e = hipMemcpyAsync(prinv.data(), X.prinv, sizeof(double) * used,
                                   hipMemcpyDeviceToHost, st)) != hipSuccess) ||
      (used && (e = hipMemcpyAsync(w.data(), X.w, sizeof(double) * used, hipMemcpyDeviceToHost,
                                   st)) != hipSuccess) ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return fail_hip(e);
  start.assign(n + 1, 0);
  live_ent.clear();
  live_w.clear();
  for (uint32_t u = 0; u < n; ++u) {
    const RowHdr r = rows[u].h;
    const bool inl = r.off == kInlineOff;
    for (uint32_t i = 0; i < r.len; ++i) {
      const size_t k = static_cast<size_t>(u) * kInline + i;
      const Ent x = inl ? Ent{rows[u].inl[i].nbr, rows[u].inl[i].qw, rinl[k]}
                        : Ent{pairs[r.off + i].nbr, pairs[r.off + i].qw, prinv[r.off + i]};
      if (x.qw == 0u) continue;
      live_ent.push_back(x);
      live_w.push_back(inl ? winl[static_cast<size_t>(u) * kInline + i] : w[r.off + i]);
    }
    start[u + 1] = live_ent.size();
  }
  return DYG_OK;
}

int sync_ctl_host(dyg_ctx* c, BatchCtl& out) {
  hipError_t e = hipMemcpyAsync(&out, c->ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_hip(e);
  c->pool_top[0] = out.pool_top[0];
  c->pool_top[1] = out.pool_top[1];
  return DYG_OK;
}

// Wait for the batch enqueued last and read the control block it copied back.
int finish_ctl(dyg_ctx* c, BatchCtl& out) {
  const hipError_t e = hipEventSynchronize(c->done_ev);
  if (e != hipSuccess) return fail_hip(e);
  out = *c->hctl;
  c->pool_top[0] = out.pool_top[0];
  c->pool_top[1] = out.pool_top[1];
  c->has_hubs = c->has_hubs || out.hubs != 0;
  return DYG_OK;
}

// Rewrite graph `which` without tombstones into a pool of at least
// `min_cap` slots.
int compact_graph(dyg_ctx* c, int which, uint64_t min_cap) {
  DevGraph& X = which ? c->H : c->G;
  BatchCtl ctl;
  int rc = sync_ctl_host(c, ctl);
  if (rc) return rc;
  std::vector<uint64_t> start;
  std::vector<Ent> le;
  std::vector<double> lw;
  rc = download_live(X, c->n, ctl.pool_top[which], start, le, lw, c->stream);
  if (rc) return rc;
  HostAdj A;
  layout(A, c->n, start, le, lw, c->params.slack);
  const uint64_t cap =
      std::max<uint64_t>(pool_capacity_for(A.ent.size(), c->n, c->params.flags), min_cap);
  if (cap >= (1ull << 32)) return DYG_E_NOMEM;
  rc = upload_graph(X, c->n, A, cap, c->stream);
  if (rc) return rc;
  ctl.pool_top[which] = A.ent.size();
  hipError_t e = hipMemcpyAsync(&c->ctl->pool_top[which], &ctl.pool_top[which],
                                sizeof(unsigned long long), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_hip(e);
  c->pool_top[which] = A.ent.size();
  c->compactions++;
  return DYG_OK;
}

int check_params(const dyg_params* p) {
  if (!p) return DYG_E_INVALID_ARG;
  if (p->Q < 1 || p->Q > 31 || p->s_default > DYG_MAX_WALKERS ||
      p->L_default > DYG_MAX_STEPS || p->dead_end > 1 || std::isnan(p->K) ||
      !(p->w_ref >= 0.0) || std::isinf(p->w_ref) || !(p->slack >= 0.0) ||
      std::isinf(p->slack))
    return DYG_E_INVALID_ARG;
  // the autotuner scores one walk launch per batch; a two-stage batch has two
  if ((p->flags & DYG_FLAG_TWO_STAGE) && (p->flags & DYG_FLAG_AUTOTUNE)) return DYG_E_INVALID_ARG;
  return DYG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------

namespace dyg {

// Checks of a graph given as CSR (dyg_init's G0, dyg_initial_sparsifier's
// input): n in range, rowptr from 0 and non-decreasing, every row in
// ascending neighbour order with ids in range, no self loop, weights
// positive and finite with a finite 1/w, and the graph symmetric with equal
// weights both ways.  *wmax = the largest weight.
int validate_csr(uint32_t n, const uint64_t* rowptr, const uint32_t* col, const double* w,
                 double* wmax) {
  if (n == 0 || n >= (1u << 31) || !rowptr) return DYG_E_INVALID_ARG;
  const uint64_t nnz = rowptr[n];
  if (rowptr[0] != 0 || (nnz && (!col || !w))) return DYG_E_INVALID_ARG;
  double wm = 0.0;
  for (uint32_t u = 0; u < n; ++u) {
    if (rowptr[u + 1] < rowptr[u]) return DYG_E_INVALID_ARG;
    for (uint64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
      if (col[k] >= n) return DYG_E_VERTEX_RANGE;
      if (col[k] == u) return DYG_E_SELF_LOOP;
      if (!(w[k] > 0.0) || std::isinf(w[k]) || std::isinf(1.0 / w[k])) return DYG_E_BAD_WEIGHT;
      if (k > rowptr[u] && col[k] <= col[k - 1]) return DYG_E_INVALID_ARG;
      wm = std::max(wm, w[k]);
    }
  }
  // symmetric with equal weights iff the transpose equals the graph: build
  // it by counting (filling rows in ascending u keeps each row ascending)
  std::vector<uint64_t> tptr(static_cast<size_t>(n) + 1, 0);
  for (uint64_t k = 0; k < nnz; ++k) tptr[col[k] + 1]++;
  for (uint32_t u = 0; u < n; ++u) tptr[u + 1] += tptr[u];
  for (uint32_t u = 0; u <= n; ++u)
    if (tptr[u] != rowptr[u]) return DYG_E_INVALID_ARG;  // asymmetric degrees
  std::vector<uint32_t> tcol(nnz);
  std::vector<double> tw(nnz);
  std::vector<uint64_t> fill(tptr.begin(), tptr.end() - 1);
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
      const uint64_t at = fill[col[k]]++;
      tcol[at] = u;
      tw[at] = w[k];
    }
  for (uint64_t k = 0; k < nnz; ++k)
    if (tcol[k] != col[k] || tw[k] != w[k]) return DYG_E_INVALID_ARG;  // asymmetric
  if (wmax) *wmax = wm;
  return DYG_OK;
}

}  // namespace dyg

extern "C" void dyg_default_params(dyg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->seed = 0;
  p->K = INFINITY;
  p->s_default = 64;
  p->L_default = 32;
  p->Q = 24;
  p->dead_end = DYG_DEAD_END_TERMINATE;
  p->w_ref = 0.0;
  p->slack = 0.5;
  p->uid_base = 0;
}

extern "C" const char* dyg_error_string(int code) {
  switch (code) {
    case DYG_OK: return "ok";
    case DYG_E_INVALID_ARG: return "invalid argument";
    case DYG_E_SELF_LOOP: return "self loop";
    case DYG_E_VERTEX_RANGE: return "vertex id out of range";
    case DYG_E_BAD_WEIGHT: return "weight not positive and finite";
    case DYG_E_EDGE_EXISTS: return "inserted edge already in the graph";
    case DYG_E_EDGE_MISSING: return "deleted edge not in the graph";
    case DYG_E_DUPLICATE_IN_BATCH: return "edge repeated in one list";
    case DYG_E_H_NOT_SUBSET: return "sparsifier edge not in the graph";
    case DYG_E_NOMEM: return "out of memory";
    case DYG_E_DEVICE: return "HIP runtime error";
    case DYG_E_TOO_LARGE: return "batch needs more working memory than the static array holds";
    case DYG_E_BUSY: return "static working memory or context busy with a batch not yet synced";
    default: return "unknown error";
  }
}

extern "C" int dyg_init(dyg_ctx** out, uint32_t n, const uint64_t* rowptr, const uint32_t* col,
                        const double* w, uint64_t h_m, const uint32_t* h_u, const uint32_t* h_v,
                        const dyg_params* params) {
  if (!out) return DYG_E_INVALID_ARG;
  int rc = check_params(params);
  if (rc) return rc;
  if (h_m && (!h_u || !h_v)) return DYG_E_INVALID_ARG;
  double wmax = 0.0;
  rc = dyg::validate_csr(n, rowptr, col, w, &wmax);
  if (rc) return rc;
  const uint64_t nnz = rowptr[n];
  auto find = [&](uint32_t a, uint32_t b) -> int64_t {
    const uint32_t* lo = col + rowptr[a];
    const uint32_t* hi = col + rowptr[a + 1];
    const uint32_t* it = std::lower_bound(lo, hi, b);
    return (it != hi && *it == b) ? static_cast<int64_t>(it - col) : -1;
  };
  // H0: range, self loop, subset of G0, repeats (first failing edge wins)
  std::vector<std::pair<uint64_t, uint64_t>> hk(h_m);
  for (uint64_t i = 0; i < h_m; ++i) {
    const uint32_t a = std::min(h_u[i], h_v[i]), b = std::max(h_u[i], h_v[i]);
    hk[i] = {(static_cast<uint64_t>(a) << 32) | b, i};
  }
  std::sort(hk.begin(), hk.end());
  std::vector<uint8_t> repeat(h_m, 0);
  for (uint64_t i = 1; i < h_m; ++i)
    if (hk[i].first == hk[i - 1].first) repeat[hk[i].second] = 1;
  for (uint64_t i = 0; i < h_m; ++i) {
    if (h_u[i] >= n || h_v[i] >= n) return DYG_E_VERTEX_RANGE;
    if (h_u[i] == h_v[i]) return DYG_E_SELF_LOOP;
    if (find(h_u[i], h_v[i]) < 0) return DYG_E_H_NOT_SUBSET;
    if (repeat[i]) return DYG_E_DUPLICATE_IN_BATCH;
  }

  dyg_ctx* c = new (std::nothrow) dyg_ctx();
  if (!c) return DYG_E_NOMEM;
  c->n = n;
  c->params = *params;
  c->Q = params->Q;
  c->w_ref = params->w_ref > 0.0 ? params->w_ref : (wmax > 0.0 ? wmax : 1.0);
  c->has_K = !(std::isinf(params->K) && params->K > 0);
  c->uid_base = params->uid_base;
  hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return fail_hip(e);
  }
  {
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) {
      (void)hipStreamDestroy(c->stream);
      delete c;
      return fail_hip(e);
    }
    c->device = dev;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
      c->cus = static_cast<uint32_t>(cus);
    // this GPU's copy of the static working memory (null if the lookup failed:
    // dyg_apply_batch_dev_static then reports DYG_E_DEVICE)
    c->static_scratch = scratch_address(dev);
  }
  if (params->flags & DYG_FLAG_AUTOTUNE) c->tune_next = 0;
  if (params->flags & (DYG_FLAG_TIMING | DYG_FLAG_TIMING_WALK | DYG_FLAG_AUTOTUNE))
    for (hipEvent_t& ev : c->ev)
      if ((e = hipEventCreate(&ev)) != hipSuccess) {
        dyg_destroy(c);
        return fail_hip(e);
      }
  // G0 layout
  std::vector<Ent> le(nnz);
  std::vector<double> lw(w, w + nnz);
  for (uint64_t k = 0; k < nnz; ++k)
    le[k] = Ent{col[k], quantize_host(w[k], c->w_ref, c->Q), 1.0 / w[k]};
  std::vector<uint64_t> start(rowptr, rowptr + n + 1);
  for (uint32_t u = 0; u < n && !c->has_hubs; ++u)  // H is a subgraph: G's rows bound both
    c->has_hubs = rowptr[u + 1] - rowptr[u] > dyg::kHub;
  HostAdj A;
  layout(A, n, start, le, lw, params->slack);
  // H0 layout: directed entries sorted by (row, neighbour), weights from G0
  std::vector<std::pair<uint64_t, uint64_t>> hd;
  hd.reserve(2 * h_m);
  for (uint64_t i = 0; i < h_m; ++i) {
    const uint64_t j = static_cast<uint64_t>(find(h_u[i], h_v[i]));
    hd.push_back({(static_cast<uint64_t>(h_u[i]) << 32) | h_v[i], j});
    hd.push_back({(static_cast<uint64_t>(h_v[i]) << 32) | h_u[i], j});
  }
  std::sort(hd.begin(), hd.end());
  std::vector<uint64_t> hstart(n + 1, 0);
  std::vector<Ent> he(hd.size());
  std::vector<double> hw(hd.size());
  for (size_t i = 0; i < hd.size(); ++i) {
    const uint32_t a = static_cast<uint32_t>(hd[i].first >> 32);
    const uint32_t b = static_cast<uint32_t>(hd[i].first);
    hstart[a + 1]++;
    he[i] = Ent{b, le[hd[i].second].qw, le[hd[i].second].rinv};
    hw[i] = w[hd[i].second];
  }
  for (uint32_t u = 0; u < n; ++u) hstart[u + 1] += hstart[u];
  {
    uint64_t pg = 0, ph = 0;
    for (uint32_t u = 0; u < n; ++u) {
      pg += rowptr[u + 1] - rowptr[u] > dyg::kInline;
      ph += hstart[u + 1] - hstart[u] > dyg::kInline;
    }
    c->pool_frac[0] = n ? double(pg) / n : 0.0;
    c->pool_frac[1] = n ? double(ph) / n : 0.0;
  }
  HostAdj B;
  layout(B, n, hstart, he, hw, params->slack);
  const uint64_t gcap = pool_capacity_for(A.ent.size(), n, params->flags);
  const uint64_t hcap = pool_capacity_for(B.ent.size(), n, params->flags);
  if (gcap >= (1ull << 32) || hcap >= (1ull << 32)) {
    (void)hipStreamDestroy(c->stream);
    delete c;
    return DYG_E_NOMEM;
  }
  rc = upload_graph(c->G, n, A, gcap, c->stream);
  if (!rc) rc = upload_graph(c->H, n, B, hcap, c->stream);
  if (!rc) {
    e = hipMalloc(&c->ctl, sizeof(BatchCtl));
    if (e == hipSuccess) e = hipMalloc(&c->dargs, sizeof(BatchArgs));
    if (e == hipSuccess) e = hipHostMalloc(&c->hargs, sizeof(BatchArgs), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&c->hctl, sizeof(BatchCtl), hipHostMallocDefault);
    if (e == hipSuccess) std::memset(c->hctl, 0, sizeof(BatchCtl));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&c->dargv, sizeof(BatchArgs*));
    if (e == hipSuccess) {
      const BatchArgs* p = c->dargs;
      e = hipMemcpy(c->dargv, &p, sizeof(p), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) rc = fail_hip(e);
  }
  if (!rc) {
    BatchCtl init{};
    init.err_key = ~0ull;
    for (const Ent& x : le) init.heavy |= x.qw >= dyg::kHeavyQw ? 1u : 0u;  // H's weights are G's
    init.pool_top[0] = A.ent.size();
    init.pool_top[1] = B.ent.size();
    e = hipMemcpyAsync(c->ctl, &init, sizeof(init), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = fail_hip(e);
    c->pool_top[0] = A.ent.size();
    c->pool_top[1] = B.ent.size();
  }
  if (rc) {
    dyg_destroy(c);
    return rc;
  }
  *out = c;
  return DYG_OK;
}

namespace {

// Size every staging buffer for a batch; returns DYG_OK or DYG_E_NOMEM.
// H-addition slots and hash-table size of a batch; false if the table would
// exceed 2^31 slots.
bool batch_table_sizes(uint64_t n_ins, uint64_t n_del, uint32_t Lcap, uint64_t& hadd_cap,
                       uint64_t& hash_slots) {
  const uint64_t nu = n_ins + n_del;
  hadd_cap = n_ins + n_del * std::max<uint32_t>(Lcap, 2);
  const uint64_t keys = std::max<uint64_t>(nu, 2 * hadd_cap);
  hash_slots = next_pow2(2 * keys + 64);
  return hash_slots <= (1ull << 31);
}

int prepare_buffers(dyg_ctx* c, uint64_t n_ins, uint64_t n_del, uint32_t Lcap,
                    uint64_t walkers, uint64_t items_cap, uint64_t& hadd_cap,
                    uint64_t& hash_slots) {
  const uint64_t nu = n_ins + n_del;
  if (!batch_table_sizes(n_ins, n_del, Lcap, hadd_cap, hash_slots)) return DYG_E_NOMEM;
  bool ok = c->ins_qw.ensure(4 * n_ins + 8) && c->ins_rinv.ensure(8 * n_ins + 8) &&
            c->in_h.ensure(n_del + 8) && c->res.ensure(sizeof(dyg_update_result) * nu + 8) &&
            c->ubytes.ensure(4 * nu + 8) && c->fb_list.ensure(4 * n_del + 8) &&
            c->hadd.ensure(sizeof(AddRec) * hadd_cap + 8) &&
            c->hash.ensure(sizeof(HashSlot) * hash_slots) &&
            c->hash2.ensure(sizeof(HashSlot) * hash_slots) &&
            (walkers == 0 || (c->wrec.ensure(sizeof(dyg_walker_record) * walkers) &&
                              c->wofs.ensure(8 * nu + 8)));
  if (ok && (c->params.flags & DYG_FLAG_BATCHED)) {
    const uint64_t tiles = (nu + 1023) / 1024 + 1;
    ok = c->qcount.ensure(4 * nu + 8) && c->qofs.ensure(8 * nu + 8) &&
         c->qtile.ensure(8 * tiles + 8) &&
         // item records only for the work queue (the range walk derives them)
         (c->updates_per_wave > 0 || c->items.ensure(sizeof(dyg::WalkItem) * items_cap + 8)) &&
         c->wres.ensure(sizeof(dyg::WalkOut) * items_cap + 16) &&
         (c->tail_lanes == 0 || (c->tstate.ensure(sizeof(dyg::TailState) * items_cap + 16) &&
                                 c->tcount.ensure(4 * nu + 8)));
  }
  for (int g = 0; g < 2 && ok; ++g) {
    const uint64_t cap = g == 0 ? 2 * n_ins : 2 * hadd_cap;
    ok = c->touched_rows[g].ensure(4 * cap + 8) && c->touched_k[g].ensure(4 * cap + 8) &&
         c->touched_need[g].ensure(4 * cap + 8) && c->add_keep[g].ensure(cap + 8) &&
         c->dirty_rows[g].ensure(4 * (cap + 2 * n_del) + 8) &&
         c->dirty_chunk0[g].ensure(4 * (cap + 2 * n_del) + 8) &&
         c->dirty_small[g].ensure(4 * (cap + 2 * n_del) + 8) && c->wide_rows[g].ensure(4 * cap + 8) &&
         c->wmerge[g].ensure(sizeof(dyg::WideMerge) * cap + 8);
  }
  return ok ? DYG_OK : DYG_E_NOMEM;
}

BatchArgs& make_args(dyg_ctx* c, uint64_t n_ins, uint64_t n_del, const uint32_t* iu,
                    const uint32_t* iv, const double* iw, const uint32_t* du, const uint32_t* dv,
                    const uint16_t* s, const uint16_t* L, uint32_t Lcap, uint64_t hadd_cap,
                    uint64_t hash_slots, dyg::UpdRes* res, bool record) {
  BatchArgs& a = *c->hargs;
  a = BatchArgs{};
  a.n = c->n;
  a.n_ins = static_cast<uint32_t>(n_ins);
  a.n_del = static_cast<uint32_t>(n_del);
  a.iu = iu;
  a.iv = iv;
  a.iw = iw;
  a.du = du;
  a.dv = dv;
  a.s = s;
  a.L = L;
  a.s_def = c->params.s_default;
  a.L_def = c->params.L_default;
  a.Lcap = Lcap;
  a.scap = kMaxWalkersHost;
  a.uid_base = c->uid_base;
  a.seed = c->params.seed;
  a.K = c->params.K;
  a.has_K = c->has_K ? 1 : 0;
  a.bounce = c->params.dead_end;
  a.variant = ((c->params.flags & DYG_FLAG_BOTH_ENDS) ? dyg::kVarBothEnds : 0u) |
              ((c->params.flags & DYG_FLAG_LOOP_ERASED) ? dyg::kVarLoopErased : 0u) |
              ((c->params.flags & DYG_FLAG_TWO_STAGE) ? dyg::kVarTwoStage : 0u);
  a.w_ref = c->w_ref;
  a.Q = c->Q;
  a.ins_qw = c->ins_qw.as<uint32_t>();
  a.ins_rinv = c->ins_rinv.as<double>();
  a.in_h = c->in_h.as<uint8_t>();
  a.res = res;
  a.wrec = record ? c->wrec.as<dyg::WalkerRec>() : nullptr;
  a.wofs = record ? c->wofs.as<uint64_t>() : nullptr;
  a.hadd = c->hadd.as<AddRec>();
  a.ubytes = c->ubytes.as<uint32_t>();
  a.fb_list = c->fb_list.as<uint32_t>();
  a.hadd_cap = static_cast<uint32_t>(hadd_cap);
  a.hash = c->hash.as<HashSlot>();
  a.hash2 = c->hash2.as<HashSlot>();
  a.hash_mask = static_cast<uint32_t>(hash_slots - 1);
  a.hash_slots = hash_slots;
  a.g[0] = c->G;
  a.g[1] = c->H;
  a.ctl = c->ctl;
  a.qctl = c->ctl;
  for (int g = 0; g < 2; ++g) {
    a.touched_rows[g] = c->touched_rows[g].as<uint32_t>();
    a.touched_k[g] = c->touched_k[g].as<uint32_t>();
    a.touched_need[g] = c->touched_need[g].as<uint32_t>();
    a.add_keep[g] = c->add_keep[g].as<uint8_t>();
    a.dirty_rows[g] = c->dirty_rows[g].as<uint32_t>();
    a.dirty_chunk0[g] = c->dirty_chunk0[g].as<uint32_t>();
    a.dirty_small[g] = c->dirty_small[g].as<uint32_t>();
    a.wide_rows[g] = c->wide_rows[g].as<uint32_t>();
    a.wmerge[g] = c->wmerge[g].as<dyg::WideMerge>();
  }
  a.qcount = c->qcount.as<uint32_t>();
  a.qofs = c->qofs.as<unsigned long long>();
  a.qtile = c->qtile.as<unsigned long long>();
  a.items = c->items.as<dyg::WalkItem>();
  a.refill_min = c->refill_min;
  a.upw = c->updates_per_wave;
  a.wres = c->wres.as<dyg::WalkOut>();
  a.tail_lanes = c->tail_lanes;
  a.tstate = c->tstate.as<dyg::TailState>();
  a.tcount = c->tcount.as<uint32_t>();
  return a;
}

// Bump allocation of 256-byte aligned pieces from a fixed region; `used`
// counts every piece asked for, so it gives the size a batch needs even
// when the region is too small (then ok is false).
struct Carve {
  char* base;
  size_t cap;
  size_t used = 0;
  bool ok = true;
  template <class T>
  T* take(size_t bytes) {
    const size_t at = (used + 255) & ~size_t(255);
    used = at + bytes;
    if (used > cap) ok = false;
    return ok ? reinterpret_cast<T*>(base + at) : nullptr;
  }
};

// Point every per-batch buffer of `a` into region `m`, with the sizes that
// prepare_buffers gives the context's own buffers (no per-walker records).
// own_results: the batch keeps its results in the region too.
void carve_batch(const dyg_ctx* c, BatchArgs& a, Carve& m, uint64_t n_ins, uint64_t n_del,
                 uint64_t items_cap, uint64_t hadd_cap, uint64_t hash_slots, bool own_results) {
  const uint64_t nu = n_ins + n_del;
  a.ins_qw = m.take<uint32_t>(4 * n_ins + 8);
  a.ins_rinv = m.take<double>(8 * n_ins + 8);
  a.in_h = m.take<uint8_t>(n_del + 8);
  if (own_results) a.res = m.take<dyg::UpdRes>(sizeof(dyg_update_result) * nu + 8);
  a.ubytes = m.take<uint32_t>(4 * nu + 8);
  a.fb_list = m.take<uint32_t>(4 * n_del + 8);
  a.hadd = m.take<AddRec>(sizeof(AddRec) * hadd_cap + 8);
  a.hash = m.take<HashSlot>(sizeof(HashSlot) * hash_slots);
  a.hash2 = m.take<HashSlot>(sizeof(HashSlot) * hash_slots);
  a.wrec = nullptr;
  a.wofs = nullptr;
  if (c->params.flags & DYG_FLAG_BATCHED) {
    const uint64_t tiles = (nu + 1023) / 1024 + 1;
    a.qcount = m.take<uint32_t>(4 * nu + 8);
    a.qofs = m.take<unsigned long long>(8 * nu + 8);
    a.qtile = m.take<unsigned long long>(8 * tiles + 8);
    a.items = c->updates_per_wave > 0 ? nullptr
                                      : m.take<dyg::WalkItem>(sizeof(dyg::WalkItem) * items_cap + 8);
    a.wres = m.take<dyg::WalkOut>(sizeof(dyg::WalkOut) * items_cap + 16);
    a.tstate = c->tail_lanes == 0 ? nullptr
                                  : m.take<dyg::TailState>(sizeof(dyg::TailState) * items_cap + 16);
    a.tcount = c->tail_lanes == 0 ? nullptr : m.take<uint32_t>(4 * nu + 8);
  } else {
    a.qcount = nullptr;
    a.qofs = nullptr;
    a.qtile = nullptr;
    a.items = nullptr;
    a.wres = nullptr;
    a.tstate = nullptr;
    a.tcount = nullptr;
  }
  for (int g = 0; g < 2; ++g) {
    const uint64_t cap = g == 0 ? 2 * n_ins : 2 * hadd_cap;
    a.touched_rows[g] = m.take<uint32_t>(4 * cap + 8);
    a.touched_k[g] = m.take<uint32_t>(4 * cap + 8);
    a.touched_need[g] = m.take<uint32_t>(4 * cap + 8);
    a.add_keep[g] = m.take<uint8_t>(cap + 8);
    a.dirty_rows[g] = m.take<uint32_t>(4 * (cap + 2 * n_del) + 8);
    a.dirty_chunk0[g] = m.take<uint32_t>(4 * (cap + 2 * n_del) + 8);
    a.dirty_small[g] = m.take<uint32_t>(4 * (cap + 2 * n_del) + 8);
    a.wide_rows[g] = m.take<uint32_t>(4 * cap + 8);
    a.wmerge[g] = m.take<dyg::WideMerge>(sizeof(dyg::WideMerge) * cap + 8);
  }
}

// Whether the plain walk kernel reads rows cooperatively: insertions walk H,
// deletions walk G; worthwhile when at least 40% of the walks start in a
// graph whose rows are mostly pool rows (by the initial degrees).
bool use_coop(const dyg_ctx* c, uint64_t n_ins, uint64_t n_del) {
  const double w = double(n_ins) * c->pool_frac[1] + double(n_del) * c->pool_frac[0];
  return n_ins + n_del > 0 && w >= 0.4 * double(n_ins + n_del);
}

// Launch geometry of this context's batch `a` alone.
dyg::Launch single_launch(dyg_ctx* c, const BatchArgs& a) {
  dyg::Launch L{};
  L.h_lo = c->h_lo;
  L.h_hi = c->h_hi;
  L.argv = c->dargv;
  L.F = 1;
  L.max_nu = a.n_ins + a.n_del;
  L.max_ins = a.n_ins;
  L.max_del = a.n_del;
  L.max_hadd_cap = a.hadd_cap;
  L.max_hash_slots = a.hash_slots;
  L.walk_blocks = c->cus * c->walk_blocks_per_cu;
  L.upw = c->updates_per_wave;
  L.hubs = c->has_hubs;
  L.coop = use_coop(c, a.n_ins, a.n_del);
  L.tail_lanes = c->tail_lanes;
  return L;
}

// The launch sequence of one batch.  `a` gives the grid sizes (the batch
// itself, or its size class when captured); kernels read the actual batch
// from device memory.
bool tuning_now(const dyg_ctx* c);

void launch_sequence(dyg_ctx* c, const BatchArgs& a, bool timed) {
  const dyg::Launch L = single_launch(c, a);
  dyg::launch_batch_begin(L, c->stream);
  dyg::launch_validate(L, c->stream);
  dyg::launch_phase1(L, c->stream);
  // the batched form's walk: walker-packed (work queue, ranges, head/tail,
  // then a reduction per update) or lockstep as in the plain form
  const bool queue = (c->params.flags & DYG_FLAG_BATCHED) != 0 && !c->lockstep;
  if (queue) dyg::launch_queue_prepare(L, c->stream);
  // the timed region is the walk kernel alone; while the autotuner tries
  // schedules it includes the rest of the decisions (the reduction of a
  // walker-packed schedule, the long-row fallbacks)
  const bool with_finish = tuning_now(c);
  if (timed) (void)hipEventRecord(c->ev[1], c->stream);
  if (queue)
    dyg::launch_walk_queue(L, c->stream);
  else
    dyg::launch_walks(L, c->stream);
  const auto finish = [&] {
    if (queue) dyg::launch_queue_finish(L, c->stream);
    else dyg::launch_walk_fallbacks(L, c->stream);
  };
  if (with_finish) finish();
  if (timed) (void)hipEventRecord(c->ev[2], c->stream);
  if (!with_finish) finish();
  dyg::launch_sum_counters(L, c->stream);
  dyg::launch_phase4_both(L, c->stream);
}

uint64_t size_class(uint64_t x) { return x ? next_pow2(x) : 0; }

// Launch sequence of the size class of `a`, captured on first use.
int graph_for(dyg_ctx* c, const BatchArgs& a, hipGraphExec_t* out) {
  BatchArgs cls = a;
  cls.n_ins = static_cast<uint32_t>(size_class(a.n_ins));
  cls.n_del = static_cast<uint32_t>(size_class(a.n_del));
  cls.hadd_cap = static_cast<uint32_t>(size_class(a.hadd_cap));
  cls.hash_slots = a.hash_slots;  // cleared by a grid-stride loop: any grid works
  const uint32_t wb = c->cus * c->walk_blocks_per_cu;
  const auto key = std::make_tuple(uint64_t(cls.n_ins), uint64_t(cls.n_del),
                                   uint64_t(cls.hadd_cap), wb, c->updates_per_wave,
                                   c->has_hubs, use_coop(c, cls.n_ins, cls.n_del),
                                   c->tail_lanes, c->lockstep);
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    *out = it->second;
    return DYG_OK;
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return fail_hip(e);
  launch_sequence(c, cls, false);
  e = hipStreamEndCapture(c->stream, &graph);
  if (e != hipSuccess) return fail_hip(e);
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail_hip(e);
  c->graphs[key] = exec;
  *out = exec;
  return DYG_OK;
}

// Enqueue one batch: copy its arguments to the device, then its launch
// sequence (directly, or as the captured graph of its size class; capturing
// and instantiating a graph allocates, so allow_graph = false launches
// directly whatever the flags say).
int enqueue_two_stage(dyg_ctx* c, BatchArgs& a);

int enqueue_pipeline(dyg_ctx* c, BatchArgs& a, bool allow_graph = true) {
  if (c->params.flags & DYG_FLAG_TWO_STAGE) return enqueue_two_stage(c, a);
  c->h_lo = 0;
  c->h_hi = ~0u;
  const bool timed = c->ev[0] != nullptr;
  // the batch itself is bracketed only under DYG_FLAG_TIMING
  const bool timed_batch = timed && (c->params.flags & DYG_FLAG_TIMING);
  hipError_t e = hipSuccess;
  if (timed_batch) (void)hipEventRecord(c->ev[0], c->stream);
  e = hipMemcpyAsync(c->dargs, &a, sizeof(BatchArgs), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return fail_hip(e);
  c->last_graph = allow_graph && (c->params.flags & DYG_FLAG_GRAPH) && !tuning_now(c);
  if (c->last_graph) {
    hipGraphExec_t exec = nullptr;
    int rc = graph_for(c, a, &exec);
    if (rc) return rc;
    if ((e = hipGraphLaunch(exec, c->stream)) != hipSuccess) return fail_hip(e);
    if (timed) {
      // the walk kernel is inside the graph: time the whole batch only
      (void)hipEventRecord(c->ev[1], c->stream);
      (void)hipEventRecord(c->ev[2], c->stream);
    }
  } else {
    launch_sequence(c, a, timed);
  }
  if (timed_batch) (void)hipEventRecord(c->ev[3], c->stream);
  c->timed_pending = timed && (a.n_ins + a.n_del) > 0;
  // the batch's control block comes back with the batch: one wait at sync
  e = hipMemcpyAsync(c->hctl, c->ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipEventRecord(c->done_ev, c->stream);
  if (e != hipSuccess) return fail_hip(e);
  return DYG_OK;
}

// Fold the events of the batch that just completed into the timers.
// Returns whether the walk kernel of the finished batch was timed.
bool collect_timing(dyg_ctx* c) {
  if (!c->timed_pending) return false;
  c->timed_pending = false;
  float walk = 0.f, batch = 0.f;
  if (c->params.flags & DYG_FLAG_TIMING) {
    if (hipEventElapsedTime(&batch, c->ev[0], c->ev[3]) != hipSuccess) return false;
    c->batch_ms_last = batch;
  }
  if (c->last_graph) return false;  // the walk kernel was inside a captured graph
  if (hipEventElapsedTime(&walk, c->ev[1], c->ev[2]) != hipSuccess) return false;
  c->walk_launches++;
  c->walk_ms_last = walk;
  c->walk_ms_total += walk;
  return true;
}

// Walk schedules the autotuner tries, one batch each: updates per wavefront
// (0 = work queue), idle lanes that trigger a refill, queue grid per CU.
struct TuneCandidate {
  uint32_t upw, refill_min, blocks_per_cu, tail_lanes, lockstep;
};
constexpr TuneCandidate kTuneCandidates[] = {
    {4, 1, 8, 0, 1}, {1, 1, 8, 0, 0},  {2, 1, 8, 0, 0},  {4, 1, 8, 0, 0},  {4, 8, 8, 0, 0},
    {8, 1, 8, 0, 0}, {0, 16, 8, 0, 0}, {4, 1, 8, 8, 0},  {4, 1, 8, 16, 0}, {8, 1, 8, 16, 0},
};
constexpr int kTuneCount = static_cast<int>(sizeof(kTuneCandidates) / sizeof(kTuneCandidates[0]));

bool tuning_now(const dyg_ctx* c) {
  return c->tune_next >= 0 && (c->params.flags & DYG_FLAG_BATCHED);
}

// Before a batch: put the next candidate in place.
void tune_begin(dyg_ctx* c, unsigned long long steps_before) {
  if (!tuning_now(c)) return;
  const TuneCandidate& k = kTuneCandidates[c->tune_next];
  c->updates_per_wave = k.upw;
  c->refill_min = k.refill_min;
  c->walk_blocks_per_cu = k.blocks_per_cu;
  c->tail_lanes = k.tail_lanes;
  c->lockstep = k.lockstep;
  c->tune_steps0 = steps_before;
}

// After it: score the candidate (walk ms per walker step); after the last,
// keep the best.
void tune_end(dyg_ctx* c, unsigned long long steps_after, bool walk_timed) {
  if (!tuning_now(c)) return;
  const unsigned long long steps = steps_after - c->tune_steps0;
  if (walk_timed && steps > 0) {
    const double score = c->walk_ms_last / static_cast<double>(steps);
    if (c->tune_best < 0 || score < c->tune_best_score) {
      c->tune_best = c->tune_next;
      c->tune_best_score = score;
    }
    ++c->tune_next;  // batches without walks do not count as a trial
  }
  if (c->tune_next >= kTuneCount) {
    c->tune_next = -1;
    if (c->tune_best >= 0) {
      const TuneCandidate& k = kTuneCandidates[c->tune_best];
      c->updates_per_wave = k.upw;
      c->refill_min = k.refill_min;
      c->walk_blocks_per_cu = k.blocks_per_cu;
      c->tail_lanes = k.tail_lanes;
      c->lockstep = k.lockstep;
    }
  }
}

int decode_err(unsigned long long key) {
  if (key == ~0ull) return DYG_OK;
  return -static_cast<int>(key & 0xFF);
}

// Finish phase 4 of graphs that ran short of pool slots: grow the pool,
// then run phase 4 again from the batch's staged additions.
int repair_nomem(dyg_ctx* c, BatchArgs& a, BatchCtl& ctl) {
  if (c->params.flags & DYG_FLAG_FAIL_POOL_GROWTH) return DYG_E_NOMEM;
  for (int attempt = 0; attempt < 4 && (ctl.nomem[0] || ctl.nomem[1]); ++attempt) {
    for (int g = 0; g < 2; ++g) {
      if (!ctl.nomem[g]) continue;
      dyg::launch_phase4_reset(single_launch(c, a), g, c->stream);
      const uint64_t want = ctl.pool_top[g] + ctl.need[g] + ctl.need[g] / 2 + 64;
      int rc = compact_graph(c, g, want);  // synchronises the stream
      if (rc) return rc;
      a.g[0] = c->G;
      a.g[1] = c->H;
      hipError_t e =
          hipMemcpyAsync(c->dargs, &a, sizeof(BatchArgs), hipMemcpyHostToDevice, c->stream);
      if (e != hipSuccess) return fail_hip(e);
      dyg::launch_phase4(single_launch(c, a), g, c->stream);
    }
    int rc = sync_ctl_host(c, ctl);
    if (rc) return rc;
  }
  return (ctl.nomem[0] || ctl.nomem[1]) ? DYG_E_NOMEM : DYG_OK;
}

// A two-stage batch (either form; in the batched form it, too, takes the
// lockstep walk, launched directly): validation, phase 1, the deletion walks
// and decisions, and H += their recovered and fallback edges (slots n_ins..),
// then -- after a host check of that first phase 4, growing H's pool if it
// ran short -- the insertion walks on the repaired H, the counters, and G +=
// insertions, H += kept insertions (slots 0..n_ins-1).  The second stage is
// enqueued like any batch and completes at dyg_sync / in dyg_apply_batch.
int enqueue_two_stage(dyg_ctx* c, BatchArgs& a) {
  hipError_t e = hipMemcpyAsync(c->dargs, &a, sizeof(BatchArgs), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return fail_hip(e);
  c->last_graph = false;
  c->timed_pending = false;  // two walk launches: not timed
  c->h_lo = a.n_ins;
  c->h_hi = a.hadd_cap;
  dyg::Launch L = single_launch(c, a);
  dyg::launch_batch_begin(L, c->stream);
  dyg::launch_validate(L, c->stream);
  dyg::launch_phase1(L, c->stream);
  L.stage = dyg::kStageDeletions;
  dyg::launch_walks(L, c->stream);
  dyg::launch_walk_fallbacks(L, c->stream);
  dyg::launch_phase4(L, 1, c->stream);
  BatchCtl ctl;
  int rc = sync_ctl_host(c, ctl);
  if (rc) return rc;
  if (decode_err(ctl.err_key) == DYG_OK && ctl.nomem[1]) {
    rc = repair_nomem(c, a, ctl);
    if (rc) {
      c->broken = true;
      return rc;
    }
  }
  c->h_lo = 0;
  c->h_hi = a.n_ins;
  L = single_launch(c, a);
  dyg::launch_phase4_clear(L, 0, c->stream);
  dyg::launch_phase4_clear(L, 1, c->stream);
  L.stage = dyg::kStageInsertions;
  dyg::launch_walks(L, c->stream);  // no deletions here: no fallbacks
  dyg::launch_sum_counters(L, c->stream);
  dyg::launch_phase4_both(L, c->stream);
  e = hipMemcpyAsync(c->hctl, c->ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipEventRecord(c->done_ev, c->stream);
  if (e != hipSuccess) return fail_hip(e);
  return DYG_OK;
}

// Keep a tenth of each pool free between batches.
int maybe_compact(dyg_ctx* c) {
  for (int g = 0; g < 2; ++g) {
    const DevGraph& X = g ? c->H : c->G;
    if (c->pool_top[g] * 10 > X.pool_cap * 9) {
      int rc = compact_graph(c, g, 0);
      if (rc) return rc;
    }
  }
  return DYG_OK;
}

}  // namespace

extern "C" int dyg_apply_batch(dyg_ctx* c, uint64_t n_ins, const uint32_t* iu,
                               const uint32_t* iv, const double* iw, uint64_t n_del,
                               const uint32_t* du, const uint32_t* dv, const uint16_t* s,
                               const uint16_t* L, dyg_update_result* results,
                               dyg_walker_record* walkers) {
  if (!c) return DYG_E_INVALID_ARG;
  if (c->broken) return DYG_E_NOMEM;
  if ((n_ins && (!iu || !iv || !iw)) || (n_del && (!du || !dv))) return DYG_E_INVALID_ARG;
  const uint64_t nu = n_ins + n_del;
  if (nu >= (1ull << 30)) return DYG_E_INVALID_ARG;
  if (c->async_inflight) {
    // the device batch enqueued before this one: its failure is this call's
    int rc = dyg_sync(c);
    if (rc) return rc;
  }
  if (c->broken) return DYG_E_NOMEM;
  uint32_t Lcap = c->params.L_default;
  uint64_t walkers_total = 0;
  std::vector<uint64_t> wofs;
  if (L)
    for (uint64_t i = 0; i < nu; ++i) Lcap = std::max<uint32_t>(Lcap, L[i]);
  Lcap = std::min<uint32_t>(std::max<uint32_t>(Lcap, 2), DYG_MAX_STEPS + 1);
  if (walkers) {
    wofs.resize(nu + 1);
    wofs[0] = 0;
    for (uint64_t i = 0; i < nu; ++i)
      wofs[i + 1] = wofs[i] + std::min<uint32_t>(s ? s[i] : c->params.s_default, DYG_MAX_WALKERS);
    walkers_total = wofs[nu];
  }
  tune_begin(c, c->hctl->steps_total);
  uint64_t items_cap = 0;
  if (c->params.flags & DYG_FLAG_BATCHED) {
    if (s)
      for (uint64_t i = 0; i < nu; ++i) items_cap += std::min<uint32_t>(s[i], DYG_MAX_WALKERS);
    else
      items_cap = nu * c->params.s_default;
  }
  uint64_t hadd_cap, hash_slots;
  if (prepare_buffers(c, n_ins, n_del, Lcap, walkers_total, items_cap, hadd_cap, hash_slots))
    return DYG_E_NOMEM;
  if (!c->iu.ensure(4 * n_ins + 8) || !c->iv.ensure(4 * n_ins + 8) ||
      !c->iw.ensure(8 * n_ins + 8) || !c->du.ensure(4 * n_del + 8) ||
      !c->dv.ensure(4 * n_del + 8) || !c->s.ensure(2 * nu + 8) || !c->L.ensure(2 * nu + 8))
    return DYG_E_NOMEM;
  // stage the batch in pinned memory, then one copy per array
  const size_t in_bytes = 16 * n_ins + 8 * n_del + 4 * nu + 8 * (nu + 1) + 64;
  if (!c->pin_in.ensure(in_bytes)) return DYG_E_NOMEM;
  char* h = static_cast<char*>(c->pin_in.p);
  hipStream_t st = c->stream;
  hipError_t e = hipSuccess;
  auto put = [&](DBuf& dst, const void* src, size_t bytes) {
    if (!bytes || e != hipSuccess) return;
    std::memcpy(h, src, bytes);
    e = hipMemcpyAsync(dst.p, h, bytes, hipMemcpyHostToDevice, st);
    h += (bytes + 15) & ~size_t(15);
  };
  put(c->iu, iu, 4 * n_ins);
  put(c->iv, iv, 4 * n_ins);
  put(c->iw, iw, 8 * n_ins);
  put(c->du, du, 4 * n_del);
  put(c->dv, dv, 4 * n_del);
  if (s) put(c->s, s, 2 * nu);
  if (L) put(c->L, L, 2 * nu);
  if (walkers) put(c->wofs, wofs.data(), 8 * nu);
  if (e != hipSuccess) return fail_hip(e);

  BatchArgs& a = make_args(c, n_ins, n_del, c->iu.as<uint32_t>(), c->iv.as<uint32_t>(),
                          c->iw.as<double>(), c->du.as<uint32_t>(), c->dv.as<uint32_t>(),
                          s ? c->s.as<uint16_t>() : nullptr, L ? c->L.as<uint16_t>() : nullptr,
                          Lcap, hadd_cap, hash_slots, c->res.as<dyg::UpdRes>(), walkers != nullptr);
  int prc = enqueue_pipeline(c, a);
  if (prc) return prc;
  if ((e = hipGetLastError()) != hipSuccess) return fail_hip(e);

  BatchCtl ctl;
  int rc = finish_ctl(c, ctl);
  if (rc) return rc;
  tune_end(c, ctl.steps_total, collect_timing(c));
  rc = decode_err(ctl.err_key);
  if (rc) return rc;
  if (ctl.nomem[0] || ctl.nomem[1]) {
    rc = repair_nomem(c, a, ctl);
    if (rc) {
      c->broken = true;
      return rc;
    }
  }
  const size_t out_bytes = sizeof(dyg_update_result) * nu + sizeof(dyg_walker_record) * walkers_total;
  if (results || walkers) {
    if (!c->pin_out.ensure(out_bytes + 64)) return DYG_E_NOMEM;
    char* o = static_cast<char*>(c->pin_out.p);
    if (results && nu)
      e = hipMemcpyAsync(o, c->res.p, sizeof(dyg_update_result) * nu, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && walkers && walkers_total)
      e = hipMemcpyAsync(o + sizeof(dyg_update_result) * nu, c->wrec.p,
                         sizeof(dyg_walker_record) * walkers_total, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail_hip(e);
    if (results) std::memcpy(results, o, sizeof(dyg_update_result) * nu);
    if (walkers)
      std::memcpy(walkers, o + sizeof(dyg_update_result) * nu,
                  sizeof(dyg_walker_record) * walkers_total);
  }
  c->uid_base += nu;
  c->batches++;
  return maybe_compact(c);
}

extern "C" int dyg_apply_batch_dev(dyg_ctx* c, const dyg_batch_dev* b, void* stream) {
  if (!c || !b) return DYG_E_INVALID_ARG;
  if (c->broken) return DYG_E_NOMEM;
  const uint64_t n_ins = b->n_ins, n_del = b->n_del, nu = n_ins + n_del;
  if ((n_ins && (!b->iu || !b->iv || !b->iw)) || (n_del && (!b->du || !b->dv)) ||
      nu >= (1ull << 30) || b->L_max > DYG_MAX_STEPS)
    return DYG_E_INVALID_ARG;
  if (c->async_inflight) {
    int rc = dyg_sync(c);
    if (rc) return rc;
  }
  if (b->s && b->s_max > DYG_MAX_WALKERS) return DYG_E_INVALID_ARG;
  const uint32_t Lcap = std::max<uint32_t>(b->L ? b->L_max : c->params.L_default, 2);
  const uint32_t scap = b->s ? b->s_max : c->params.s_default;
  tune_begin(c, c->hctl->steps_total);
  uint64_t hadd_cap, hash_slots;
  if (prepare_buffers(c, n_ins, n_del, Lcap, 0, nu * scap, hadd_cap, hash_slots))
    return DYG_E_NOMEM;
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
  std::swap(st, c->stream);  // every launcher below runs on the caller's stream
  BatchArgs& a = make_args(c, n_ins, n_del, b->iu, b->iv, b->iw, b->du, b->dv, b->s, b->L, Lcap,
                          hadd_cap, hash_slots,
                          b->results ? reinterpret_cast<dyg::UpdRes*>(b->results)
                                     : c->res.as<dyg::UpdRes>(),
                          false);
  a.scap = scap;
  int prc = enqueue_pipeline(c, a);
  std::swap(st, c->stream);
  if (prc) return prc;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(e);
  c->async_inflight = true;
  c->async_nu = nu;
  c->pending_status = DYG_OK;
  return DYG_OK;
}

extern "C" int dyg_apply_batch_dev_static(dyg_ctx* c, const dyg_batch_dev* b, void* stream) {
  if (!c || !b) return DYG_E_INVALID_ARG;
  if (c->broken) return DYG_E_NOMEM;
  const uint64_t n_ins = b->n_ins, n_del = b->n_del, nu = n_ins + n_del;
  if ((n_ins && (!b->iu || !b->iv || !b->iw)) || (n_del && (!b->du || !b->dv)) ||
      nu >= (1ull << 30) || b->L_max > DYG_MAX_STEPS || (b->s && b->s_max > DYG_MAX_WALKERS))
    return DYG_E_INVALID_ARG;
  // completing an earlier batch may grow a pool, which allocates: the caller
  // does that with dyg_sync before this call
  if (c->async_inflight) return DYG_E_BUSY;
  // a two-stage batch checks (and may grow) H's pool between its stages
  if (c->params.flags & DYG_FLAG_TWO_STAGE) return DYG_E_INVALID_ARG;
  if (!c->static_scratch) return DYG_E_DEVICE;
  const uint32_t Lcap = std::max<uint32_t>(b->L ? b->L_max : c->params.L_default, 2);
  const uint32_t scap = b->s ? b->s_max : c->params.s_default;
  uint64_t hadd_cap, hash_slots;
  if (!batch_table_sizes(n_ins, n_del, Lcap, hadd_cap, hash_slots)) return DYG_E_TOO_LARGE;
  StaticScratch& ss = static_scratch();
  std::lock_guard<std::mutex> lock(ss.mu);
  if (ss.owner[c->device]) return DYG_E_BUSY;  // another context's batch is not synced yet
  tune_begin(c, c->hctl->steps_total);
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
  std::swap(st, c->stream);  // every launcher below runs on the caller's stream
  BatchArgs& a = make_args(c, n_ins, n_del, b->iu, b->iv, b->iw, b->du, b->dv, b->s, b->L, Lcap,
                          hadd_cap, hash_slots,
                          reinterpret_cast<dyg::UpdRes*>(b->results), false);
  a.scap = scap;
  Carve m{static_cast<char*>(c->static_scratch), kStaticScratchBytes};
  carve_batch(c, a, m, n_ins, n_del, nu * scap, hadd_cap, hash_slots, b->results == nullptr);
  int prc = m.ok ? enqueue_pipeline(c, a, false) : DYG_E_TOO_LARGE;
  std::swap(st, c->stream);
  if (prc) return prc;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(e);
  ss.owner[c->device] = c;
  c->static_inflight = true;
  c->async_inflight = true;
  c->async_nu = nu;
  c->pending_status = DYG_OK;
  return DYG_OK;
}

namespace {

// The static working memory of c's GPU is free again (c's batch has ended).
void release_static(dyg_ctx* c) {
  if (!c->static_inflight) return;
  StaticScratch& s = static_scratch();
  std::lock_guard<std::mutex> lock(s.mu);
  if (s.owner[c->device] == c) s.owner[c->device] = nullptr;
  c->static_inflight = false;
}

int sync_batch(dyg_ctx* c);

}  // namespace

extern "C" int dyg_sync(dyg_ctx* c) {
  if (!c) return DYG_E_INVALID_ARG;
  const int rc = sync_batch(c);
  release_static(c);  // after any pool repair, which reads the batch's staged additions
  return rc;
}

namespace {

int sync_batch(dyg_ctx* c) {
  if (!c->async_inflight) return DYG_OK;  // a batch's status is reported once
  c->async_inflight = false;
  BatchCtl ctl;
  int rc = finish_ctl(c, ctl);
  if (rc) return c->pending_status = rc;
  tune_end(c, ctl.steps_total, collect_timing(c));
  rc = decode_err(ctl.err_key);
  if (rc) return c->pending_status = rc;
  if (ctl.nomem[0] || ctl.nomem[1]) {
    // the staged additions of this batch are still intact: grow the pool and
    // finish its phase 4 (its device arguments are still in c->hargs)
    rc = repair_nomem(c, *c->hargs, ctl);
    if (rc) {
      c->broken = true;
      return c->pending_status = rc;
    }
  }
  c->uid_base += c->async_nu;
  c->batches++;
  return c->pending_status = maybe_compact(c);
}

}  // namespace

namespace {

int query_graph(dyg_ctx* c, int which, uint64_t cap, uint64_t* m, uint32_t* u, uint32_t* v,
                double* w) {
  if (!c || !m) return DYG_E_INVALID_ARG;
  if (c->async_inflight) {
    int rc = dyg_sync(c);
    if (rc) return rc;
  }
  BatchCtl ctl;
  int rc = sync_ctl_host(c, ctl);
  if (rc) return rc;
  const DevGraph& X = which ? c->H : c->G;
  std::vector<uint64_t> start;
  std::vector<Ent> le;
  std::vector<double> lw;
  rc = download_live(X, c->n, ctl.pool_top[which], start, le, lw, c->stream);
  if (rc) return rc;
  uint64_t cnt = 0;
  for (uint32_t a = 0; a < c->n; ++a)
    for (uint64_t k = start[a]; k < start[a + 1]; ++k)
      if (le[k].nbr > a) ++cnt;
  *m = cnt;
  if (cap < cnt) return DYG_OK;
  if (cnt && (!u || !v || !w)) return DYG_E_INVALID_ARG;
  uint64_t i = 0;
  for (uint32_t a = 0; a < c->n; ++a)
    for (uint64_t k = start[a]; k < start[a + 1]; ++k)
      if (le[k].nbr > a) {
        u[i] = a;
        v[i] = le[k].nbr;
        w[i] = lw[k];
        ++i;
      }
  return DYG_OK;
}

}  // namespace

extern "C" int dyg_query_sparsifier(dyg_ctx* c, uint64_t cap, uint64_t* m, uint32_t* u,
                                    uint32_t* v, double* w) {
  return query_graph(c, 1, cap, m, u, v, w);
}

extern "C" int dyg_query_graph(dyg_ctx* c, uint64_t cap, uint64_t* m, uint32_t* u, uint32_t* v,
                               double* w) {
  return query_graph(c, 0, cap, m, u, v, w);
}

extern "C" int dyg_stats(dyg_ctx* c, dyg_stats_t* out) {
  if (!c || !out) return DYG_E_INVALID_ARG;
  if (c->async_inflight) {
    int rc = dyg_sync(c);
    if (rc) return rc;
  }
  BatchCtl ctl;
  int rc = sync_ctl_host(c, ctl);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  out->n = c->n;
  for (int g = 0; g < 2; ++g) {
    const DevGraph& X = g ? c->H : c->G;
    std::vector<Row> rows(c->n);
    hipError_t e =
        hipMemcpyAsync(rows.data(), X.rows, sizeof(Row) * c->n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail_hip(e);
    uint64_t live = 0, dead = 0;
    for (const Row& r : rows) {
      live += r.h.len - r.h.dead;
      dead += r.h.dead;
    }
    if (g == 0) {
      out->g_edges = live / 2;
      out->g_dead = dead;
      out->g_pool_used = ctl.pool_top[0];
      out->g_pool_cap = X.pool_cap;
    } else {
      out->h_edges = live / 2;
      out->h_dead = dead;
      out->h_pool_used = ctl.pool_top[1];
      out->h_pool_cap = X.pool_cap;
    }
  }
  out->uid_base = c->uid_base;
  out->batches = c->batches;
  out->compactions = c->compactions;
  out->w_ref = c->w_ref;
  out->walk_steps = ctl.steps_total;
  out->walk_alg_bytes = ctl.alg_bytes_total;
  out->walk_launches = c->walk_launches;
  out->walk_ms_total = c->walk_ms_total;
  out->walk_ms_last = c->walk_ms_last;
  out->batch_ms_last = c->batch_ms_last;
  return DYG_OK;
}

namespace {

struct HostImage {
  std::vector<Row> rows;
  std::vector<Ent> ent;
  std::vector<double> w;
  std::vector<unsigned long long> tree;
  std::vector<double> rinl, winl;
  Ent get(uint32_t u, uint32_t i) const {
    if (rows[u].h.off != kInlineOff) return ent[rows[u].h.off + i];
    const Pair& p = rows[u].inl[i];
    return Ent{p.nbr, p.qw, rinl[static_cast<size_t>(u) * kInline + i]};
  }
  double wt(uint32_t u, uint32_t i) const {
    return rows[u].h.off == kInlineOff ? winl[static_cast<size_t>(u) * kInline + i]
                                       : w[rows[u].h.off + i];
  }
};

int download_image(const DevGraph& X, uint32_t n, uint64_t used, HostImage& I, hipStream_t st) {
  I.rows.resize(n);
  I.ent.resize(used);
  I.w.resize(used);
  I.tree.resize(used / 4 + dyg::kFan);
  I.rinl.resize(static_cast<size_t>(n) * kInline);
  I.winl.resize(static_cast<size_t>(n) * kInline);
  hipError_t e = hipMemcpyAsync(I.rows.data(), X.rows, sizeof(Row) * n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(I.rinl.data(), X.rinl, sizeof(double) * I.rinl.size(),
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(I.winl.data(), X.winl, sizeof(double) * I.winl.size(),
                       hipMemcpyDeviceToHost, st);
  std::vector<Pair> pairs(used);
  std::vector<double> prinv(used);
  if (e == hipSuccess && used)
    e = hipMemcpyAsync(pairs.data(), X.ent, sizeof(Pair) * used, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && used)
    e = hipMemcpyAsync(prinv.data(), X.prinv, sizeof(double) * used, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && used)
    e = hipMemcpyAsync(I.w.data(), X.w, sizeof(double) * used, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(I.tree.data(), X.tree, sizeof(unsigned long long) * I.tree.size(),
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (uint64_t i = 0; i < used; ++i) I.ent[i] = Ent{pairs[i].nbr, pairs[i].qw, prinv[i]};
  return e == hipSuccess ? DYG_OK : fail_hip(e);
}

int find_live(const HostImage& I, uint32_t a, uint32_t b) {
  const RowHdr r = I.rows[a].h;
  uint32_t lo = 0, hi = r.len;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) / 2;
    if (I.get(a, mid).nbr < b) lo = mid + 1;
    else hi = mid;
  }
  if (lo < r.len && I.get(a, lo).nbr == b && I.get(a, lo).qw != 0u) return static_cast<int>(lo);
  return -1;
}

}  // namespace

extern "C" int dyg_check_state(dyg_ctx* c, char* msg, uint64_t msg_len) {
  if (!c) return DYG_E_INVALID_ARG;
  auto fail = [&](const char* what, int g, uint64_t a, uint64_t b) {
    if (msg && msg_len)
      std::snprintf(msg, msg_len, "%s: graph %s row %llu item %llu", what, g ? "H" : "G",
                    static_cast<unsigned long long>(a), static_cast<unsigned long long>(b));
    return DYG_E_DEVICE;
  };
  if (msg && msg_len) msg[0] = 0;
  if (c->async_inflight) {
    int rc = dyg_sync(c);
    if (rc) return rc;
  }
  BatchCtl ctl;
  int rc = sync_ctl_host(c, ctl);
  if (rc) return rc;
  HostImage img[2];
  for (int g = 0; g < 2; ++g) {
    const DevGraph& X = g ? c->H : c->G;
    rc = download_image(X, c->n, ctl.pool_top[g], img[g], c->stream);
    if (rc) return rc;
    const HostImage& I = img[g];
    std::vector<std::pair<uint64_t, uint64_t>> spans;
    for (uint32_t u = 0; u < c->n; ++u) {
      const RowHdr r = I.rows[u].h;
      const bool inl = r.off == kInlineOff;
      if (r.len > r.cap) return fail("len exceeds cap", g, u, r.len);
      if (inl && r.cap != kInline) return fail("inline row capacity", g, u, r.cap);
      if (!ctl.heavy)  // the walks sum in 32 bits while the flag is clear
        for (uint32_t i = 0; i < r.len; ++i)
          if (I.get(u, i).qw >= dyg::kHeavyQw) return fail("heavy weight, flag clear", g, u, i);
      if (inl)  // the walk's inline selection relies on weight 0 past len
        for (uint32_t i = r.len; i < kInline; ++i)
          if (I.rows[u].inl[i].qw != 0u) return fail("inline slot past len in use", g, u, i);
      if (!inl && static_cast<uint64_t>(r.off) + r.cap > ctl.pool_top[g])
        return fail("segment beyond pool top", g, u, r.off);
      if (!inl && (r.off % 2 != 0 || r.cap % 2 != 0))  // the walk reads two pairs per load
        return fail("segment start or capacity odd", g, u, r.off);
      if (!inl && r.cap) spans.push_back({r.off, static_cast<uint64_t>(r.off) + r.cap});
      uint32_t dead = 0;
      for (uint32_t i = 0; i < r.len; ++i) {
        const Ent e = I.get(u, i);
        if (e.nbr >= c->n || e.nbr == u) return fail("bad neighbour id", g, u, i);
        if (i && I.get(u, i - 1).nbr >= e.nbr) return fail("segment not sorted", g, u, i);
        if (e.qw == 0u) ++dead;
        if (e.qw != 0u && !(e.rinv == 1.0 / I.wt(u, i))) return fail("1/w mismatch", g, u, i);
      }
      if (!inl && r.len > dyg::kHub) {
        // the weight tree: placement, then every value of every level
        if (r.off % dyg::kHubAlign != 0 || r.cap % dyg::kFan != 0)
          return fail("long segment not aligned for its weight tree", g, u, r.off);
        const uint32_t K = dyg::tree_top(r.len);
        std::vector<unsigned long long> tb(dyg::tree_base(r.len, K + 1));
        build_tree_host(&I.ent[r.off], r.len, tb.data());
        for (uint32_t i = 0; i < tb.size(); ++i)
          if (I.tree[r.off / 4 + i] != tb[i]) return fail("stale weight tree level >= 1", g, u, i);
        if (dyg::top_inline(r.len)) {
          // the words a walker reads: values 0 .. n-2 and the total (the
          // others keep whatever the row held before)
          Row want = I.rows[u];
          inline_top_host(want, r.len, tb.data());
          unsigned long long a[kInline], b[kInline];
          std::memcpy(a, want.inl, sizeof(a));
          std::memcpy(b, I.rows[u].inl, sizeof(b));
          const uint32_t n = dyg::tree_n(r.len, K);
          for (uint32_t j = 0; j < kInline; ++j)
            if ((j + 1 < n || j == kInline - 1) && a[j] != b[j])
              return fail("stale inline copy of the top tree block", g, u, j);
        }
      }
      if (dead != r.dead) {
        if (msg && msg_len)
          std::snprintf(msg, msg_len,
                        "tombstone count: graph %s row %u off %u len %u cap %u dead %u counted %u",
                        g ? "H" : "G", u, r.off, r.len, r.cap, r.dead, dead);
        return DYG_E_DEVICE;
      }
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
      if (spans[i].first < spans[i - 1].second) return fail("overlapping segments", g, i, 0);
    for (uint32_t u = 0; u < c->n; ++u) {
      const RowHdr r = I.rows[u].h;
      for (uint32_t i = 0; i < r.len; ++i) {
        const Ent e = I.get(u, i);
        if (e.qw == 0u) continue;
        const int j = find_live(I, e.nbr, u);
        if (j < 0) return fail("asymmetric edge", g, u, e.nbr);
        const Ent f = I.get(e.nbr, j);
        if (f.qw != e.qw || I.wt(e.nbr, j) != I.wt(u, i))
          return fail("asymmetric weight", g, u, e.nbr);
      }
    }
  }
  for (uint32_t u = 0; u < c->n; ++u) {
    const RowHdr r = img[1].rows[u].h;
    for (uint32_t i = 0; i < r.len; ++i) {
      const Ent e = img[1].get(u, i);
      if (e.qw == 0u) continue;
      const int j = find_live(img[0], u, e.nbr);
      if (j < 0) return fail("H edge missing from G", 1, u, e.nbr);
      if (img[0].wt(u, j) != img[1].wt(u, i)) return fail("H weight differs from G", 1, u, e.nbr);
    }
  }
  return DYG_OK;
}

extern "C" int dyg_get_tuning(dyg_ctx* c, dyg_tuning* out) {
  if (!c || !out) return DYG_E_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  out->walk_blocks_per_cu = c->walk_blocks_per_cu;
  out->refill_min = c->refill_min;
  out->updates_per_wave = c->updates_per_wave;
  out->tail_lanes = c->tail_lanes;
  out->lockstep = c->lockstep;
  return DYG_OK;
}

extern "C" int dyg_set_tuning(dyg_ctx* c, const dyg_tuning* t) {
  if (!c || !t) return DYG_E_INVALID_ARG;
  if (t->walk_blocks_per_cu < 1 || t->walk_blocks_per_cu > 64 || t->refill_min < 1 ||
      t->refill_min > 64 || t->updates_per_wave > dyg::kMaxUpw || t->tail_lanes > 64 ||
      t->lockstep > 1)
    return DYG_E_INVALID_ARG;
  c->walk_blocks_per_cu = t->walk_blocks_per_cu;
  c->refill_min = t->refill_min;
  c->updates_per_wave = t->updates_per_wave;
  c->tail_lanes = t->tail_lanes;
  c->lockstep = t->lockstep;
  return DYG_OK;
}

extern "C" int dyg_reserve(dyg_ctx* c, uint64_t max_ins, uint64_t max_del, uint32_t max_s,
                           uint32_t max_L) {
  if (!c || max_ins + max_del >= (1ull << 30) || max_s > DYG_MAX_WALKERS ||
      max_L > DYG_MAX_STEPS)
    return DYG_E_INVALID_ARG;
  if (c->async_inflight) {
    int rc = dyg_sync(c);
    if (rc) return rc;
  }
  const uint64_t nu = max_ins + max_del;
  const uint32_t Lcap = std::max<uint32_t>(std::max<uint32_t>(max_L, c->params.L_default), 2);
  const uint32_t scap = std::max<uint32_t>(max_s, c->params.s_default);
  uint64_t hadd_cap, hash_slots;
  if (prepare_buffers(c, max_ins, max_del, Lcap, 0, nu * scap, hadd_cap, hash_slots))
    return DYG_E_NOMEM;
  // host-array batches stage through these
  if (!c->iu.ensure(4 * max_ins + 8) || !c->iv.ensure(4 * max_ins + 8) ||
      !c->iw.ensure(8 * max_ins + 8) || !c->du.ensure(4 * max_del + 8) ||
      !c->dv.ensure(4 * max_del + 8) || !c->s.ensure(2 * nu + 8) || !c->L.ensure(2 * nu + 8) ||
      !c->pin_in.ensure(24 * nu + 64))
    return DYG_E_NOMEM;
  return DYG_OK;
}

extern "C" int dyg_compact(dyg_ctx* c) {
  if (!c) return DYG_E_INVALID_ARG;
  if (c->async_inflight) {
    int rc = dyg_sync(c);
    if (rc) return rc;
  }
  for (int g = 0; g < 2; ++g) {
    int rc = compact_graph(c, g, 0);
    if (rc) return rc;
  }
  return DYG_OK;
}

extern "C" void dyg_destroy(dyg_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->static_inflight) {
    // a batch on a caller stream may still use the static working memory
    (void)hipEventSynchronize(c->done_ev);
    release_static(c);
  }
  free_graph(c->G);
  free_graph(c->H);
  if (c->ctl) (void)hipFree(c->ctl);
  if (c->dargs) (void)hipFree(c->dargs);
  if (c->dargv) (void)hipFree(c->dargv);
  if (c->hargs) (void)hipHostFree(c->hargs);
  if (c->hctl) (void)hipHostFree(c->hctl);
  if (c->done_ev) (void)hipEventDestroy(c->done_ev);
  DBuf* bufs[] = {&c->iu, &c->iv, &c->iw, &c->du, &c->dv, &c->s, &c->L, &c->ins_qw,
                  &c->ins_rinv, &c->in_h, &c->res, &c->ubytes, &c->wrec, &c->wofs, &c->hadd,
                  &c->hash};
  for (DBuf* b : bufs) b->release();
  c->hash2.release();
  c->fb_list.release();
  DBuf* qbufs[] = {&c->qcount, &c->qofs, &c->qtile, &c->items, &c->wres, &c->tstate, &c->tcount};
  for (DBuf* b : qbufs) b->release();
  for (int g = 0; g < 2; ++g) {
    c->touched_rows[g].release();
    c->touched_k[g].release();
    c->touched_need[g].release();
    c->add_keep[g].release();
    c->dirty_rows[g].release();
    c->dirty_chunk0[g].release();
    c->dirty_small[g].release();
    c->wide_rows[g].release();
    c->wmerge[g].release();
  }
  c->pin_in.release();
  c->pin_out.release();
  for (hipEvent_t ev : c->ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

// ---------------------------------------------------------------------------
// Serving: continuous batching over many resident graphs.

namespace {

struct ServerRequest {
  uint64_t id = 0;
  uint32_t graph = 0;
  std::vector<uint32_t> iu, iv, du, dv;
  std::vector<double> iw;
  dyg_update_result* out = nullptr;
  double t_submit = 0, t_start = 0, t_done = 0;
  uint64_t mem = 0;
  int status = DYG_OK;
  uint64_t nu() const { return iu.size() + du.size(); }
};

struct ServerRound {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  BatchCtl* qctl = nullptr;              // shared work-queue control (device)
  const BatchArgs** argv = nullptr;      // device, kMaxFused entries
  const BatchArgs** argv_host = nullptr; // pinned staging of argv
  DBuf items, wres;
  HBuf pin_out;                          // per request: control block + results
  std::vector<ServerRequest*> reqs;
  std::vector<size_t> out_ofs;
  uint64_t mem = 0;
  bool busy = false;
};

}  // namespace

struct dyg_server {
  dyg_server_params p{};
  std::vector<dyg_ctx*> graphs;
  std::vector<std::deque<ServerRequest*>> queues;
  std::vector<uint8_t> busy;
  std::vector<ServerRound> rounds;
  uint64_t mem_in_flight = 0;
  uint64_t next_id = 1;
  uint64_t pending = 0;
  std::deque<dyg_request_done> finished;
  std::chrono::steady_clock::time_point t0;
};

namespace {

double server_clock(const dyg_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

// Working memory a batch holds while in flight (device staging, hash, queue
// items and walker records, phase-4 scratch), for admission.
uint64_t batch_memory(const dyg_ctx* c, uint64_t n_ins, uint64_t n_del) {
  const uint64_t nu = n_ins + n_del;
  const uint64_t L = std::max<uint32_t>(c->params.L_default, 2);
  const uint64_t hadd = n_ins + n_del * L;
  const uint64_t items = nu * c->params.s_default;
  return 32 * nu + sizeof(AddRec) * hadd + 2 * 16 * std::max<uint64_t>(nu, 2 * hadd) +
         (sizeof(dyg::WalkItem) + sizeof(dyg_walker_record)) * items + 30 * (2 * n_ins + 2 * hadd);
}

int round_init(ServerRound& r) {
  hipError_t e = hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r.done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&r.qctl, sizeof(BatchCtl));
  if (e == hipSuccess) e = hipMalloc(&r.argv, sizeof(BatchArgs*) * dyg::kMaxFused);
  if (e == hipSuccess)
    e = hipHostMalloc(&r.argv_host, sizeof(BatchArgs*) * dyg::kMaxFused, hipHostMallocDefault);
  return e == hipSuccess ? DYG_OK : fail_hip(e);
}

void round_free(ServerRound& r) {
  if (r.stream) (void)hipStreamSynchronize(r.stream);
  r.items.release();
  r.wres.release();
  r.pin_out.release();
  if (r.qctl) (void)hipFree(r.qctl);
  if (r.argv) (void)hipFree(r.argv);
  if (r.argv_host) (void)hipHostFree(r.argv_host);
  if (r.done) (void)hipEventDestroy(r.done);
  if (r.stream) (void)hipStreamDestroy(r.stream);
  r = ServerRound{};
}

// Stage request q's batch into its context and fill the context's batch
// arguments for a fused launch on round r.  Returns the arguments.
int stage_request(ServerRound& r, ServerRequest* q, dyg_ctx* c, uint64_t item_cap_total,
                  BatchArgs** out) {
  const uint64_t n_ins = q->iu.size(), n_del = q->du.size(), nu = n_ins + n_del;
  const uint32_t Lcap = std::max<uint32_t>(c->params.L_default, 2);
  uint64_t hadd_cap, hash_slots;
  if (prepare_buffers(c, n_ins, n_del, Lcap, 0, 0, hadd_cap, hash_slots)) return DYG_E_NOMEM;
  if (c->params.flags & DYG_FLAG_BATCHED) {
    // the context's own queue buffers are not used in a fused round
  }
  if (!c->iu.ensure(4 * n_ins + 8) || !c->iv.ensure(4 * n_ins + 8) ||
      !c->iw.ensure(8 * n_ins + 8) || !c->du.ensure(4 * n_del + 8) ||
      !c->dv.ensure(4 * n_del + 8) || !c->qcount.ensure(4 * nu + 8) ||
      !c->qofs.ensure(8 * nu + 8) || !c->qtile.ensure(8 * ((nu + 1023) / 1024 + 1) + 8))
    return DYG_E_NOMEM;
  const size_t in_bytes = 16 * n_ins + 8 * n_del + 64;
  if (!c->pin_in.ensure(in_bytes)) return DYG_E_NOMEM;
  char* h = static_cast<char*>(c->pin_in.p);
  hipError_t e = hipSuccess;
  auto put = [&](DBuf& dst, const void* src, size_t bytes) {
    if (!bytes || e != hipSuccess) return;
    std::memcpy(h, src, bytes);
    e = hipMemcpyAsync(dst.p, h, bytes, hipMemcpyHostToDevice, r.stream);
    h += (bytes + 15) & ~size_t(15);
  };
  put(c->iu, q->iu.data(), 4 * n_ins);
  put(c->iv, q->iv.data(), 4 * n_ins);
  put(c->iw, q->iw.data(), 8 * n_ins);
  put(c->du, q->du.data(), 4 * n_del);
  put(c->dv, q->dv.data(), 4 * n_del);
  if (e != hipSuccess) return fail_hip(e);
  BatchArgs& a = make_args(c, n_ins, n_del, c->iu.as<uint32_t>(), c->iv.as<uint32_t>(),
                           c->iw.as<double>(), c->du.as<uint32_t>(), c->dv.as<uint32_t>(),
                           nullptr, nullptr, Lcap, hadd_cap, hash_slots,
                           c->res.as<dyg::UpdRes>(), false);
  a.qctl = r.qctl;
  a.items = r.items.as<dyg::WalkItem>();
  a.wres = r.wres.as<dyg::WalkOut>();
  a.tail_lanes = 0;  // serving rounds use the range walk or the work queue
  a.tstate = nullptr;
  a.tcount = nullptr;
  (void)item_cap_total;
  e = hipMemcpyAsync(c->dargs, &a, sizeof(BatchArgs), hipMemcpyHostToDevice, r.stream);
  if (e != hipSuccess) return fail_hip(e);
  *out = &a;
  return DYG_OK;
}

// Launch round r over its admitted requests.
int launch_round(dyg_server* s, ServerRound& r) {
  const uint32_t F = static_cast<uint32_t>(r.reqs.size());
  uint64_t items = 0;
  for (ServerRequest* q : r.reqs) items += q->nu() * s->graphs[q->graph]->params.s_default;
  const bool queue = s->graphs[r.reqs[0]->graph]->updates_per_wave == 0;
  if ((queue && !r.items.ensure(sizeof(dyg::WalkItem) * items + 64)) ||
      !r.wres.ensure(sizeof(dyg::WalkOut) * items + 64))
    return DYG_E_NOMEM;
  dyg::Launch L{};
  L.argv = r.argv;
  L.F = F;
  L.walk_blocks = s->graphs[r.reqs[0]->graph]->cus * s->p.walk_blocks_per_cu;
  L.upw = s->graphs[r.reqs[0]->graph]->updates_per_wave;
  for (ServerRequest* q : r.reqs) L.hubs = L.hubs || s->graphs[q->graph]->has_hubs;
  size_t out_bytes = 0;
  r.out_ofs.assign(F, 0);
  for (uint32_t i = 0; i < F; ++i) {
    r.out_ofs[i] = out_bytes;
    out_bytes += sizeof(BatchCtl) + sizeof(dyg_update_result) * r.reqs[i]->nu() + 16;
    out_bytes = (out_bytes + 15) & ~size_t(15);
  }
  if (!r.pin_out.ensure(out_bytes + 64)) return DYG_E_NOMEM;
  for (uint32_t i = 0; i < F; ++i) {
    ServerRequest* q = r.reqs[i];
    dyg_ctx* c = s->graphs[q->graph];
    BatchArgs* a = nullptr;
    int rc = stage_request(r, q, c, items, &a);
    if (rc) return rc;
    r.argv_host[i] = c->dargs;
    L.max_nu = std::max<uint32_t>(L.max_nu, a->n_ins + a->n_del);
    L.max_ins = std::max<uint32_t>(L.max_ins, a->n_ins);
    L.max_del = std::max<uint32_t>(L.max_del, a->n_del);
    L.max_hadd_cap = std::max<uint64_t>(L.max_hadd_cap, a->hadd_cap);
    L.max_hash_slots = std::max<uint64_t>(L.max_hash_slots, a->hash_slots);
  }
  hipError_t e = hipMemcpyAsync(r.argv, r.argv_host, sizeof(BatchArgs*) * F,
                                hipMemcpyHostToDevice, r.stream);
  if (e != hipSuccess) return fail_hip(e);
  dyg::launch_batch_begin(L, r.stream);
  dyg::launch_validate(L, r.stream);
  dyg::launch_phase1(L, r.stream);
  dyg::launch_queue_prepare(L, r.stream);
  dyg::launch_walk_queue(L, r.stream);
  dyg::launch_queue_finish(L, r.stream);
  dyg::launch_sum_counters(L, r.stream);
  dyg::launch_phase4_both(L, r.stream);
  char* o = static_cast<char*>(r.pin_out.p);
  for (uint32_t i = 0; i < F; ++i) {
    dyg_ctx* c = s->graphs[r.reqs[i]->graph];
    e = hipMemcpyAsync(o + r.out_ofs[i], c->ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost,
                       r.stream);
    if (e == hipSuccess && r.reqs[i]->nu())
      e = hipMemcpyAsync(o + r.out_ofs[i] + sizeof(BatchCtl), c->res.p,
                         sizeof(dyg_update_result) * r.reqs[i]->nu(), hipMemcpyDeviceToHost,
                         r.stream);
    if (e != hipSuccess) return fail_hip(e);
  }
  if ((e = hipEventRecord(r.done, r.stream)) != hipSuccess) return fail_hip(e);
  if ((e = hipGetLastError()) != hipSuccess) return fail_hip(e);
  return DYG_OK;
}

// A graph whose pool repair failed takes no more batches: its waiting
// requests finish with `rc` at once (their state could no longer be that of
// the requests before them applied in order).
void fail_waiting(dyg_server* s, uint32_t g, int rc) {
  const double now = server_clock(s);
  while (!s->queues[g].empty()) {
    ServerRequest* q = s->queues[g].front();
    s->queues[g].pop_front();
    s->finished.push_back(dyg_request_done{q->id, q->graph, rc, q->nu(), q->t_submit, now, now});
    delete q;
  }
}

// A finished round: decide each request, finish pool repairs, report.
void retire_round(dyg_server* s, ServerRound& r) {
  const double now = server_clock(s);
  const char* o = static_cast<const char*>(r.pin_out.p);
  for (size_t i = 0; i < r.reqs.size(); ++i) {
    ServerRequest* q = r.reqs[i];
    dyg_ctx* c = s->graphs[q->graph];
    BatchCtl ctl;
    std::memcpy(&ctl, o + r.out_ofs[i], sizeof(BatchCtl));
    int rc = decode_err(ctl.err_key);
    if (!rc && (ctl.nomem[0] || ctl.nomem[1])) {
      // rare: a pool ran short; finish this batch's phase 4 alone
      rc = repair_nomem(c, *c->hargs, ctl);
      if (!rc) {
        const hipError_t e = hipMemcpy(const_cast<char*>(o) + r.out_ofs[i] + sizeof(BatchCtl),
                                       c->res.p, sizeof(dyg_update_result) * q->nu(),
                                       hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail_hip(e);
      } else {
        c->broken = true;
      }
    }
    if (!rc) {
      c->uid_base += q->nu();
      c->batches++;
      c->pool_top[0] = ctl.pool_top[0];
      c->pool_top[1] = ctl.pool_top[1];
      if (q->out && q->nu())
        std::memcpy(q->out, o + r.out_ofs[i] + sizeof(BatchCtl),
                    sizeof(dyg_update_result) * q->nu());
      rc = maybe_compact(c);
    }
    q->status = rc;
    q->t_done = now;
    dyg_request_done d{q->id, q->graph, rc, q->nu(), q->t_submit, q->t_start, q->t_done};
    s->finished.push_back(d);
    s->busy[q->graph] = 0;
    if (c->broken) fail_waiting(s, q->graph, rc ? rc : DYG_E_NOMEM);
    delete q;
  }
  s->mem_in_flight -= r.mem;
  r.mem = 0;
  r.reqs.clear();
  r.busy = false;
}

// Admit the oldest waiting heads of idle graphs into round r.
void admit(dyg_server* s, ServerRound& r) {
  std::vector<uint32_t> cand;
  for (uint32_t g = 0; g < s->graphs.size(); ++g)
    if (!s->busy[g] && !s->queues[g].empty() && !s->graphs[g]->broken) cand.push_back(g);
  std::sort(cand.begin(), cand.end(), [&](uint32_t a, uint32_t b) {
    return s->queues[a].front()->id < s->queues[b].front()->id;
  });
  for (uint32_t g : cand) {
    if (r.reqs.size() >= s->p.max_fused) break;
    ServerRequest* q = s->queues[g].front();
    const bool alone = s->mem_in_flight == 0 && r.reqs.empty();
    if (!alone && s->mem_in_flight + r.mem + q->mem > s->p.mem_budget) continue;
    s->queues[g].pop_front();
    s->busy[g] = 1;
    r.reqs.push_back(q);
    r.mem += q->mem;
  }
}

}  // namespace

extern "C" void dyg_server_default_params(dyg_server_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->mem_budget = 8ull << 30;
  p->max_fused = 32;
  p->max_inflight = 2;
  p->walk_blocks_per_cu = 4;
}

extern "C" int dyg_server_create(dyg_server** out, const dyg_server_params* p) {
  if (!out || !p || p->max_fused < 1 || p->max_fused > dyg::kMaxFused || p->max_inflight < 1 ||
      p->max_inflight > 8 || p->walk_blocks_per_cu < 1 || p->walk_blocks_per_cu > 64)
    return DYG_E_INVALID_ARG;
  dyg_server* s = new (std::nothrow) dyg_server();
  if (!s) return DYG_E_NOMEM;
  s->p = *p;
  s->t0 = std::chrono::steady_clock::now();
  s->rounds.resize(p->max_inflight);
  for (ServerRound& r : s->rounds) {
    int rc = round_init(r);
    if (rc) {
      dyg_server_destroy(s);
      return rc;
    }
  }
  *out = s;
  return DYG_OK;
}

extern "C" int dyg_server_add_graph(dyg_server* s, dyg_ctx* ctx, uint32_t* graph_id) {
  if (!s || !ctx || !graph_id) return DYG_E_INVALID_ARG;
  // fused rounds run every update of a batch in one walk launch
  if (ctx->params.flags & DYG_FLAG_TWO_STAGE) return DYG_E_INVALID_ARG;
  if (ctx->async_inflight) {
    int rc = dyg_sync(ctx);
    if (rc) return rc;
  }
  *graph_id = static_cast<uint32_t>(s->graphs.size());
  s->graphs.push_back(ctx);
  s->queues.emplace_back();
  s->busy.push_back(0);
  return DYG_OK;
}

extern "C" int dyg_server_submit(dyg_server* s, uint32_t graph_id, uint64_t n_ins,
                                 const uint32_t* iu, const uint32_t* iv, const double* iw,
                                 uint64_t n_del, const uint32_t* du, const uint32_t* dv,
                                 dyg_update_result* results, uint64_t* request_id) {
  if (!s || graph_id >= s->graphs.size()) return DYG_E_INVALID_ARG;
  if ((n_ins && (!iu || !iv || !iw)) || (n_del && (!du || !dv))) return DYG_E_INVALID_ARG;
  if (n_ins + n_del >= (1ull << 30)) return DYG_E_INVALID_ARG;
  ServerRequest* q = new (std::nothrow) ServerRequest();
  if (!q) return DYG_E_NOMEM;
  q->id = s->next_id++;
  q->graph = graph_id;
  q->iu.assign(iu, iu + n_ins);
  q->iv.assign(iv, iv + n_ins);
  q->iw.assign(iw, iw + n_ins);
  q->du.assign(du, du + n_del);
  q->dv.assign(dv, dv + n_del);
  q->out = results;
  q->t_submit = server_clock(s);
  q->mem = batch_memory(s->graphs[graph_id], n_ins, n_del);
  s->queues[graph_id].push_back(q);
  s->pending++;
  if (request_id) *request_id = q->id;
  return DYG_OK;
}

extern "C" int dyg_server_poll(dyg_server* s, dyg_request_done* done, uint32_t cap,
                               uint32_t* n_done) {
  if (!s) return DYG_E_INVALID_ARG;
  for (ServerRound& r : s->rounds) {
    if (!r.busy) continue;
    const hipError_t e = hipEventQuery(r.done);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) return fail_hip(e);
    retire_round(s, r);
  }
  // graphs broken outside the server (or before their requests arrived)
  for (uint32_t g = 0; g < s->graphs.size(); ++g)
    if (s->graphs[g]->broken && !s->busy[g] && !s->queues[g].empty())
      fail_waiting(s, g, DYG_E_NOMEM);
  for (ServerRound& r : s->rounds) {
    if (r.busy) continue;
    admit(s, r);
    if (r.reqs.empty()) break;
    const double now = server_clock(s);
    for (ServerRequest* q : r.reqs) q->t_start = now;
    s->mem_in_flight += r.mem;
    r.busy = true;
    int rc = launch_round(s, r);
    if (rc) {
      (void)hipStreamSynchronize(r.stream);
      for (ServerRequest* q : r.reqs) {
        q->status = rc;
        q->t_done = server_clock(s);
        s->finished.push_back(
            dyg_request_done{q->id, q->graph, rc, q->nu(), q->t_submit, q->t_start, q->t_done});
        s->busy[q->graph] = 0;
        delete q;
      }
      s->mem_in_flight -= r.mem;
      r.mem = 0;
      r.reqs.clear();
      r.busy = false;
      return rc;
    }
  }
  uint32_t k = 0;
  while (k < cap && !s->finished.empty()) {
    if (done) done[k] = s->finished.front();
    s->finished.pop_front();
    ++k;
    s->pending--;
  }
  if (n_done) *n_done = k;
  return DYG_OK;
}

extern "C" uint64_t dyg_server_pending(const dyg_server* s) { return s ? s->pending : 0; }

extern "C" double dyg_server_now(const dyg_server* s) { return s ? server_clock(s) : 0.0; }

extern "C" void dyg_server_destroy(dyg_server* s) {
  if (!s) return;
  for (ServerRound& r : s->rounds) round_free(r);
  for (auto& qd : s->queues)
    for (ServerRequest* q : qd) delete q;
  delete s;
}
