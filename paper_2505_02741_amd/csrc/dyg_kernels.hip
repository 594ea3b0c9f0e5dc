// HIP kernels of one dyGRASS update batch on gfx950.
//
// Batch pipeline (Sec. III-F: the GPU version applies a batch's updates at
// the end of the batch), every step on one stream, no host round trip:
//   begin     reset the batch control block and the hash table
//   validate  per-update checks; the first failing update (in uid order) is
//             kept in ctl->err_key and every later kernel becomes a no-op
//   phase 1   deleted edges become tombstones in G and, if present, in H
//             (Sec. III-C: an edge outside H leaves H unchanged)
//   walks     one wavefront per update, one lane per walker, lanes stepping
//             in lockstep: weight-biased non-backtracking walks (Sec. III-B)
//             on H for insertions and on G for deletions (Sec. III-C); ballot
//             for "some walker reached q", wavefront argmin for the least
//             resistance (Eq. 12); a deletion replays its winner to emit the
//             path edges missing from H, or the fallback edges when nobody hit
//             (the batched form splits this step: walker counts and offsets,
//             a walk schedule — head/tail, range or work queue — and a
//             per-update reduction that takes the decisions)
//   phase 4   G += insertions, H += accepted + recovered edges: revive
//             tombstones, append into per-node slack, relocate a segment that
//             overflows, then merge the appended tail into sorted order
#include "dyg_internal.h"
#include "dyg_philox.h"

#include <math.h>

namespace dyg {
namespace {

constexpr int kWave = 64;
constexpr int kWalkBlock = 256;  // four updates per workgroup
constexpr int kBlock = 256;
// Workgroup of the lockstep walk kernel.  On graphs with hub rows the
// wavefronts' lifetimes are heavy-tailed (a few updates walk long chains of
// weight-tree levels), and a compute unit takes a new workgroup only when it
// has room for all of its wavefronts, so there a workgroup is one wavefront;
// elsewhere four.
template <bool kHubs>
constexpr int kLockstepBlock = kHubs ? kWave : kWalkBlock;

enum : int {
  E_INVALID_ARG = 1,
  E_SELF_LOOP = 2,
  E_VERTEX_RANGE = 3,
  E_BAD_WEIGHT = 4,
  E_EDGE_EXISTS = 5,
  E_EDGE_MISSING = 6,
  E_DUPLICATE = 7,
};

// ---- argument loading -------------------------------------------------------------

// A pointer read from device memory is generic to the compiler, which then
// accesses it with flat instructions and can neither keep uniform arguments
// in scalar registers nor aggregate uniform atomics.  Every buffer of this
// library is global memory: the argument records and the pointers they hold
// are read here as global (address space 1) pointers, which the compiler
// propagates to every access made through them.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

// Pointer stored at global address f, pointing to global memory.
template <class T>
__device__ __forceinline__ T* load_gptr(T* const __attribute__((address_space(1)))* f) {
  const uint64_t bits = *reinterpret_cast<const uint64_t __attribute__((address_space(1)))*>(f);
  return (T*)(gptr<T>)bits;
}

// Argument record of batch b of the launch.
__device__ __forceinline__ gptr<const BatchArgs> args_of(const BatchArgs* const* __restrict__ argv,
                                                        uint32_t b) {
  return (gptr<const BatchArgs>)argv[b];
}

__device__ __forceinline__ void load_graph(DevGraph& X, gptr<const BatchArgs> ap, int w) {
  X.rows = load_gptr(&ap->g[w].rows);
  X.ent = load_gptr(&ap->g[w].ent);
  X.prinv = load_gptr(&ap->g[w].prinv);
  X.w = load_gptr(&ap->g[w].w);
  X.rinl = load_gptr(&ap->g[w].rinl);
  X.winl = load_gptr(&ap->g[w].winl);
  X.pending = load_gptr(&ap->g[w].pending);
  X.tree = load_gptr(&ap->g[w].tree);
  X.mark = load_gptr(&ap->g[w].mark);
}

// Arguments of batch b of the launch, read once at kernel entry.
__device__ __forceinline__ BatchArgs load_args(const BatchArgs* const* __restrict__ argv,
                                               uint32_t b) {
  const gptr<const BatchArgs> ap = args_of(argv, b);
  BatchArgs a;
  __builtin_memcpy(&a, (const BatchArgs*)ap, sizeof(BatchArgs));
  a.iu = load_gptr(&ap->iu);
  a.iv = load_gptr(&ap->iv);
  a.iw = load_gptr(&ap->iw);
  a.du = load_gptr(&ap->du);
  a.dv = load_gptr(&ap->dv);
  a.s = load_gptr(&ap->s);
  a.L = load_gptr(&ap->L);
  a.ins_qw = load_gptr(&ap->ins_qw);
  a.ins_rinv = load_gptr(&ap->ins_rinv);
  a.in_h = load_gptr(&ap->in_h);
  a.res = load_gptr(&ap->res);
  a.wrec = load_gptr(&ap->wrec);
  a.wofs = load_gptr(&ap->wofs);
  a.hadd = load_gptr(&ap->hadd);
  a.ubytes = load_gptr(&ap->ubytes);
  a.fb_list = load_gptr(&ap->fb_list);
  a.hash = load_gptr(&ap->hash);
  a.hash2 = load_gptr(&ap->hash2);
  load_graph(a.g[0], ap, 0);
  load_graph(a.g[1], ap, 1);
  a.ctl = load_gptr(&ap->ctl);
  a.qctl = load_gptr(&ap->qctl);
  for (int w = 0; w < 2; ++w) {
    a.touched_rows[w] = load_gptr(&ap->touched_rows[w]);
    a.touched_k[w] = load_gptr(&ap->touched_k[w]);
    a.touched_need[w] = load_gptr(&ap->touched_need[w]);
    a.add_keep[w] = load_gptr(&ap->add_keep[w]);
    a.dirty_rows[w] = load_gptr(&ap->dirty_rows[w]);
    a.dirty_chunk0[w] = load_gptr(&ap->dirty_chunk0[w]);
    a.dirty_small[w] = load_gptr(&ap->dirty_small[w]);
    a.wide_rows[w] = load_gptr(&ap->wide_rows[w]);
  }
  a.qcount = load_gptr(&ap->qcount);
  a.qofs = load_gptr(&ap->qofs);
  a.qtile = load_gptr(&ap->qtile);
  a.items = load_gptr(&ap->items);
  a.wres = load_gptr(&ap->wres);
  return a;
}

// Control block of batch b of the launch.
__device__ __forceinline__ BatchCtl* ctl_of(const BatchArgs* const* __restrict__ argv, uint32_t b) {
  return load_gptr(&args_of(argv, b)->ctl);
}

__device__ __forceinline__ bool batch_failed(const BatchCtl* c) {
  return c->err_key != ~0ull;
}

__device__ __forceinline__ unsigned long long edge_key(uint32_t a, uint32_t b) {
  const uint32_t lo = a < b ? a : b;
  const uint32_t hi = a < b ? b : a;
  return (static_cast<unsigned long long>(lo) << 32) | hi;
}

// Header of row u.
__device__ __forceinline__ RowHdr row_hdr(const DevGraph& X, uint32_t u) {
  return X.rows[u].h;
}

__device__ __forceinline__ RowHdr& row_hdr_ref(const DevGraph& X, uint32_t u) {
  return X.rows[u].h;
}

// Entries of one row, inline or in the pool: entry i has its (nbr, qw) pair
// at pair[i], its 1/w at rinv[i] and its weight at w[i].
struct Seg {
  Pair* pair;
  double* rinv;
  double* w;
  __device__ __forceinline__ uint32_t nbr(uint32_t i) const { return pair[i].nbr; }
  __device__ __forceinline__ uint32_t& qw(uint32_t i) const { return pair[i].qw; }
  __device__ __forceinline__ double& r(uint32_t i) const { return rinv[i]; }
  __device__ __forceinline__ Ent get(uint32_t i) const { return Ent{nbr(i), qw(i), r(i)}; }
  __device__ __forceinline__ void put(uint32_t i, const Ent& e, double wt) const {
    pair[i] = Pair{e.nbr, e.qw};
    r(i) = e.rinv;
    w[i] = wt;
  }
};

// Row u's entries (off: its header's pool offset or kInlineOff).
__device__ __forceinline__ Seg seg_of(const DevGraph& X, uint32_t u, uint32_t off) {
  if (off == kInlineOff) {
    const uint64_t b = static_cast<uint64_t>(u) * kInline;
    return Seg{&X.rows[u].inl[0], X.rinl + b, X.winl + b};
  }
  return Seg{X.ent + off, X.prinv + off, X.w + off};
}

// Index of neighbour v among the first len entries (tombstones included), or -1.
__device__ __forceinline__ int find_nbr(const Seg& seg, uint32_t len, uint32_t v) {
  int lo = 0, hi = static_cast<int>(len) - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const uint32_t x = seg.nbr(mid);
    if (x == v) return mid;
    if (x < v) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// First index among the first len entries whose neighbour is >= v.
__device__ __forceinline__ uint32_t lower_nbr(const Seg& seg, uint32_t len, uint32_t v) {
  uint32_t lo = 0, hi = len;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (seg.nbr(mid) < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The same for a pool segment.
__device__ __forceinline__ int find_nbr_pool(const Pair* seg, uint32_t len, uint32_t v) {
  int lo = 0, hi = static_cast<int>(len) - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const uint32_t x = seg[mid].nbr;
    if (x == v) return mid;
    if (x < v) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

__device__ __forceinline__ bool has_live(const DevGraph& X, uint32_t a, uint32_t b) {
  const RowHdr h = row_hdr(X, a);
  const Seg seg = seg_of(X, a, h.off);
  const int k = find_nbr(seg, h.len, b);
  return k >= 0 && seg.qw(k) != 0u;
}

// ---- weight trees of long segments ---------------------------------------------
// (layout in dyg_internal.h)

// The kFan values of one tree block (128 bytes, 16-byte aligned).
__device__ __forceinline__ void tree_block(const unsigned long long* p, unsigned long long v[kFan]) {
  const ulonglong2* p2 = reinterpret_cast<const ulonglong2*>(p);
#pragma unroll
  for (uint32_t j = 0; j < kFan / 2; ++j) {
    const ulonglong2 x = p2[j];
    v[2 * j] = x.x;
    v[2 * j + 1] = x.y;
  }
}

// Child of a block for residual target r: the number of its values at or
// below r (they never decrease along the block, and padding never counts);
// r becomes the residual within that child.
__device__ __forceinline__ uint32_t tree_child(const unsigned long long v[kFan],
                                               unsigned long long& r) {
  uint32_t c = 0;
  unsigned long long below = 0;
#pragma unroll
  for (uint32_t j = 0; j < kFan; ++j) {
    const bool le = v[j] <= r;
    c += le ? 1u : 0u;
    below = le ? v[j] : below;
  }
  r -= below;
  return c;
}

// Level 0 of a long segment's weight tree is not stored: leaf block `node`
// is read as its kFan (neighbour, weight) pairs (128 bytes, 16-byte
// aligned: long segments start at multiples of kHubAlign and own multiples
// of kFan slots), whose running weight sums are the level-0 values.  Only
// the weights are kept; the picked pair is read again afterwards, from the
// line this read just brought in.
struct Leaf {
  uint32_t qw[kFan];
};

__device__ __forceinline__ void leaf_pairs(const Pair* seg, uint32_t node, Leaf& f) {
  const uint4* p = reinterpret_cast<const uint4*>(seg + kFan * node);
#pragma unroll
  for (uint32_t j = 0; j < kFan / 2; ++j) {
    const uint4 x = p[j];
    f.qw[2 * j] = x.y;
    f.qw[2 * j + 1] = x.w;
  }
}

// Entries of a leaf whose running weight sum is at or below r; the n
// entries of the leaf that belong to the segment count (the slots after
// them are padding, above any target).
__device__ __forceinline__ uint32_t leaf_count(const Leaf& f, uint32_t n, unsigned long long r) {
  unsigned long long run = 0;
  uint32_t c = 0;
#pragma unroll
  for (uint32_t j = 0; j < kFan; ++j) {
    run += f.qw[j];
    c += (j < n && run <= r) ? 1u : 0u;
  }
  return c;
}

// Entries of a segment of len entries in leaf block `node`.
__device__ __forceinline__ uint32_t leaf_len(uint32_t len, uint32_t node) {
  return len - kFan * node < kFan ? len - kFan * node : kFan;
}

// First entry of a long segment whose running weight total exceeds t
// (t < the segment total): one block per level, top to bottom, then the
// leaf's pairs.
__device__ __forceinline__ uint32_t tree_find(const Pair* seg, const unsigned long long* tb,
                                              uint32_t len, unsigned long long t) {
  const uint32_t K = tree_top(len);
  unsigned long long v[kFan];
  uint32_t node = 0;
  for (uint32_t l = K; l >= 1; --l) {
    tree_block(tb + tree_base(len, l) + kFan * node, v);
    node = kFan * node + tree_child(v, t);
  }
  Leaf f;
  leaf_pairs(seg, node, f);
  return kFan * node + leaf_count(f, leaf_len(len, node), t);
}

// Add `delta` (two's complement) to every stored tree value that covers
// entry k of row r's long segment at `off` with `len` entries: the rest of
// k's block on every level from 1 up, the total in the top block, and the
// top block's inline copy (level 0 follows from the entry's weight itself).  Atomic, so concurrent
// changes to one segment commute.
// The 64-bit words of row r's inline bytes (the inline copy of a long
// segment's top tree block).
__device__ __forceinline__ unsigned long long* row_top(const DevGraph& X, uint32_t r) {
  return reinterpret_cast<unsigned long long*>(&X.rows[r].inl[0]);
}

__device__ void tree_add(const DevGraph& X, uint32_t r, uint32_t off, uint32_t len, uint32_t k,
                         unsigned long long delta) {
  const uint32_t K = tree_top(len);
  unsigned long long* tb = X.tree + (off >> 2);
  uint32_t b = k;
  for (uint32_t l = 1; l <= K; ++l) {
    b >>= 4;
    const uint32_t n = tree_n(len, l);
    unsigned long long* lv = tb + tree_base(len, l);
    const uint32_t end = ((b | (kFan - 1)) + 1) < n ? ((b | (kFan - 1)) + 1) : n;
    for (uint32_t j = b; j < end; ++j) atomicAdd(&lv[j], delta);
    if (l == K && n < kFan) atomicAdd(&lv[kFan - 1], delta);  // the segment total
    if (l == K && n <= kInlineTop) {  // and the row's inline copy of the top block
      unsigned long long* it = row_top(X, r);
      for (uint32_t j = b; j + 1 < n; ++j) atomicAdd(&it[j], delta);
      atomicAdd(&it[kInline - 1], delta);
    }
  }
}

// ---- hash table (validation duplicates, phase-4 dedup) ---------------------

__device__ __forceinline__ uint32_t hash_home(unsigned long long key, uint32_t mask) {
  key ^= key >> 33;
  key *= 0xff51afd7ed558ccdull;
  key ^= key >> 33;
  key *= 0xc4ceb9fe1a85ec53ull;
  key ^= key >> 33;
  return static_cast<uint32_t>(key) & mask;
}

// Insert key; keep the minimum index seen for it.  The table holds at least
// twice as many slots as keys, so a probe sequence always meets an empty slot
// or the key within mask+1 probes.
__device__ void hash_insert_min(HashSlot* h, uint32_t mask, unsigned long long key,
                                uint32_t idx) {
  uint32_t s = hash_home(key, mask);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev = atomicCAS(&h[s].key, ~0ull, key);
    if (prev == ~0ull || prev == key) {
      atomicMin(&h[s].minidx, idx);
      return;
    }
    s = (s + 1) & mask;
  }
}

__device__ uint32_t hash_min_of(const HashSlot* h, uint32_t mask, unsigned long long key) {
  uint32_t s = hash_home(key, mask);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long k = h[s].key;
    if (k == key) return h[s].minidx;
    if (k == ~0ull) return ~0u;
    s = (s + 1) & mask;
  }
  return ~0u;
}

// True for the first inserter of key.
__device__ bool hash_insert_first(HashSlot* h, uint32_t mask, unsigned long long key) {
  uint32_t s = hash_home(key, mask);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev = atomicCAS(&h[s].key, ~0ull, key);
    if (prev == ~0ull) return true;
    if (prev == key) return false;
    s = (s + 1) & mask;
  }
  return false;
}

// ---- begin ------------------------------------------------------------------

// One workgroup per batch resets that batch's control block; the first also
// resets the work-queue control the batches share.
// Start of a batch: reset its control block (and, from batch 0, the shared
// queue control of the launch) and clear both hash tables.
__global__ void k_batch_begin(const BatchArgs* const* __restrict__ argv) {
  const gptr<const BatchArgs> ap = args_of(argv, blockIdx.y);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    BatchCtl* ctl = load_gptr(&ap->ctl);
    if (blockIdx.y == 0) {
      BatchCtl* q = load_gptr(&args_of(argv, 0)->qctl);
      q->walk_items = 0;
      q->queue_next = 0;
    }
    ctl->err_key = ~0ull;
    ctl->fb_count = 0;
    for (int w = 0; w < 2; ++w) {
      ctl->touched[w] = 0;
      ctl->stage_used[w] = 0;
      ctl->wpack[w] = 0;
      ctl->need[w] = 0;
      ctl->nomem[w] = 0;
      ctl->tpack[w] = 0;
      ctl->tsmall[w] = 0;
      ctl->wide[w] = 0;
    }
  }
  HashSlot* h1 = load_gptr(&ap->hash);
  HashSlot* h2 = load_gptr(&ap->hash2);
  const uint64_t slots = ap->hash_slots;
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < slots;
       i += uint64_t(gridDim.x) * blockDim.x) {
    h1[i].key = ~0ull;
    h1[i].minidx = ~0u;
    h2[i].key = ~0ull;
    h2[i].minidx = ~0u;
  }
}

// ---- validation ---------------------------------------------------------------

constexpr unsigned long long kDelTag = 1ull << 63;  // n < 2^31 keeps bit 63 free

__global__ void k_validate_a(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_ins + a.n_del) return;
  if (i < a.n_ins) {
    const uint32_t u = a.iu[i], v = a.iv[i];
    if (u < a.n && v < a.n && u != v) hash_insert_min(a.hash, a.hash_mask, edge_key(u, v), i);
  } else {
    const uint32_t j = i - a.n_ins;
    const uint32_t u = a.du[j], v = a.dv[j];
    if (u < a.n && v < a.n && u != v)
      hash_insert_min(a.hash, a.hash_mask, edge_key(u, v) | kDelTag, j);
  }
}

__device__ __forceinline__ void report(BatchCtl* ctl, unsigned long long phase, uint32_t idx,
                                       int code) {
  atomicMin(&ctl->err_key, (phase << 56) | (static_cast<unsigned long long>(idx) << 8) |
                               static_cast<unsigned long long>(code));
}

// Quantised weight: round-half-even(w / w_ref * 2^Q) clamped to [1, 2^32-1].
__device__ __forceinline__ uint32_t quantize(double w, double w_ref, int Q) {
  const double y = rint((w / w_ref) * ldexp(1.0, Q));
  if (!(y >= 1.0)) return 1u;
  if (y > 4294967295.0) return 4294967295u;
  return static_cast<uint32_t>(y);
}

__global__ void k_validate_b(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  const DevGraph G = a.g[0];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_ins + a.n_del) return;
  if (i < a.n_ins) {
    const uint32_t u = a.iu[i], v = a.iv[i];
    const double w = a.iw[i];
    int code = 0;
    if (u >= a.n || v >= a.n) code = E_VERTEX_RANGE;
    else if (u == v) code = E_SELF_LOOP;
    else if (!(w > 0.0) || isinf(w) || isinf(1.0 / w)) code = E_BAD_WEIGHT;
    else if (has_live(G, u, v)) code = E_EDGE_EXISTS;
    else if (hash_min_of(a.hash, a.hash_mask, edge_key(u, v)) < i) code = E_DUPLICATE;
    if (code) report(a.ctl, 0, i, code);
    else {
      const uint32_t qw = quantize(w, a.w_ref, a.Q);
      a.ins_qw[i] = qw;
      a.ins_rinv[i] = 1.0 / w;
      // later walks may meet this weight (a failed batch only costs speed)
      if (qw >= kHeavyQw) a.ctl->heavy = 1u;
    }
  } else {
    const uint32_t j = i - a.n_ins;
    const uint32_t u = a.du[j], v = a.dv[j];
    int code = 0;
    if (u >= a.n || v >= a.n) code = E_VERTEX_RANGE;
    else if (u == v) code = E_SELF_LOOP;
    else if (!has_live(G, u, v)) code = E_EDGE_MISSING;
    else if (hash_min_of(a.hash, a.hash_mask, edge_key(u, v) | kDelTag) < j) code = E_DUPLICATE;
    if (code) report(a.ctl, 1, j, code);
  }
  const uint32_t s = a.s ? a.s[i] : a.s_def;
  const uint32_t L = a.L ? a.L[i] : a.L_def;
  if (s > kMaxWalkers || s > a.scap || L > kMaxSteps || L > a.Lcap)
    report(a.ctl, 2, i, E_INVALID_ARG);
}

// ---- phase 1 -------------------------------------------------------------------

// A deleted edge becomes a tombstone in row u (weight 0; a long segment's
// weight tree loses its weight).
__device__ __forceinline__ void tombstone(const DevGraph& X, uint32_t u, uint32_t v) {
  const RowHdr h = row_hdr(X, u);
  const Seg seg = seg_of(X, u, h.off);
  const int k = find_nbr(seg, h.len, v);
  if (k < 0) return;
  const uint32_t old = seg.qw(k);  // each edge is deleted once per batch
  seg.qw(k) = 0u;
  atomicAdd(&row_hdr_ref(X, u).dead, 1u);
  if (h.len > kHub)
    tree_add(X, u, h.off, h.len, static_cast<uint32_t>(k), 0ull - static_cast<unsigned long long>(old));
}

__global__ void k_phase1(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  const DevGraph G = a.g[0];
  const DevGraph H = a.g[1];
  if (batch_failed(a.ctl)) return;
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_del) return;
  const uint32_t u = a.du[j], v = a.dv[j];
  const bool in_h = has_live(H, u, v);
  tombstone(G, u, v);
  tombstone(G, v, u);
  if (in_h) {
    tombstone(H, u, v);
    tombstone(H, v, u);
  }
  a.in_h[j] = in_h ? 1 : 0;
}

// Entries of the sorted array v[0, n) at or below x, by the whole block:
// rounds of kBlock evenly spaced probes (__syncthreads_count) narrow the
// range kBlock times per round.
__device__ uint32_t block_count_le(const uint32_t* v, uint32_t n, uint32_t x) {
  uint32_t lo = 0, hi = n;  // the answer is in [lo, hi]
  while (hi > lo) {
    const uint32_t step = (hi - lo + kBlock - 1) / kBlock;
    const uint32_t at = lo + threadIdx.x * step;
    const int below = __syncthreads_count(at < hi && v[at] <= x);
    if (below == 0) return lo;
    const uint32_t nlo = lo + (below - 1) * step + 1;
    if (step == 1) return nlo;
    const uint32_t nhi = lo + below * step;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
  return lo;
}

// Rebuild the weight tree (levels 1.. in tree) of every long
// segment listed dirty by phase 4 (merged or relocated) and longer than
// kTreeSmall entries (shorter ones: k_hub_tree_small), a chunk of
// kTreeChunk = 16^3 entries per workgroup iteration; each workgroup takes a
// contiguous share of the chunks of all rows.  A chunk fills levels 1-2 of
// its part of the tree on its own: the weights are staged in LDS with
// coalesced reads and each thread sums one block of 16 entries (level 0 is
// not stored: walks read the block's pairs).  A row longer than one
// chunk gets its chunk totals on level 3; the workgroup that finishes its
// last chunk (the row's mark counts finished chunks) sums levels 3.. from
// them.  The graph is which0 + blockIdx.z.
constexpr uint32_t kTreeChunk = kBlock * kFan;  // 4096 entries: one level-2 block
static_assert(kTreeChunk == kFan * kFan * kFan, "a chunk is one level-2 block");
constexpr uint32_t kTreeSmall = kWave * kFan;  // rows whose tree one wavefront rebuilds

__host__ __device__ constexpr uint32_t lds_pad(uint32_t i) { return i + (i >> 4); }

// Weight tree of a row of kHub < len <= kTreeSmall entries (top level 1 or
// 2) by one wavefront: lane l sums level-0 block l; level 1 is a scan of the
// block totals within groups of 16 lanes; level 2 (len > 256) sums the group
// totals; the top block also goes to the row's inline copy when it fits.
__device__ void wave_tree(const DevGraph& X, uint32_t r, const RowHdr& row, uint32_t lane) {
  const uint32_t len = row.len;
  const uint32_t K = tree_top(len);
  const uint32_t n1 = tree_n(len, 1);  // at most kWave
  const Pair* seg = X.ent + row.off;
  unsigned long long* tb = X.tree + (row.off >> 2);
  unsigned long long run = 0;  // the total of level-0 block `lane`
  if (lane < n1) {
    uint32_t q[kFan];
#pragma unroll
    for (uint32_t j = 0; j < kFan; ++j) {  // loads issued together
      const uint32_t i = kFan * lane + j;
      q[j] = i < len ? seg[i].qw : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kFan; ++j) run += q[j];
  }
  unsigned long long v1 = run;  // block total; running sum within 16 lanes next
  for (uint32_t d = 1; d < kFan; d <<= 1) {
    const unsigned long long o = __shfl_up(v1, d, kFan);
    if ((lane & (kFan - 1)) >= d) v1 += o;
  }
  const unsigned long long g0 = __shfl(v1, kFan - 1, kWave), g1 = __shfl(v1, 2 * kFan - 1, kWave);
  const unsigned long long g2 = __shfl(v1, 3 * kFan - 1, kWave), g3 = __shfl(v1, 4 * kFan - 1, kWave);
  const unsigned long long total = g0 + g1 + g2 + g3;
  if (lane < round_fan(n1))
    tb[lane] = (K == 1 && lane == kFan - 1) ? total : (lane < n1 ? v1 : kTreePad);
  unsigned long long* it = row_top(X, r);  // the top block's inline copy
  if (K == 1 && n1 <= kInlineTop && lane + 1 < n1) it[lane] = v1;
  if (K == 2 && lane < kFan) {
    const uint32_t n2 = tree_n(len, 2);  // at most 4: always inline
    const unsigned long long v2 =
        g0 + (lane >= 1 ? g1 : 0ull) + (lane >= 2 ? g2 : 0ull) + (lane >= 3 ? g3 : 0ull);
    tb[tree_base(len, 2) + lane] = lane == kFan - 1 ? total : (lane < n2 ? v2 : kTreePad);
    if (lane + 1 < n2) it[lane] = v2;
  }
  if (lane == 0 && top_inline(len)) it[kInline - 1] = total;
}

// Weight trees of the rows of at most kTreeSmall entries listed by phase 4,
// a wavefront each (no LDS, so the grid runs at full occupancy).  The graph
// is which0 + blockIdx.z.
__global__ __launch_bounds__(kBlock) void k_hub_tree_small(const BatchArgs* const* __restrict__ argv,
                                                           uint32_t which0) {
  const uint32_t which = which0 + blockIdx.z;
  const gptr<const BatchArgs> ap = args_of(argv, blockIdx.y);
  BatchCtl* ctl = load_gptr(&ap->ctl);
  if (batch_failed(ctl)) return;
  DevGraph X;
  load_graph(X, ap, static_cast<int>(which));
  const uint32_t* small = load_gptr(&ap->dirty_small[which]);
  const uint32_t ns = static_cast<uint32_t>(ctl->tsmall[which]);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  for (uint32_t q = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; q < ns;
       q += gridDim.x * (kBlock / kWave)) {
    const uint32_t r = small[q];
    wave_tree(X, r, row_hdr(X, r), lane);
    if (lane == 0) X.mark[r] = 0u;
  }
}

__global__ __launch_bounds__(kBlock) void k_hub_tree(const BatchArgs* const* __restrict__ argv,
                                                     uint32_t which0) {
  const uint32_t which = which0 + blockIdx.z;
  const gptr<const BatchArgs> ap = args_of(argv, blockIdx.y);
  BatchCtl* ctl = load_gptr(&ap->ctl);
  if (batch_failed(ctl)) return;
  DevGraph X;
  load_graph(X, ap, static_cast<int>(which));
  const uint32_t* dirty_rows = load_gptr(&ap->dirty_rows[which]);
  const uint32_t* chunk0 = load_gptr(&ap->dirty_chunk0[which]);
  const unsigned long long pack = ctl->tpack[which];
  const uint32_t rows = static_cast<uint32_t>(pack), units = static_cast<uint32_t>(pack >> 32);
  __shared__ uint32_t s_q[lds_pad(kTreeChunk)];  // weights of the chunk
  __shared__ unsigned long long s_t[kBlock];               // block totals
  __shared__ uint32_t s_last;
  const uint32_t t = threadIdx.x;
  // a contiguous share of the units: one search finds the first unit's row,
  // the others follow in order (a row's chunks are consecutive units)
  const uint32_t per = (units + gridDim.x - 1) / gridDim.x;
  const uint32_t u0 = blockIdx.x * per < units ? blockIdx.x * per : units;
  const uint32_t u1 = u0 + per < units ? u0 + per : units;
  if (u0 == u1) return;  // block-uniform
  uint32_t p = block_count_le(chunk0, rows, u0) - 1;
  uint32_t r = dirty_rows[p];
  RowHdr row = row_hdr(X, r);  // len > kHub: a pool segment, aligned
  uint32_t first = chunk0[p];
  for (uint32_t u = u0; u < u1; ++u) {
    if (u >= first + (row.len + kTreeChunk - 1) / kTreeChunk) {
      first += (row.len + kTreeChunk - 1) / kTreeChunk;
      r = dirty_rows[++p];
      row = row_hdr(X, r);
    }
    const uint32_t ch = u - first;
    const uint32_t len = row.len;
    const uint32_t K = tree_top(len);
    const uint32_t n1 = tree_n(len, 1), n2 = tree_n(len, 2);
    const Pair* seg = X.ent + row.off;
    unsigned long long* tb = X.tree + (row.off >> 2);
    unsigned long long* l1 = tb;  // tree_base(len, 1) == 0
    unsigned long long* l2 = tb + tree_base(len, 2);
    const uint32_t chunks = (len + kTreeChunk - 1) / kTreeChunk;
    const uint32_t e0 = ch * kTreeChunk;
    const uint32_t ne = len - e0 < kTreeChunk ? len - e0 : kTreeChunk;
#pragma unroll
    for (uint32_t j = 0; j < kFan; ++j) {
      const uint32_t i = t + kBlock * j;
      s_q[lds_pad(i)] = i < ne ? seg[e0 + i].qw : 0u;
    }
    __syncthreads();
    // thread t: the total of level-0 block t of the chunk (level 0 itself is
    // not stored)
    unsigned long long run = 0;
#pragma unroll
    for (uint32_t j = 0; j < kFan; ++j) run += s_q[lds_pad(kFan * t + j)];
    s_t[t] = run;
    __syncthreads();
    // level 1: value b = running sum of block totals within b's group of 16
    const uint32_t b = ch * kBlock + t;  // level-1 index of block t
    {
      unsigned long long v1 = 0;
      for (uint32_t j = t & ~(kFan - 1); j <= t; ++j) v1 += s_t[j];
      if (b < round_fan(n1)) l1[b] = b < n1 ? v1 : kTreePad;
    }
    __syncthreads();
    // group totals (level-2 inputs) into s_t[0..15], chunk total
    unsigned long long gsum = 0;
    if (t < kFan)
      for (uint32_t j = 0; j < kFan; ++j) gsum += s_t[kFan * t + j];
    __syncthreads();
    if (t < kFan) s_t[t] = gsum;
    __syncthreads();
    unsigned long long ctot = 0;
    for (uint32_t j = 0; j < kFan; ++j) ctot += s_t[j];
    if (K == 1 && t == kFan - 1) l1[kFan - 1] = ctot;  // top block slot: the total
    if (K >= 2 && t < kFan) {
      const uint32_t c = ch * kFan + t;  // level-2 index
      unsigned long long v2 = 0;
      for (uint32_t j = 0; j <= t; ++j) v2 += s_t[j];
      if (K == 2 && t == kFan - 1) l2[c] = ctot;  // top block slot: the total
      else l2[c] = c < n2 ? v2 : kTreePad;
      if (K == 2 && n2 <= kInlineTop) {  // the top block's inline copy
        unsigned long long* it = row_top(X, r);
        if (t + 1 < n2) it[t] = v2;
        if (t == kFan - 1) it[kInline - 1] = ctot;
      }
    }
    if (K >= 3 && t == 0) tb[tree_base(len, 3) + ch] = ctot;  // raw chunk total
    if (chunks == 1) {
      if (t == 0) X.mark[r] = 0u;
      __syncthreads();
      continue;
    }
    if (t == 0) {
      __threadfence();  // this chunk's total before its count
      s_last = atomicAdd(&X.mark[r], 1u) == chunks ? 1u : 0u;  // mark starts at 1
      __threadfence();  // every other chunk's total after the count
    }
    __syncthreads();
    if (s_last && t == 0) {
      // levels 3..K from the raw totals on level 3: running sums within
      // blocks of 16, each block total handed up as the next level's raw
      // value; the top block's last slot is the row total
      unsigned long long total = 0;
      for (uint32_t l = 3; l <= K; ++l) {
        const uint32_t n = tree_n(len, l);
        unsigned long long* lv = tb + tree_base(len, l);
        unsigned long long* up = l < K ? tb + tree_base(len, l + 1) : nullptr;
        unsigned long long run3 = 0;
        for (uint32_t i = 0; i < n; ++i) {
          run3 += lv[i];
          if (l == 3) total += lv[i];
          lv[i] = run3;
          if ((i & (kFan - 1)) == kFan - 1 || i == n - 1) {
            if (up) up[i >> 4] = run3;
            run3 = 0;
          }
        }
        for (uint32_t i = n; i < round_fan(n); ++i) lv[i] = kTreePad;
        if (l == K) lv[kFan - 1] = total;
        if (l == K && n <= kInlineTop) {  // the top block's inline copy
          unsigned long long* it = row_top(X, r);
          for (uint32_t i = 0; i + 1 < n; ++i) it[i] = lv[i];
          it[kInline - 1] = total;
        }
      }
      X.mark[r] = 0u;
    }
    __syncthreads();
  }
}

// ---- walks ------------------------------------------------------------------------

struct Walk {
  uint32_t steps;
  uint32_t end;
  double R;
  bool hit;
  uint32_t bytes;  // algorithmic gathered bytes of the steps taken
};

// Bytes one step must gather at a vertex of live degree d: the row (offset and
// degree, 8 B), the (id, weight) pair of every live neighbour (8 B each) and
// the resistance of the chosen edge (8 B); above 64 neighbours a cumulative-
// weight binary search instead: 32 B plus 12 B per halving.
__device__ __forceinline__ uint32_t step_bytes(uint32_t d) {
  if (d <= 64u) return 16u + 8u * d;
  return 32u + 12u * (32u - static_cast<uint32_t>(__clz(d - 1u)));
}

struct WalkParams {
  const Row* rows;
  const Pair* ent;
  const double* prinv;
  const unsigned long long* tree;
  const double* rinl;
  uint32_t p, q;
  bool use_K;
  double w_pq, K;
  uint32_t L;
  uint32_t key0, key1, uid_lo, uid_hi;
  bool bounce;
  bool heavy;  // a weight may reach kHeavyQw: 64-bit running sums
  bool both;   // odd walkers start at q and aim at p
};

// Walker `walker`'s own start (p) and target (q): the endpoints swap for odd
// walkers under the both-ends variant.
__device__ __forceinline__ void walker_ends(WalkParams& P, uint32_t walker) {
  if (P.both && (walker & 1u)) {
    const uint32_t t = P.p;
    P.p = P.q;
    P.q = t;
  }
}

// Emits nothing; the replay variant below passes an edge sink.
struct NoSink {
  __device__ __forceinline__ void operator()(uint32_t, uint32_t, uint32_t, uint32_t) const {}
};

// State of one walker between steps.
struct WState {
  uint32_t x, prev, steps, block_of, bytes;
  uint32_t qprev;  // quantised weight of the edge just taken (the same both ways)
  double R;
  const double* rpend;  // 1/w of the last edge taken, not yet added to R (else kZeroR)
  Philox4 rnd;
  bool hit;
};

// What a walker's pending resistance points to when nothing is pending:
// adding it leaves R unchanged (R >= 0), so the pending addition needs no test.
__device__ double kZeroR = 0.0;  // never written

__device__ __forceinline__ void walker_start(WState& S, uint32_t p) {
  S.x = p;
  S.prev = kNone;
  S.qprev = 0;
  S.steps = 0;
  S.block_of = kNone;
  S.bytes = 0;
  S.R = 0.0;
  S.rpend = &kZeroR;
  S.hit = false;
}

__device__ __forceinline__ unsigned long long step_random(WState& S, const WalkParams& P,
                                                          uint32_t walker, uint32_t t) {
  if (S.block_of != (t >> 1)) {
    S.rnd = philox4x32_10(t >> 1, walker, P.uid_lo, P.uid_hi, P.key0, P.key1);
    S.block_of = t >> 1;
  }
  return (t & 1u) ? (uint64_t(S.rnd.x2) | (uint64_t(S.rnd.x3) << 32))
                  : (uint64_t(S.rnd.x0) | (uint64_t(S.rnd.x1) << 32));
}

// step_random for lanes stepping in lockstep from step 0 (t uniform): the
// block of steps t, t+1 is drawn at every even t.
__device__ __forceinline__ unsigned long long step_random_lockstep(WState& S, const WalkParams& P,
                                                                   uint32_t walker, uint32_t t) {
  if ((t & 1u) == 0u) S.rnd = philox4x32_10(t >> 1, walker, P.uid_lo, P.uid_hi, P.key0, P.key1);
  return (t & 1u) ? (uint64_t(S.rnd.x2) | (uint64_t(S.rnd.x3) << 32))
                  : (uint64_t(S.rnd.x0) | (uint64_t(S.rnd.x1) << 32));
}

// floor(r * tot / 2^64), the selection target.  With tot < 2^32 (every row
// of fewer than 256 neighbours whose weights do not exceed w_ref) the high
// half of the 128-bit product takes two 32x32 products: r*tot = rh*tot*2^32 +
// rl*tot, and rh*tot + floor(rl*tot / 2^32) < 2^64.
__device__ __forceinline__ unsigned long long scale_random(unsigned long long r,
                                                           unsigned long long tot) {
  if ((tot >> 32) == 0) {
    const unsigned long long lo = (r & 0xFFFFFFFFull) * tot;
    return ((r >> 32) * tot + (lo >> 32)) >> 32;
  }
  return __umul64hi(r, tot);
}

// One step of a walker: weight-biased choice among the neighbours other than
// the previous vertex; stop on the distortion threshold, on reaching q, at a
// dead end or after L steps (Sec. III-B).  Returns false once the walker has
// stopped (then S holds its final state; finish_walk completes R).  The whole 64-byte row
// is loaded at once: for a vertex with at most kInline neighbours it is the
// only dependent access of the step.  Without a threshold nothing decides on
// R before the walk ends, so the 1/w of the edge taken is loaded with the next
// step's row and added then (the additions keep their order).
// kHubs: the graphs may hold rows longer than kHub (else that branch, and the
// bookkeeping it needs, are compiled out).
//
// walk_step_row takes the step's inputs already loaded: t = S.steps (a
// caller stepping lanes in lockstep passes its wavefront-uniform count),
// rprev = *S.rpend,
// the row of S.x as four 16-byte pieces (ignored once
// S.steps >= P.L), and the step's random number step_random(S, P, walker,
// S.steps).  walk_step loads them itself.
template <bool kHubs, class Sink>
__device__ __forceinline__ bool walk_step_row(const WalkParams& P, WState& S, Sink& sink,
                                              uint32_t t, double rprev, unsigned long long rnd,
                                              const uint4 q0, const uint4 q1, const uint4 q2,
                                              const uint4 q3) {
  if (t >= P.L) {
    S.R = S.R + rprev;
    S.rpend = &kZeroR;
    return false;
  }
  const RowHdr h{q0.x, q0.y, q0.z, q0.w};
  uint32_t pick_nbr, pick_idx, pick_q, sbytes;
  const double* pick_r;
  bool stop = false;
  if (h.off == kInlineOff) {
    // inline pairs (nbr, qw): q1 = pairs 0-1, q2 = 2-3, q3 = 4-5.  The slots
    // at and past len hold weight 0 (an inline row is zeroed when laid out
    // and only grows), as do tombstones, so leaving out the previous vertex
    // is the only masking the selection needs.
    static_assert(kInline == 6, "inline branch reads six pairs");
    const uint32_t n0 = q1.x, n1 = q1.z, n2 = q2.x, n3 = q2.z, n4 = q3.x, n5 = q3.z;
    const uint32_t c0 = n0 != S.prev ? q1.y : 0u;
    const uint32_t c1 = n1 != S.prev ? q1.w : 0u;
    const uint32_t c2 = n2 != S.prev ? q2.y : 0u;
    const uint32_t c3 = n3 != S.prev ? q2.w : 0u;
    const uint32_t c4 = n4 != S.prev ? q3.y : 0u;
    const uint32_t c5 = n5 != S.prev ? q3.w : 0u;
    // Running sums r0..r4 and tot; the pick is the first index whose running
    // sum exceeds the target, i.e. the number of running sums r0..r4 at or
    // below it (they never decrease, and a zero weight never crosses the
    // target).  With every weight below kHeavyQw = 2^29 the six-term sums
    // fit 32 bits exactly; once the context holds a heavier weight (a
    // context-wide flag, uniform) the walks take the 64-bit sums.
    bool b1, b2, b3, b4, b5;  // pick index >= 1 .. >= 5
    bool leaf;
    if (!P.heavy) {
      const uint32_t r0 = c0, r1 = r0 + c1, r2 = r1 + c2, r3 = r2 + c3, r4 = r3 + c4,
                     tot = r4 + c5;
      const uint32_t tg = static_cast<uint32_t>(scale_random(rnd, tot));
      leaf = tot == 0u;
      b1 = r0 <= tg;
      b2 = r1 <= tg;
      b3 = r2 <= tg;
      b4 = r3 <= tg;
      b5 = r4 <= tg;
    } else {
      const unsigned long long r0 = c0, r1 = r0 + c1, r2 = r1 + c2, r3 = r2 + c3, r4 = r3 + c4,
                               tot = r4 + c5;
      const unsigned long long tg = scale_random(rnd, tot);
      leaf = tot == 0ull;
      b1 = r0 <= tg;
      b2 = r1 <= tg;
      b3 = r2 <= tg;
      b4 = r3 <= tg;
      b5 = r4 <= tg;
    }
    // chains of selects on the monotone flags (an index compare chain would
    // cost the compares again, an equality chain would become a branch tree)
    pick_idx = b5 ? 5u : b4 ? 4u : b3 ? 3u : b2 ? 2u : b1 ? 1u : 0u;
    pick_nbr = b5 ? n5 : b4 ? n4 : b3 ? n3 : b2 ? n2 : b1 ? n1 : n0;
    pick_q = b5 ? q3.w : b4 ? q3.y : b3 ? q2.w : b2 ? q2.y : b1 ? q1.w : q1.y;
    if (leaf) {
      // the walker stops, or steps back along the edge just used
      stop = true;
      if (P.bounce && S.prev != kNone) {
        const uint32_t back = (h.len > 0 && n0 == S.prev)   ? 0u
                              : (h.len > 1 && n1 == S.prev) ? 1u
                              : (h.len > 2 && n2 == S.prev) ? 2u
                              : (h.len > 3 && n3 == S.prev) ? 3u
                              : (h.len > 4 && n4 == S.prev) ? 4u
                              : (h.len > 5 && n5 == S.prev) ? 5u
                                                            : kNone;
        stop = back == kNone;
        pick_idx = stop ? 0u : back;
        pick_nbr = S.prev;
        pick_q = pick_idx == 0u   ? q1.y
                 : pick_idx == 1u ? q1.w
                 : pick_idx == 2u ? q2.y
                 : pick_idx == 3u ? q2.w
                 : pick_idx == 4u ? q3.y
                                  : q3.w;
      }
    }
    pick_r = P.rinl + (static_cast<uint64_t>(S.x) * kInline + pick_idx);
    sbytes = 16u + 8u * (h.len - h.dead);
  } else if (kHubs && h.len > kHub) {
    // long segment: a descent of its weight tree.  The candidates are every
    // entry but the previous vertex's, whose weight (that of the edge just
    // taken) is qprev.  With i1 the first entry whose running total exceeds
    // the target and i2 the first whose running total exceeds target +
    // qprev, the pick is i1 if it lies before the previous vertex (compare
    // ids: the row is sorted) and i2 otherwise.  i2 usually shares i1's leaf
    // block, whose 16 pairs give both (their weights are the level-0 running
    // sums; the picked pair is then read from the same cache line); when the
    // two agree the comparison is moot.
    const Pair* seg = P.ent + h.off;
    const uint32_t d = h.len;
    const uint32_t K = tree_top(d);
    const uint32_t nK = tree_n(d, K);
    const unsigned long long* tb = P.tree + (h.off >> 2);
    unsigned long long v[kFan];  // the top block; slot kFan-1 = the total
    if (nK <= kInlineTop) {
      // its inline copy, read with the row: values 0 .. nK-2 and the total
      // (value nK-1 is the total too, which no target reaches: padding)
      const unsigned long long a[kInline] = {
          q1.x | (static_cast<unsigned long long>(q1.y) << 32),
          q1.z | (static_cast<unsigned long long>(q1.w) << 32),
          q2.x | (static_cast<unsigned long long>(q2.y) << 32),
          q2.z | (static_cast<unsigned long long>(q2.w) << 32),
          q3.x | (static_cast<unsigned long long>(q3.y) << 32),
          q3.z | (static_cast<unsigned long long>(q3.w) << 32)};
#pragma unroll
      for (uint32_t j = 0; j < kFan - 1; ++j) v[j] = (j + 1 < nK) ? a[j < kInline ? j : 0] : kTreePad;
      v[kFan - 1] = a[kInline - 1];
    } else {
      tree_block(tb + tree_base(d, K), v);
    }
    const uint32_t qprev = S.prev != kNone ? S.qprev : 0u;
    const unsigned long long tot = v[kFan - 1] - qprev;
    if (tot == 0) {
      // every other entry is a tombstone
      const int jp = (P.bounce && S.prev != kNone) ? find_nbr_pool(seg, h.len, S.prev) : -1;
      stop = jp < 0;
      pick_idx = jp >= 0 ? static_cast<uint32_t>(jp) : 0u;
    } else {
      const unsigned long long target = scale_random(rnd, tot);
      unsigned long long r1 = target;
      uint32_t node = tree_child(v, r1);
      for (uint32_t l = K - 1; l >= 1; --l) {
        tree_block(tb + tree_base(d, l) + kFan * node, v);
        node = kFan * node + tree_child(v, r1);
      }
      Leaf f;
      leaf_pairs(seg, node, f);
      const uint32_t in_leaf = leaf_len(d, node);
      const uint32_t c1 = leaf_count(f, in_leaf, r1);
      const uint32_t c2 = leaf_count(f, in_leaf, r1 + qprev);  // target + qprev, if in this leaf
      const uint32_t i1 = kFan * node + c1;
      pick_idx = i1;
      if (c2 != c1) {
        const uint32_t i2 = c2 < in_leaf ? kFan * node + c2 : tree_find(seg, tb, d, target + qprev);
        if (seg[i1].nbr >= S.prev) pick_idx = i2;
      }
    }
    pick_nbr = stop ? kNone : seg[pick_idx].nbr;
    pick_q = stop ? 0u : seg[pick_idx].qw;
    pick_r = P.prinv + h.off + pick_idx;
    sbytes = step_bytes(h.len - h.dead);
  } else {
    // pool segment: (nbr, qw) pairs, two per 16-byte load (the segment starts
    // at an even slot); the slot past an odd len is masked
    const Pair* seg = P.ent + h.off;
    const uint4* e4 = reinterpret_cast<const uint4*>(seg);
    const uint32_t n4 = (h.len + 1) >> 1;
    const bool odd = h.len & 1u;
    unsigned long long tot = 0;
    if (kHubs) {
#pragma unroll 8
      for (uint32_t i = 0; i < n4; ++i) {  // unrolled: the loads go out together
        const uint4 e = e4[i];
        tot += (e.x != S.prev) ? e.y : 0u;
        tot += (e.z != S.prev && (i + 1 < n4 || !odd)) ? e.w : 0u;
      }
    } else {
      for (uint32_t i = 0; i < n4; ++i) {
        const uint4 e = e4[i];
        tot += (e.x != S.prev) ? e.y : 0u;
        tot += (e.z != S.prev && (i + 1 < n4 || !odd)) ? e.w : 0u;
      }
    }
    pick_idx = 0;
    if (tot == 0) {
      const int back = (P.bounce && S.prev != kNone) ? find_nbr_pool(seg, h.len, S.prev) : -1;
      stop = back < 0;  // leaf: the walker stops (the edge just used is always live)
      pick_idx = back >= 0 ? static_cast<uint32_t>(back) : 0u;
    } else {
      const unsigned long long target = scale_random(rnd, tot);
      unsigned long long run = 0;
      pick_idx = h.len - 1;
      if (kHubs) {
#pragma unroll 8
        for (uint32_t i = 0; i < n4; ++i) {
          const uint4 e = e4[i];
          run += (e.x != S.prev) ? e.y : 0u;
          if (run > target) {
            pick_idx = 2 * i;
            break;
          }
          run += (e.z != S.prev && (i + 1 < n4 || !odd)) ? e.w : 0u;
          if (run > target) {
            pick_idx = 2 * i + 1;
            break;
          }
        }
      } else {
        for (uint32_t i = 0; i < n4; ++i) {
          const uint4 e = e4[i];
          run += (e.x != S.prev) ? e.y : 0u;
          if (run > target) {
            pick_idx = 2 * i;
            break;
          }
          run += (e.z != S.prev && (i + 1 < n4 || !odd)) ? e.w : 0u;
          if (run > target) {
            pick_idx = 2 * i + 1;
            break;
          }
        }
      }
    }
    const Pair pe = seg[pick_idx];
    pick_nbr = stop ? kNone : pe.nbr;
    pick_q = stop ? 0u : pe.qw;
    pick_r = P.prinv + h.off + pick_idx;
    sbytes = step_bytes(h.len - h.dead);
  }
  S.R = S.R + rprev;
  S.rpend = &kZeroR;
  if (stop) return false;
  S.bytes += sbytes;
  sink(S.x, pick_nbr, pick_idx, h.off);
  S.prev = S.x;
  if (kHubs) S.qprev = pick_q;
  S.x = pick_nbr;
  S.steps = t + 1;
  if (P.use_K) {
    S.R = S.R + *pick_r;
    if (P.w_pq * S.R > P.K) return false;
  } else {
    S.rpend = pick_r;
  }
  if (S.x == P.q) {
    // the last 1/w stays pending: finish_walk adds it once the walker has
    // stopped, so the wavefront does not wait for that load inside a step
    S.hit = true;
    return false;
  }
  return true;
}

// Complete R of a walker that has stopped: add the pending 1/w (R is final
// after this; kZeroR when nothing is pending).
__device__ __forceinline__ void finish_walk(WState& S) {
  S.R = S.R + *S.rpend;
  S.rpend = &kZeroR;
}

template <bool kHubs, class Sink>
__device__ __forceinline__ bool walk_step(const WalkParams& P, uint32_t walker, WState& S,
                                          Sink& sink) {
  const double rprev = *S.rpend;
  if (S.steps >= P.L)
    return walk_step_row<kHubs>(P, S, sink, S.steps, rprev, 0ull, {}, {}, {}, {});
  const uint4* rq = reinterpret_cast<const uint4*>(P.rows + S.x);
  const uint4 q0 = rq[0], q1 = rq[1], q2 = rq[2], q3 = rq[3];
  // the step's random number depends only on (walker, step, update): drawn
  // while the row is in flight (a dead end leaves it unused)
  const unsigned long long rnd = step_random(S, P, walker, S.steps);
  return walk_step_row<kHubs>(P, S, sink, S.steps, rprev, rnd, q0, q1, q2, q3);
}

template <bool kHubs, class Sink>
__device__ __forceinline__ Walk walk_one(const WalkParams& Pu, uint32_t walker, Sink& sink) {
  WalkParams P = Pu;
  walker_ends(P, walker);
  WState S;
  walker_start(S, P.p);
  while (walk_step<kHubs>(P, walker, S, sink)) {
  }
  finish_walk(S);
  return Walk{S.steps, S.x, S.R, S.hit, S.bytes};
}

// Index of this thread's wavefront in its block, as a value the compiler
// knows to be the same on every lane (so per-wavefront data stays scalar).
__device__ __forceinline__ uint32_t wave_in_block() {
  return static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave)));
}

// A compiler barrier for memory accesses.  Lanes of one wavefront exchange
// data through LDS below; the hardware keeps a wavefront's LDS accesses in
// order, so only the compiler must not move them across each other.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ uint4 ld_lds4(const volatile uint4* p) {
  return make_uint4(p->x, p->y, p->z, p->w);
}

// The walk of every lane's walker, all lanes stepping together (active =
// the lane has a walker), until every walker has stopped or, with handoff >
// 0, until at most `handoff` still walk (walk_lockstep then returns true on
// their lanes, S holding their state).  With kCoop, rows may be read
// cooperatively: load k fetches
// the rows of lanes 16k..16k+15, four lanes per row and 16 bytes per lane, so
// an instruction touches 16 cache lines instead of the 64 of a per-lane row
// read (the vector cache looks up each line an instruction touches); the
// pieces come back to their walkers through `st` (kStageWords uint4 of LDS,
// private to the wavefront): piece c of lane m's row sits at c * kStagePitch
// + m, so the reads (consecutive lanes, consecutive slots) and the writes
// (pitch 66 spreads the four pieces of a row over distinct banks) are free of
// bank conflicts.  Same results as walk_one.
constexpr uint32_t kStagePitch = kWave + 2;
constexpr uint32_t kStageWords = 4 * kStagePitch;
// The cooperative read pays off for pool rows, whose 64-byte row is only a
// header: a step reads it together with the segment.  It is used for a step
// when at least kCoopLanes walkers need a row and stood at a pool row last
// step; a launch over graphs of mostly inline rows compiles it out (kCoop),
// as its exchange only adds latency there and its registers cost occupancy.
constexpr int kCoopLanes = 8;
template <bool kHubs, bool kCoop>
__device__ __forceinline__ bool walk_lockstep(const WalkParams& Pu, uint32_t walker, bool active,
                                              uint4* st, uint32_t lane, uint32_t handoff,
                                              WState& S) {
  WalkParams P = Pu;
  walker_ends(P, walker);
  walker_start(S, P.p);
  bool alive = active;
  const uint4* rows4 = reinterpret_cast<const uint4*>(P.rows);
  const uint32_t piece = lane & 3u;
  NoSink none;
  bool at_pool = false;  // the lane's last row was a pool row
  // Every live lane has taken one step per iteration, so its step count is
  // the iteration count t, which the compiler then knows to be uniform.
  for (uint32_t t = 0;; ++t) {
    const unsigned long long live = __ballot(alive);
    if (live == 0ull || static_cast<uint32_t>(__popcll(live)) <= handoff) break;
    const bool need = alive && t < P.L;
    const unsigned long long needm = __ballot(need);
    const double rprev = alive ? *S.rpend : 0.0;
    // read only by lanes that need a row (walk_step_row ignores them past L)
    uint4 q0, q1, q2, q3;
    unsigned long long rnd;
    if (kCoop && __popcll(__ballot(need && at_pool)) >= kCoopLanes) {
      uint4 c[4];
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t src = 16u * k + (lane >> 2);
        const uint32_t xs =
            static_cast<uint32_t>(__shfl(static_cast<int>(S.x), static_cast<int>(src), kWave));
        c[k] = make_uint4(0u, 0u, 0u, 0u);
        if ((needm >> src) & 1ull) c[k] = rows4[static_cast<uint64_t>(xs) * 4u + piece];
      }
      // drawn while the rows are in flight
      rnd = step_random_lockstep(S, P, walker, t);
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) st[piece * kStagePitch + 16u * k + (lane >> 2)] = c[k];
      wave_lds_order();
      // whole 16-byte reads (volatile: not narrowed to the fields used)
      const volatile uint4* vs = st;
      q0 = ld_lds4(vs + lane);
      q1 = ld_lds4(vs + kStagePitch + lane);
      q2 = ld_lds4(vs + 2 * kStagePitch + lane);
      q3 = ld_lds4(vs + 3 * kStagePitch + lane);
      wave_lds_order();
    } else {
      // each lane reads its own row
      if (need) {
        const uint4* rq = rows4 + static_cast<uint64_t>(S.x) * 4u;
        q0 = rq[0];
        q1 = rq[1];
        q2 = rq[2];
        q3 = rq[3];
      }
      // drawn on every lane (the cost is per instruction) while rows load
      rnd = step_random_lockstep(S, P, walker, t);
    }
    at_pool = need && q0.x != kInlineOff;
    if (alive) alive = walk_step_row<kHubs>(P, S, none, t, rprev, rnd, q0, q1, q2, q3);
  }
  if (!alive) finish_walk(S);  // a walker handed on keeps its pending 1/w
  return alive;
}

template <bool kHubs, bool kCoop>
__device__ __forceinline__ Walk walk_wave(const WalkParams& P, uint32_t walker, bool active,
                                          uint4* st, uint32_t lane) {
  WState S;
  walk_lockstep<kHubs, kCoop>(P, walker, active, st, lane, 0u, S);
  return Walk{S.steps, S.x, S.R, S.hit, S.bytes};
}

// Wavefront argmin of (R, walker): smaller R wins, ties go to the lower walker.
__device__ __forceinline__ void wave_argmin(double& R, uint32_t& w) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const double oR = __shfl_xor(R, off, kWave);
    const uint32_t ow = __shfl_xor(w, off, kWave);
    if (oR < R || (oR == R && ow < w)) {
      R = oR;
      w = ow;
    }
  }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sink of the winner replay: path edges absent from H_mid, first occurrence.
// With `erase` (loop-erased variant) it keeps the loop erasure of the path
// instead: an edge x -> y whose head y is already on the kept path cuts the
// path back to y (the loop is dropped), any other is appended; drop_in_h()
// then leaves out the edges live in H.
struct RecoverSink {
  DevGraph G, H;
  AddRec* out;  // reserved block of `cap` records
  uint32_t cap;
  uint32_t count;
  bool erase;
  // edge x -> y is entry i of x's row in G (off: that row's pool offset)
  __device__ void operator()(uint32_t x, uint32_t y, uint32_t i, uint32_t off) {
    if (erase) {
      for (uint32_t z = 0; z < count; ++z)
        if (out[z].a == y) {  // y was reached before: erase the loop since then
          count = z;
          return;
        }
      if (count >= cap) return;  // cannot happen: at most one edge per step
      const Seg seg = seg_of(G, x, off);
      const Ent e = seg.get(i);
      out[count++] = AddRec{x, y, e.qw, 0u, e.rinv, seg.w[i]};
      return;
    }
    if (has_live(H, x, y)) return;
    const unsigned long long k = edge_key(x, y);
    for (uint32_t z = 0; z < count; ++z)
      if (edge_key(out[z].a, out[z].b) == k) return;
    if (count >= cap) return;
    const Seg seg = seg_of(G, x, off);
    const Ent e = seg.get(i);
    out[count] = AddRec{x, y, e.qw, 0u, e.rinv, seg.w[i]};
    ++count;
  }
  __device__ void drop_in_h() {
    uint32_t o = 0;
    for (uint32_t z = 0; z < count; ++z)
      if (!has_live(H, out[z].a, out[z].b)) out[o++] = out[z];
    count = o;
  }
};

// Sink of a replay run by every lane of a wavefront in lockstep (the same
// walk on every lane): lane t keeps the edge of step t (walks of at most
// kWave steps).
struct PathSink {
  uint32_t lane, t;
  uint32_t x, y, i, off;
  __device__ __forceinline__ void operator()(uint32_t x_, uint32_t y_, uint32_t i_,
                                             uint32_t off_) {
    if (t == lane) {
      x = x_;
      y = y_;
      i = i_;
      off = off_;
    }
    ++t;
  }
};

// Update `upd` of the batch: its endpoints, walk graph and limits.
struct UpdateView {
  WalkParams P;
  uint32_t s;
  bool is_ins;
  bool walks;  // insertions always; deletions only of H edges
};

__device__ __forceinline__ UpdateView view_update(const BatchArgs& a, const DevGraph& G,
                                                  const DevGraph& H, uint32_t upd) {
  UpdateView v;
  v.is_ins = upd < a.n_ins;
  const uint32_t j = upd - a.n_ins;
  v.s = a.s ? a.s[upd] : a.s_def;
  const uint64_t uid = a.uid_base + upd;
  WalkParams& P = v.P;
  P.p = v.is_ins ? a.iu[upd] : a.du[j];
  P.q = v.is_ins ? a.iv[upd] : a.dv[j];
  P.use_K = v.is_ins && a.has_K;
  P.w_pq = v.is_ins ? a.iw[upd] : 0.0;
  P.K = a.K;
  P.L = a.L ? a.L[upd] : a.L_def;
  P.key0 = static_cast<uint32_t>(a.seed);
  P.key1 = static_cast<uint32_t>(a.seed >> 32);
  P.uid_lo = static_cast<uint32_t>(uid);
  P.uid_hi = static_cast<uint32_t>(uid >> 32);
  P.bounce = a.bounce != 0;
  P.heavy = a.ctl->heavy != 0u;
  P.both = (a.variant & kVarBothEnds) != 0;
  P.rows = v.is_ins ? H.rows : G.rows;  // H_mid for insertions, G_mid for deletions
  P.ent = v.is_ins ? H.ent : G.ent;
  P.prinv = v.is_ins ? H.prinv : G.prinv;
  P.tree = v.is_ins ? H.tree : G.tree;
  P.rinl = v.is_ins ? H.rinl : G.rinl;
  v.walks = v.is_ins || a.in_h[j];
  return v;
}

__device__ __forceinline__ UpdRes empty_result(bool is_ins) {
  UpdRes res;
  res.kind = is_ins ? 0 : 1;
  res.flag = 0;
  res.any_hit = 0;
  res.reserved = 0;
  res.winner = 0xFFFF;
  res.n_rec = 0;
  res.steps = 0;
  res.reserved2 = 0;
  res.Rmin = INFINITY;
  return res;
}

// H additions have fixed slots: insertion i owns slot i, deletion j owns the
// a.Lcap slots from n_ins + j * a.Lcap (unused ones hold kNoAdd).
constexpr AddRec kNoAdd{kNone, kNone, 0u, 0u, 0.0, 0.0};

__device__ __forceinline__ AddRec* del_slots(const BatchArgs& a, uint32_t upd) {
  return a.hadd + a.n_ins + static_cast<uint64_t>(upd - a.n_ins) * a.Lcap;
}

// An update without walks (a deletion of an edge not in H): empty result and
// empty slots, written by the lanes of one wavefront.
__device__ __forceinline__ void no_walk_update(const BatchArgs& a, const UpdateView& v,
                                               uint32_t upd, uint32_t lane) {
  if (a.wrec)
    for (uint32_t k = lane; k < v.s; k += kWave)
      a.wrec[a.wofs[upd] + k] = WalkerRec{0, 0, 0, v.P.p, 0.0};
  if (!v.is_ins) {
    AddRec* out = del_slots(a, upd);
    for (uint32_t z = lane; z < a.Lcap; z += kWave) out[z] = kNoAdd;
  }
  if (lane == 0) {
    a.res[upd] = empty_result(v.is_ins);
    a.ubytes[upd] = 0u;
  }
}

// No-hit fallback (Sec. III-C, local edges near the deleted edge): the G
// edge at `end` of least resistance 1/w (largest weight) that is not live in
// H, ties to the smaller neighbour.  Thread `part` of `parts` scans one
// contiguous slice of end's G row, merging it against end's H row (both
// sorted by neighbour), and returns its slice's best (br = INFINITY, bn =
// kNone if none); the caller takes the minimum of (br, bn) over the parts.
// Rows longer than kWideFallback are left to k_fallback_wide (a workgroup).
constexpr uint32_t kWideFallback = 1024;
constexpr uint32_t kFallbackUnroll = 8;  // G entries loaded together
constexpr uint32_t kFallbackLds = 12288;  // H-row entries k_fallback_wide stages in LDS
constexpr uint32_t kFallbackSearch = 8192;  // largest step of its searches (2 * 8192 > kFallbackLds)
constexpr uint32_t kFbBlock = 1024;  // threads of a k_fallback_wide workgroup (one long row each)

__device__ __forceinline__ void fallback_slice(const DevGraph& G, const DevGraph& H, uint32_t end,
                                               uint32_t part, uint32_t parts, double& br,
                                               uint32_t& bn, uint32_t& bi) {
  const RowHdr r = row_hdr(G, end);
  const Seg seg = seg_of(G, end, r.off);
  const RowHdr hr = row_hdr(H, end);
  const Seg hseg = seg_of(H, end, hr.off);
  const uint32_t per = (r.len + parts - 1) / parts;
  const uint32_t a0 = part * per < r.len ? part * per : r.len;
  const uint32_t a1 = a0 + per < r.len ? a0 + per : r.len;
  uint32_t j = a0 < a1 ? lower_nbr(hseg, hr.len, seg.nbr(a0)) : hr.len;
  br = INFINITY;
  bn = kNone;
  bi = 0;
  for (uint32_t i0 = a0; i0 < a1; i0 += kFallbackUnroll) {
    uint32_t en[kFallbackUnroll], eq[kFallbackUnroll];
    double er[kFallbackUnroll];
#pragma unroll
    for (uint32_t m = 0; m < kFallbackUnroll; ++m) {  // loads issued together
      const uint32_t i = i0 + m < a1 ? i0 + m : a1 - 1;
      en[m] = seg.nbr(i);
      eq[m] = seg.qw(i);
      er[m] = seg.r(i);
    }
#pragma unroll
    for (uint32_t m = 0; m < kFallbackUnroll; ++m) {
      if (i0 + m >= a1 || eq[m] == 0u) continue;
      while (j < hr.len && hseg.nbr(j) < en[m]) ++j;
      if (j < hr.len && hseg.nbr(j) == en[m] && hseg.qw(j) != 0u) continue;  // live in H
      if (er[m] < br || (er[m] == br && en[m] < bn)) {
        br = er[m];
        bn = en[m];
        bi = i0 + m;
      }
    }
  }
}

// Decision of one update once its walkers are reduced, taken by the whole
// wavefront (every lane holds the same any_hit, bestR, bestW, steps): an
// insertion is kept iff no walker reached q (Sec. III-B); a deletion of an H
// edge recovers the winner's path edges missing from H (one lane replays the
// winner), or the fallback edges when nobody hit (Sec. III-C), whose search
// over the endpoints' G rows the lanes share.
template <bool kHubs>
__device__ __forceinline__ void decide_update(const BatchArgs& a, const DevGraph& Gref,
                                              const DevGraph& Href, uint32_t upd,
                                              const UpdateView& v, bool any_hit, double bestR,
                                              uint32_t bestW, uint32_t steps, uint32_t lane) {
  // value copies: the inline-or-pool choices below then select between
  // registers, not between fields of the argument record
  const DevGraph G = Gref, H = Href;
  UpdRes res = empty_result(v.is_ins);
  res.any_hit = any_hit ? 1 : 0;
  res.steps = steps;
  if (any_hit) {
    res.Rmin = bestR;
    res.winner = static_cast<uint16_t>(bestW);
  }
  const WalkParams& P = v.P;
  if (v.is_ins) {
    res.flag = any_hit ? 0 : 1;
    if (lane == 0) {
      a.hadd[upd] = any_hit ? kNoAdd
                            : AddRec{P.p, P.q, a.ins_qw[upd], 0u, a.ins_rinv[upd], a.iw[upd]};
      a.res[upd] = res;
    }
    return;
  }
  res.flag = 1;
  const uint32_t cap = P.L > 2 ? P.L : 2;  // <= a.Lcap
  AddRec* out = del_slots(a, upd);
  uint32_t count = 0;
  if (any_hit && P.L <= kWave) {
    // every lane replays the winner (same counters, same snapshot); lane t
    // then checks step t's edge against H and against the earlier steps
    PathSink ps{lane, 0u, kNone, kNone, 0u, 0u};
    const Walk wk = walk_one<kHubs>(P, bestW, ps);
    const bool mine = lane < wk.steps;
    const unsigned long long key = mine ? edge_key(ps.x, ps.y) : ~0ull;
    unsigned long long path = wk.steps >= kWave ? ~0ull : (1ull << wk.steps) - 1ull;
    if (a.variant & kVarLoopErased) {
      // loop erasure: with x_t the vertex step t leaves, the erased path
      // leaves x_0 at its last visit s0, then x_(s0+1) at its last visit,
      // and so on up to the target (reached once, at the end)
      uint32_t last = lane;
      for (uint32_t t = 0; t < wk.steps; ++t)
        if (static_cast<uint32_t>(__shfl(static_cast<int>(ps.x), static_cast<int>(t), kWave)) ==
            ps.x)
          last = t;
      path = 0ull;
      for (uint32_t i = 0; i < wk.steps;) {  // uniform
        const uint32_t sg =
            static_cast<uint32_t>(__shfl(static_cast<int>(last), static_cast<int>(i), kWave));
        path |= 1ull << sg;
        i = sg + 1;
      }
    }
    bool keep = mine && ((path >> lane) & 1ull) && !has_live(H, ps.x, ps.y);
    for (uint32_t t = 0; t < wk.steps; ++t) {  // first occurrence in path order
      const unsigned long long k2 = __shfl(key, static_cast<int>(t), kWave);
      if (t < lane && ((path >> t) & 1ull) && k2 == key) keep = false;
    }
    const unsigned long long kept = __ballot(keep);
    if (keep) {
      const Seg seg = seg_of(G, ps.x, ps.off);
      const Ent e = seg.get(ps.i);
      const uint32_t pos = static_cast<uint32_t>(__popcll(kept & ((1ull << lane) - 1ull)));
      out[pos] = AddRec{ps.x, ps.y, e.qw, 0u, e.rinv, seg.w[ps.i]};
    }
    count = static_cast<uint32_t>(__popcll(kept));  // <= steps <= cap
  } else if (any_hit) {
    if (lane == 0) {
      RecoverSink sink{G, H, out, cap, 0u, (a.variant & kVarLoopErased) != 0};
      walk_one<kHubs>(P, bestW, sink);  // replay: same counters, same snapshot
      if (sink.erase) sink.drop_in_h();
      count = sink.count;
    }
    count = static_cast<uint32_t>(__shfl(static_cast<int>(count), 0, kWave));
  } else if (row_hdr(G, P.p).len > kWideFallback || row_hdr(G, P.q).len > kWideFallback) {
    // no hit at a long row: the fallback scan is left to k_fallback_wide,
    // which gives it a workgroup (n_rec and the slots are written there)
    if (lane == 0) a.fb_list[atomicAdd(&a.ctl->fb_count, 1u)] = upd;
  } else {
    // no hit: per endpoint the least-resistance G edge not in H, ties to the
    // smaller neighbour; each lane scans a slice of the G row, then the
    // wavefront's minimum of (1/w, neighbour)
    for (int z = 0; z < 2; ++z) {
      const uint32_t end = z == 0 ? P.p : P.q;
      double br;
      uint32_t bn, bi;
      const RowHdr r = row_hdr(G, end);
      const Seg seg = seg_of(G, end, r.off);
      fallback_slice(G, H, end, lane, kWave, br, bn, bi);
      double wr = br;
      uint32_t wn = bn;
      wave_argmin(wr, wn);
      if (wn == kNone) continue;  // uniform: every lane holds the same minimum
      const unsigned long long own = __ballot(bn == wn);
      const uint32_t src = static_cast<uint32_t>(__builtin_ctzll(own));
      bi = static_cast<uint32_t>(__shfl(static_cast<int>(bi), static_cast<int>(src), kWave));
      if (lane == 0) out[count] = AddRec{end, wn, seg.qw(bi), 0u, seg.r(bi), seg.w[bi]};
      ++count;
    }
  }
  for (uint32_t z = count + lane; z < a.Lcap; z += kWave) out[z] = kNoAdd;
  if (lane == 0) {
    res.n_rec = static_cast<uint16_t>(count);
    a.res[upd] = res;
  }
}

// Plain form: one wavefront per update, one lane per walker (more walkers
// than lanes run in successive rounds of 64), walks and decision in one
// kernel, so one update's decision overlaps other updates' walks.
template <bool kHubs, bool kCoop>
__global__ __launch_bounds__(kLockstepBlock<kHubs>) void k_walks(
    const BatchArgs* const* __restrict__ argv, uint32_t updates) {
  __shared__ uint4 stage[kCoop ? kLockstepBlock<kHubs> / kWave : 1][kCoop ? kStageWords : 1];
  const BatchArgs a = load_args(argv, blockIdx.y);
  const DevGraph G = a.g[0];
  const DevGraph H = a.g[1];
  if (batch_failed(a.ctl)) return;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t upd = blockIdx.x * (kLockstepBlock<kHubs> / kWave) + wave_in_block();
  if (upd >= a.n_ins + a.n_del) return;  // uniform across the wavefront
  // two-stage batches: stage 1 takes the deletions, stage 2 the insertions
  if ((updates == kStageDeletions && upd < a.n_ins) ||
      (updates == kStageInsertions && upd >= a.n_ins))
    return;
  const UpdateView v = view_update(a, G, H, upd);
  if (!v.walks) {
    no_walk_update(a, v, upd, lane);
    return;
  }
  bool any_hit = false;
  double bestR = INFINITY;
  uint32_t bestW = kNone;
  uint32_t steps = 0, bytes = 0;
  for (uint32_t base = 0; base < v.s; base += kWave) {
    const uint32_t walker = base + lane;
    const bool active = walker < v.s;
    const Walk o =
        walk_wave<kHubs, kCoop>(v.P, walker, active, stage[kCoop ? wave_in_block() : 0], lane);
    if (active && a.wrec)
      a.wrec[a.wofs[upd] + walker] =
          WalkerRec{static_cast<uint8_t>(o.hit), 0, static_cast<uint16_t>(o.steps), o.end, o.R};
    const bool h = active && o.hit;
    any_hit = any_hit || (__ballot(h) != 0ull);
    double cR = h ? o.R : INFINITY;
    uint32_t cW = h ? walker : kNone;
    wave_argmin(cR, cW);
    // a later round only wins with a strictly smaller R; a hit whose sum
    // overflowed to +inf still names its walker when nothing better exists
    if (cW != kNone && (bestW == kNone || cR < bestR)) {
      bestR = cR;
      bestW = cW;
    }
    steps += wave_sum(active ? o.steps : 0u);
    bytes += wave_sum(active ? o.bytes : 0u);
  }
  if (lane == 0) a.ubytes[upd] = bytes;
  decide_update<kHubs>(a, G, H, upd, v, any_hit, bestR, bestW, steps, lane);
}

// ---- batched form: walker work queue ----------------------------------------

// Walkers per update once phase 1 is known.
__global__ void k_count_walkers(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  if (batch_failed(a.ctl)) return;
  const uint32_t upd = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nu = a.n_ins + a.n_del;
  if (upd >= nu) return;
  const bool walks = upd < a.n_ins || a.in_h[upd - a.n_ins];
  a.qcount[upd] = walks ? (a.s ? a.s[upd] : a.s_def) : 0u;
}

// Exclusive scan of qcount into qofs (u64), in three launches.
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const unsigned long long o = __shfl_up(v, off, kWave);
    if (lane >= static_cast<uint32_t>(off)) v += o;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ unsigned long long block_excl_scan(unsigned long long v, unsigned long long& excl) {
  __shared__ unsigned long long wsum[kBlock / kWave];
  const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const unsigned long long inc = wave_incl_scan(v);
  if (lane == kWave - 1) wsum[wv] = inc;
  __syncthreads();
  unsigned long long before = 0, total = 0;
  for (uint32_t k = 0; k < kBlock / kWave; ++k) {
    if (k < wv) before += wsum[k];
    total += wsum[k];
  }
  __syncthreads();
  excl = before + inc - v;
  return total;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  if (batch_failed(a.ctl)) return;
  const uint32_t nu = a.n_ins + a.n_del;
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
  unsigned long long v[kScanItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < nu) ? a.qcount[base + k] : 0u;
    sum += v[k];
  }
  unsigned long long excl;
  const unsigned long long total = block_excl_scan(sum, excl);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < nu) a.qofs[base + k] = excl;
    excl += v[k];
  }
  if (threadIdx.x == 0) a.qtile[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_top(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  const uint32_t tiles = (a.n_ins + a.n_del + kScanTile - 1) / kScanTile;
  if (batch_failed(a.ctl)) return;
  unsigned long long carry = 0;
  for (uint32_t base = 0; base < tiles; base += kBlock) {
    const uint32_t i = base + threadIdx.x;
    const unsigned long long v = i < tiles ? a.qtile[i] : 0ull;
    unsigned long long excl;
    const unsigned long long total = block_excl_scan(v, excl);
    if (i < tiles) a.qtile[i] = carry + excl;
    carry += total;
  }
  // this batch's walkers take a contiguous range of the shared queue
  if (threadIdx.x == 0) a.ctl->item_base = atomicAdd(&a.qctl->walk_items, carry);
}

__global__ __launch_bounds__(kBlock) void k_scan_add(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  if (batch_failed(a.ctl)) return;
  const uint32_t nu = a.n_ins + a.n_del;
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile;
  const unsigned long long add = a.qtile[blockIdx.x];
  for (uint32_t k = threadIdx.x; k < kScanTile; k += kBlock)
    if (base + k < nu) a.qofs[base + k] += add;
}

// Queue items: one wavefront per update writes one record per walker.
__global__ __launch_bounds__(kBlock) void k_expand_items(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  if (batch_failed(a.ctl)) return;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t upd = blockIdx.x * (kBlock / kWave) + wave_in_block();
  if (upd >= a.n_ins + a.n_del) return;
  const uint32_t cnt = a.qcount[upd];
  if (cnt == 0) return;
  const bool is_ins = upd < a.n_ins;
  const uint32_t j = upd - a.n_ins;
  WalkItem it;
  it.p = is_ins ? a.iu[upd] : a.du[j];
  it.q = is_ins ? a.iv[upd] : a.dv[j];
  it.upd = upd;
  it.L = static_cast<uint16_t>(a.L ? a.L[upd] : a.L_def);
  it.w_pq = is_ins ? a.iw[upd] : 0.0;
  const unsigned long long base = a.ctl->item_base + a.qofs[upd];
  const bool both = (a.variant & kVarBothEnds) != 0;
  for (uint32_t k = lane; k < cnt; k += kWave) {
    WalkItem mine = it;
    mine.walker = static_cast<uint16_t>(k | (blockIdx.y << kWalkerBits));
    if (both && (k & 1u)) {  // odd walkers start at q and aim at p
      mine.p = it.q;
      mine.q = it.p;
    }
    a.items[base + k] = mine;
  }
}

// Persistent walk kernel over the queue of walker items of one or more batches
// (argv[0..F), each item tagged with its batch).  A wavefront takes 64 items
// at a time with one atomic; a lane whose walker stops gets the next item of
// that pool.  The new item's record is loaded before the other lanes' step
// and used after it, so its latency hides behind the step's own loads.  Every
// walker's outcome goes to wres[item].  A batch that failed validation queued
// no items.
// Items a wavefront takes from the shared queue with one atomic.
constexpr uint32_t kQueueChunk = 4 * kWave;

// kFused: the launch carries several batches (items name theirs); otherwise
// every item belongs to batch 0 and its per-batch values stay scalar.
template <bool kFused, bool kHubs = true>
__global__ __launch_bounds__(kBlock) void k_walk_queue(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a0 = load_args(argv, 0);
  BatchCtl* q = a0.qctl;
  const WalkItem* __restrict__ items = a0.items;  // shared by all batches of the launch
  WalkOut* __restrict__ wres = a0.wres;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const unsigned long long total = q->walk_items;
  const unsigned long long lanes_below = (1ull << lane) - 1ull;
  const uint32_t refill_min = a0.refill_min < 1 ? 1u : (a0.refill_min > 64 ? 64u : a0.refill_min);
  unsigned long long pool_next = 0, pool_end = 0;  // this wavefront's items
  bool drained = false;
  bool active = false, pending = false;
  unsigned long long item = 0, next_item = 0;
  WalkItem rec{0, 0, 0, 0, 0, 0.0};
  WalkParams P;
  // per-batch values: set once here for a single batch, per item when fused
  P.K = a0.K;
  P.key0 = static_cast<uint32_t>(a0.seed);
  P.key1 = static_cast<uint32_t>(a0.seed >> 32);
  P.bounce = a0.bounce != 0;
  P.heavy = a0.ctl->heavy != 0u;
  P.both = false;  // each queue item already holds its walker's own ends
  P.rows = a0.g[1].rows;
  P.ent = a0.g[1].ent;
  P.prinv = a0.g[1].prinv;
  P.tree = a0.g[1].tree;
  P.rinl = a0.g[1].rinl;
  P.p = P.q = 0;
  P.use_K = false;
  P.w_pq = 0.0;
  P.L = 0;
  P.uid_lo = P.uid_hi = 0;
  uint32_t walker = 0;
  WState S;
  walker_start(S, 0);
  while (true) {
    // (1) hand pool items to idle lanes
    const unsigned long long idle = __ballot(!active && !pending);
    const uint32_t n_idle = static_cast<uint32_t>(__popcll(idle));
    if (n_idle && (n_idle >= refill_min || n_idle == kWave)) {
      if (pool_next >= pool_end && !drained) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&q->queue_next, static_cast<unsigned long long>(kQueueChunk));
        base = __shfl(base, 0, kWave);
        pool_next = base;
        pool_end = base < total ? (base + kQueueChunk < total ? base + kQueueChunk : total) : base;
        if (base + kQueueChunk >= total) drained = true;
      }
      const unsigned long long avail = pool_end - pool_next;
      const uint32_t take = avail < n_idle ? static_cast<uint32_t>(avail) : n_idle;
      if (!active && !pending) {
        const uint32_t rank = static_cast<uint32_t>(__popcll(idle & lanes_below));
        if (rank < take) {
          next_item = pool_next + rank;
          rec = items[next_item];
          pending = true;
        }
      }
      pool_next += take;
    }
    // (2) one step of every running walker
    NoSink none;
    if (active && !walk_step<kHubs>(P, walker, S, none)) {
      finish_walk(S);
      wres[item] = WalkOut{S.x, static_cast<uint16_t>(S.steps), static_cast<uint8_t>(S.hit), 0,
                           static_cast<uint32_t>(S.bytes), 0u, S.R};
      active = false;
    }
    // (3) lanes that received an item start its walker
    if (pending) {
      item = next_item;
      if (kFused) {
        const uint32_t b = rec.walker >> kWalkerBits;
        const gptr<const BatchArgs> A = args_of(argv, b);
        const bool is_ins = rec.upd < A->n_ins;
        const uint64_t uid = A->uid_base + rec.upd;
        P.use_K = is_ins && A->has_K;
        P.K = A->K;
        P.key0 = static_cast<uint32_t>(A->seed);
        P.key1 = static_cast<uint32_t>(A->seed >> 32);
        P.uid_lo = static_cast<uint32_t>(uid);
        P.uid_hi = static_cast<uint32_t>(uid >> 32);
        P.bounce = A->bounce != 0;
        P.heavy = load_gptr(&A->ctl)->heavy != 0u;
        const int gw = is_ins ? 1 : 0;  // H_mid for insertions, G_mid for deletions
        P.rows = load_gptr(&A->g[gw].rows);
        P.ent = load_gptr(&A->g[gw].ent);
        P.prinv = load_gptr(&A->g[gw].prinv);
        P.tree = load_gptr(&A->g[gw].tree);
        P.rinl = load_gptr(&A->g[gw].rinl);
      } else {
        const bool is_ins = rec.upd < a0.n_ins;
        const uint64_t uid = a0.uid_base + rec.upd;
        P.use_K = is_ins && a0.has_K;
        P.uid_lo = static_cast<uint32_t>(uid);
        P.uid_hi = static_cast<uint32_t>(uid >> 32);
        const DevGraph& X = is_ins ? a0.g[1] : a0.g[0];  // H_mid / G_mid
        P.rows = X.rows;
        P.ent = X.ent;
        P.prinv = X.prinv;
        P.tree = X.tree;
        P.rinl = X.rinl;
      }
      P.p = rec.p;
      P.q = rec.q;
      P.w_pq = rec.w_pq;
      P.L = rec.L;
      walker = rec.walker & ((1u << kWalkerBits) - 1u);
      walker_start(S, rec.p);
      active = true;
      pending = false;
    }
    if (!__ballot(active) && drained && pool_next >= pool_end) break;
  }
}

// Batched form, range walk: wavefront w of a batch walks every walker of
// updates [w*upw, w*upw + upw).  Walker i of the range (updates in order,
// qcount walkers each) goes to the next idle lane; a lane whose walker stops
// takes the next one, so lanes stay busy until the range runs out.  A lane
// that receives a walker loads its update's endpoints during the other lanes'
// step and starts one iteration later.  Every walker's outcome goes to
// wres[item_base + qofs[update] + walker] for the per-update reduction.
template <bool kHubs>
__global__ __launch_bounds__(kBlock) void k_walk_range(const BatchArgs* const* __restrict__ argv,
                                                       uint32_t upw) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  if (batch_failed(a.ctl)) return;
  const uint32_t nu = a.n_ins + a.n_del;
  const uint32_t u0 = (blockIdx.x * (kBlock / kWave) + wave_in_block()) * upw;
  if (u0 >= nu) return;  // uniform across the wavefront
  const uint32_t nr = (nu - u0) < upw ? (nu - u0) : upw;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const unsigned long long lanes_below = (1ull << lane) - 1ull;
  // end (exclusive) of each update's walkers within the range
  uint32_t endw[kMaxUpw];
  uint32_t total = 0;
#pragma unroll
  for (uint32_t j = 0; j < kMaxUpw; ++j) {
    if (j < nr) total += a.qcount[u0 + j];
    endw[j] = total;
  }
  const unsigned long long base = a.ctl->item_base + a.qofs[u0];
  const uint32_t refill_min = a.refill_min < 1 ? 1u : (a.refill_min > 64 ? 64u : a.refill_min);
  WalkParams P;
  P.K = a.K;
  P.key0 = static_cast<uint32_t>(a.seed);
  P.key1 = static_cast<uint32_t>(a.seed >> 32);
  P.bounce = a.bounce != 0;
  P.both = (a.variant & kVarBothEnds) != 0;
  P.heavy = a.ctl->heavy != 0u;
  P.rows = a.g[1].rows;
  P.ent = a.g[1].ent;
  P.prinv = a.g[1].prinv;
  P.tree = a.g[1].tree;
  P.rinl = a.g[1].rinl;
  P.p = P.q = 0;
  P.use_K = false;
  P.w_pq = 0.0;
  P.L = 0;
  P.uid_lo = P.uid_hi = 0;
  WState S;
  walker_start(S, 0);
  uint32_t next = 0;  // walkers of the range handed out so far (uniform)
  uint32_t walker = 0;
  unsigned long long item = 0;
  bool active = false, pending = false;
  while (true) {
    // (1) hand the next walkers of the range to idle lanes
    const unsigned long long idle = __ballot(!active && !pending);
    const uint32_t n_idle = static_cast<uint32_t>(__popcll(idle));
    if (next < total && n_idle && (n_idle >= refill_min || n_idle == kWave)) {
      const uint32_t rank = static_cast<uint32_t>(__popcll(idle & lanes_below));
      if (!active && !pending && next + rank < total) {
        const uint32_t idx = next + rank;
        uint32_t j = 0, start = 0;
#pragma unroll
        for (uint32_t k = 0; k < kMaxUpw; ++k)
          if (endw[k] <= idx) {
            j = k + 1;
            start = endw[k];
          }
        const uint32_t upd = u0 + j;
        const bool is_ins = upd < a.n_ins;
        const uint32_t jd = upd - a.n_ins;
        const uint64_t uid = a.uid_base + upd;
        P.p = is_ins ? a.iu[upd] : a.du[jd];
        P.q = is_ins ? a.iv[upd] : a.dv[jd];
        P.w_pq = is_ins ? a.iw[upd] : 0.0;
        P.use_K = is_ins && a.has_K;
        P.L = a.L ? a.L[upd] : a.L_def;
        P.uid_lo = static_cast<uint32_t>(uid);
        P.uid_hi = static_cast<uint32_t>(uid >> 32);
        const DevGraph& X = is_ins ? a.g[1] : a.g[0];  // H_mid for insertions, G_mid for deletions
        P.rows = X.rows;
        P.ent = X.ent;
        P.prinv = X.prinv;
        P.tree = X.tree;
        P.rinl = X.rinl;
        walker = idx - start;
        walker_ends(P, walker);
        item = base + idx;
        pending = true;
      }
      next = (next + n_idle) < total ? next + n_idle : total;
    }
    // (2) one step of every running walker
    NoSink none;
    if (active && !walk_step<kHubs>(P, walker, S, none)) {
      finish_walk(S);
      a.wres[item] = WalkOut{S.x, static_cast<uint16_t>(S.steps), static_cast<uint8_t>(S.hit), 0,
                             S.bytes, 0u, S.R};
      active = false;
    }
    // (3) lanes that received a walker start it
    if (pending) {
      walker_start(S, P.p);
      active = true;
      pending = false;
    }
    if (__ballot(active) == 0ull && next >= total) break;
  }
}

// Batched form, head/tail schedule.  Walks are short and heavy-tailed: most
// walkers of an update stop within a few steps while a few run to L, and a
// wavefront's instructions cost the same however few lanes still walk.  The
// head walk runs each update's walkers in lockstep (one wavefront per update,
// as the plain form) until at most tail_lanes of them (and at most a quarter
// of the round) still walk, records the finished walkers' outcomes and
// hands the rest to the tail walk, which packs the survivors of several
// updates into each wavefront.  Same results as the plain form.
template <bool kHubs>
__global__ __launch_bounds__(kWalkBlock) void k_walk_head(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  const DevGraph G = a.g[0];
  const DevGraph H = a.g[1];
  if (batch_failed(a.ctl)) return;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t upd = blockIdx.x * (kWalkBlock / kWave) + wave_in_block();
  if (upd >= a.n_ins + a.n_del) return;  // uniform across the wavefront
  const UpdateView v = view_update(a, G, H, upd);
  const unsigned long long first = a.ctl->item_base + a.qofs[upd];
  const unsigned long long lanes_below = (1ull << lane) - 1ull;
  uint32_t tails = 0;
  if (v.walks) {
    for (uint32_t base = 0; base < v.s; base += kWave) {
      const uint32_t walker = base + lane;
      const bool active = walker < v.s;
      const uint32_t n_round = (v.s - base) < kWave ? (v.s - base) : kWave;
      const uint32_t handoff = a.tail_lanes < n_round / 4 ? a.tail_lanes : n_round / 4;
      WState S;
      const bool more = walk_lockstep<kHubs, false>(v.P, walker, active, nullptr, lane, handoff, S);
      const unsigned long long moving = __ballot(more);
      if (more) {
        const uint32_t r = tails + static_cast<uint32_t>(__popcll(moving & lanes_below));
        a.tstate[first + r] =
            TailState{S.x, S.prev, S.steps, S.bytes, S.qprev, walker, S.R, S.rpend};
      } else if (active) {
        a.wres[first + walker] = WalkOut{S.x, static_cast<uint16_t>(S.steps),
                                         static_cast<uint8_t>(S.hit), 0, S.bytes, 0u, S.R};
      }
      tails += static_cast<uint32_t>(__popcll(moving));
    }
  }
  if (lane == 0) a.tcount[upd] = tails;
}

// Tail walk: wavefront w walks the survivors of updates [w*upw, w*upw + upw)
// (tcount of each, states in tstate), a lane whose walker stops taking the
// next one; each outcome goes to its walker's slot in wres.
template <bool kHubs>
__global__ __launch_bounds__(kBlock) void k_walk_tail(const BatchArgs* const* __restrict__ argv,
                                                      uint32_t upw) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  if (batch_failed(a.ctl)) return;
  const uint32_t nu = a.n_ins + a.n_del;
  const uint32_t u0 = (blockIdx.x * (kBlock / kWave) + wave_in_block()) * upw;
  if (u0 >= nu) return;  // uniform across the wavefront
  const uint32_t nr = (nu - u0) < upw ? (nu - u0) : upw;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const unsigned long long lanes_below = (1ull << lane) - 1ull;
  uint32_t endw[kMaxUpw];  // end (exclusive) of each update's survivors within the range
  uint32_t total = 0;
#pragma unroll
  for (uint32_t j = 0; j < kMaxUpw; ++j) {
    if (j < nr) total += a.tcount[u0 + j];
    endw[j] = total;
  }
  if (total == 0) return;
  const unsigned long long item0 = a.ctl->item_base;
  WalkParams P;
  P.K = a.K;
  P.key0 = static_cast<uint32_t>(a.seed);
  P.key1 = static_cast<uint32_t>(a.seed >> 32);
  P.bounce = a.bounce != 0;
  P.both = (a.variant & kVarBothEnds) != 0;
  P.heavy = a.ctl->heavy != 0u;
  P.rows = a.g[1].rows;
  P.ent = a.g[1].ent;
  P.prinv = a.g[1].prinv;
  P.tree = a.g[1].tree;
  P.rinl = a.g[1].rinl;
  P.p = P.q = 0;
  P.use_K = false;
  P.w_pq = 0.0;
  P.L = 0;
  P.uid_lo = P.uid_hi = 0;
  WState S;
  walker_start(S, 0);
  uint32_t next = 0;  // survivors of the range handed out so far (uniform)
  uint32_t walker = 0;
  unsigned long long out = 0;
  bool active = false;
  while (true) {
    // hand the next survivors of the range to idle lanes
    const unsigned long long idle = __ballot(!active);
    const uint32_t n_idle = static_cast<uint32_t>(__popcll(idle));
    if (next < total && n_idle) {
      const uint32_t rank = static_cast<uint32_t>(__popcll(idle & lanes_below));
      if (!active && next + rank < total) {
        const uint32_t idx = next + rank;
        uint32_t j = 0, start = 0;
#pragma unroll
        for (uint32_t k = 0; k < kMaxUpw; ++k)
          if (endw[k] <= idx) {
            j = k + 1;
            start = endw[k];
          }
        const uint32_t upd = u0 + j;
        const bool is_ins = upd < a.n_ins;
        const uint32_t jd = upd - a.n_ins;
        const uint64_t uid = a.uid_base + upd;
        const TailState ts = a.tstate[item0 + a.qofs[upd] + (idx - start)];
        P.p = is_ins ? a.iu[upd] : a.du[jd];  // the survivor's state holds where it is
        P.q = is_ins ? a.iv[upd] : a.dv[jd];
        walker_ends(P, ts.walker);
        P.w_pq = is_ins ? a.iw[upd] : 0.0;
        P.use_K = is_ins && a.has_K;
        P.L = a.L ? a.L[upd] : a.L_def;
        P.uid_lo = static_cast<uint32_t>(uid);
        P.uid_hi = static_cast<uint32_t>(uid >> 32);
        const DevGraph& X = is_ins ? a.g[1] : a.g[0];  // H_mid for insertions, G_mid for deletions
        P.rows = X.rows;
        P.ent = X.ent;
        P.prinv = X.prinv;
        P.tree = X.tree;
        P.rinl = X.rinl;
        const unsigned long long first = item0 + a.qofs[upd];
        S.x = ts.x;
        S.prev = ts.prev;
        S.steps = ts.t;
        S.bytes = ts.bytes;
        S.qprev = ts.qprev;
        S.R = ts.R;
        S.rpend = ts.rpend;
        S.block_of = kNone;  // the next step draws its block afresh
        S.hit = false;
        walker = ts.walker;
        out = first + ts.walker;
        active = true;
      }
      next = (next + n_idle) < total ? next + n_idle : total;
    }
    NoSink none;
    if (active && !walk_step<kHubs>(P, walker, S, none)) {
      finish_walk(S);
      a.wres[out] = WalkOut{S.x, static_cast<uint16_t>(S.steps), static_cast<uint8_t>(S.hit), 0,
                            S.bytes, 0u, S.R};
      active = false;
    }
    if (__ballot(active) == 0ull && next >= total) break;
  }
}

// Reduce each update's walker records and decide it (one wavefront per update).
template <bool kHubs>
__global__ __launch_bounds__(kWalkBlock) void k_reduce_updates(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  const DevGraph G = a.g[0];
  const DevGraph H = a.g[1];
  if (batch_failed(a.ctl)) return;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t upd = blockIdx.x * (kWalkBlock / kWave) + wave_in_block();
  if (upd >= a.n_ins + a.n_del) return;
  const UpdateView v = view_update(a, G, H, upd);
  if (!v.walks) {
    no_walk_update(a, v, upd, lane);
    return;
  }
  const unsigned long long first = a.ctl->item_base + a.qofs[upd];
  bool any_hit = false;
  double bestR = INFINITY;
  uint32_t bestW = kNone;
  uint32_t steps = 0, bytes = 0;
  for (uint32_t base = 0; base < v.s; base += kWave) {
    const uint32_t walker = base + lane;
    const bool active = walker < v.s;
    // lanes past the last walker read walker `base` (in range); every use of
    // the record below is guarded by `active`
    const WalkOut o = a.wres[first + (active ? walker : base)];
    if (active && a.wrec)
      a.wrec[a.wofs[upd] + walker] = WalkerRec{o.hit, 0, o.steps, o.end, o.R};
    const bool h = active && o.hit;
    any_hit = any_hit || (__ballot(h) != 0ull);
    double cR = h ? o.R : INFINITY;
    uint32_t cW = h ? walker : kNone;
    wave_argmin(cR, cW);
    if (cW != kNone && (bestW == kNone || cR < bestR)) {
      bestR = cR;
      bestW = cW;
    }
    steps += wave_sum(active ? static_cast<uint32_t>(o.steps) : 0u);
    bytes += wave_sum(active ? o.bytes : 0u);
  }
  if (lane == 0) a.ubytes[upd] = bytes;
  decide_update<kHubs>(a, G, H, upd, v, any_hit, bestR, bestW, steps, lane);
}

// No-hit fallbacks of deletions at long G rows (listed by decide_update):
// one workgroup per deletion.  Per endpoint, its H row (up to kFallbackLds
// entries) is staged in LDS, the G row is read coalesced, each live G entry
// looked up in the staged H row by binary search, then the workgroup's
// minimum of (1/w, neighbour) over the entries not live in H; a longer H row
// takes the merged slices of fallback_slice instead.  Writes the deletion's
// fallback slots and n_rec (the rest of its result is final).
__global__ __launch_bounds__(kFbBlock) void k_fallback_wide(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  if (batch_failed(a.ctl)) return;
  const uint32_t count = a.ctl->fb_count;
  const DevGraph G = a.g[0];
  const DevGraph H = a.g[1];
  __shared__ double s_r[kFbBlock / kWave];
  __shared__ uint32_t s_n[kFbBlock / kWave];
  __shared__ uint32_t s_count;
  __shared__ uint32_t s_hn[kFallbackLds];         // the endpoint's H row: neighbours
  __shared__ uint32_t s_hlive[kFallbackLds / 32];  // and which of them are live
  const uint32_t t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
  for (uint32_t f = blockIdx.x; f < count; f += gridDim.x) {
    const uint32_t upd = a.fb_list[f];
    const uint32_t j = upd - a.n_ins;
    const uint32_t p = a.du[j], q = a.dv[j];
    AddRec* out = del_slots(a, upd);
    if (t == 0) s_count = 0;
    __syncthreads();
    for (int z = 0; z < 2; ++z) {
      const uint32_t end = z == 0 ? p : q;
      double br = INFINITY;
      uint32_t bn = kNone, bi = 0;
      const RowHdr hr = row_hdr(H, end);
      if (hr.len <= kFallbackLds) {
        // H row in LDS; G row read coalesced, membership by binary search
        const Seg hseg = seg_of(H, end, hr.off);
        for (uint32_t i = t; i < (hr.len + 31) / 32; i += kFbBlock) s_hlive[i] = 0u;
        __syncthreads();
        for (uint32_t i = t; i < hr.len; i += kFbBlock) {
          s_hn[i] = hseg.nbr(i);
          if (hseg.qw(i) != 0u) atomicOr(&s_hlive[i >> 5], 1u << (i & 31));
        }
        __syncthreads();
        const RowHdr gr = row_hdr(G, end);
        const Seg seg = seg_of(G, end, gr.off);
        for (uint32_t i0 = 0; i0 < gr.len; i0 += kFbBlock * kFallbackUnroll) {
          uint32_t en[kFallbackUnroll], eq[kFallbackUnroll];
          double er[kFallbackUnroll];
#pragma unroll
          for (uint32_t m = 0; m < kFallbackUnroll; ++m) {  // loads issued together
            const uint32_t i = i0 + m * kFbBlock + t;
            const uint32_t ii = i < gr.len ? i : gr.len - 1;
            en[m] = seg.nbr(ii);
            eq[m] = seg.qw(ii);
            er[m] = seg.r(ii);
          }
          // H entries below each neighbour: fixed-length searches, so that
          // the kFallbackUnroll lookups are independent and overlap
          uint32_t lo[kFallbackUnroll];
#pragma unroll
          for (uint32_t m = 0; m < kFallbackUnroll; ++m) lo[m] = 0;
#pragma unroll
          for (uint32_t w = kFallbackSearch; w >= 1; w >>= 1) {
#pragma unroll
            for (uint32_t m = 0; m < kFallbackUnroll; ++m)
              if (lo[m] + w <= hr.len && s_hn[lo[m] + w - 1] < en[m]) lo[m] += w;
          }
#pragma unroll
          for (uint32_t m = 0; m < kFallbackUnroll; ++m) {
            const uint32_t i = i0 + m * kFbBlock + t;
            if (i >= gr.len || eq[m] == 0u) continue;
            const uint32_t at = lo[m];
            if (at < hr.len && s_hn[at] == en[m] && ((s_hlive[at >> 5] >> (at & 31)) & 1u))
              continue;  // live in H
            if (er[m] < br || (er[m] == br && en[m] < bn)) {
              br = er[m];
              bn = en[m];
              bi = i;
            }
          }
        }
      } else {
        fallback_slice(G, H, end, t, kFbBlock, br, bn, bi);
      }
      double wr = br;
      uint32_t wn = bn;
      wave_argmin(wr, wn);
      if (lane == 0) {
        s_r[wv] = wr;
        s_n[wv] = wn;
      }
      __syncthreads();
      for (uint32_t k = 0; k < kFbBlock / kWave; ++k)  // same order on every thread
        if (s_r[k] < wr || (s_r[k] == wr && s_n[k] < wn)) {
          wr = s_r[k];
          wn = s_n[k];
        }
      const uint32_t c = s_count;
      if (wn != kNone && bn == wn) {  // neighbour ids are unique: one owner
        const RowHdr r = row_hdr(G, end);
        const Seg seg = seg_of(G, end, r.off);
        out[c] = AddRec{end, wn, seg.qw(bi), 0u, seg.r(bi), seg.w[bi]};
      }
      __syncthreads();
      if (t == 0 && wn != kNone) s_count = c + 1;
      __syncthreads();
    }
    const uint32_t n = s_count;
    for (uint32_t zz = n + t; zz < a.Lcap; zz += kFbBlock) out[zz] = kNoAdd;
    if (t == 0) a.res[upd].n_rec = static_cast<uint16_t>(n);
    __syncthreads();
  }
}

// Batch totals of walker steps and algorithmic bytes (from the per-update
// counts), added to the context's running totals: one atomic per block.
__global__ __launch_bounds__(kBlock) void k_sum_counters(const BatchArgs* const* __restrict__ argv) {
  const BatchArgs a = load_args(argv, blockIdx.y);
  if (batch_failed(a.ctl)) return;
  const uint32_t nu = a.n_ins + a.n_del;
  unsigned long long st = 0, by = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nu; i += gridDim.x * blockDim.x) {
    st += a.res[i].steps;
    by += a.ubytes[i];
  }
  __shared__ unsigned long long part[2][kBlock / kWave];
  st = wave_sum64(st);
  by = wave_sum64(by);
  const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  if (lane == 0) {
    part[0][wv] = st;
    part[1][wv] = by;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st = by = 0;
    for (uint32_t w = 0; w < kBlock / kWave; ++w) {
      st += part[0][w];
      by += part[1][w];
    }
    if (st) atomicAdd(&a.ctl->steps_total, st);
    if (by) atomicAdd(&a.ctl->alg_bytes_total, by);
  }
}

// ---- phase 4 ------------------------------------------------------------------------
//
// One launch per step serves both graphs: blockIdx.z picks the graph (which =
// which0 + blockIdx.z), and its per-graph state is read from the argument
// record in global memory.

struct P4 {
  DevGraph X;
  BatchCtl* ctl;
  uint32_t *touched_rows, *touched_k, *touched_need, *dirty_rows, *dirty_chunk0, *dirty_small,
      *wide_rows;
  WideMerge* wmerge;
  uint8_t* add_keep;
  uint32_t n, n_ins, hadd_cap, hash_mask;
  const uint32_t *iu, *iv, *ins_qw;
  const double *iw, *ins_rinv;
  const AddRec* hadd;
  HashSlot* hash;  // the phase-4 dedup table
};

__device__ __forceinline__ P4 load_p4(const BatchArgs* const* __restrict__ argv, uint32_t b,
                                      uint32_t which) {
  const gptr<const BatchArgs> ap = args_of(argv, b);
  P4 v;
  load_graph(v.X, ap, static_cast<int>(which));
  v.X.pool_cap = ap->g[which].pool_cap;
  v.ctl = load_gptr(&ap->ctl);
  v.touched_rows = load_gptr(&ap->touched_rows[which]);
  v.touched_k = load_gptr(&ap->touched_k[which]);
  v.touched_need = load_gptr(&ap->touched_need[which]);
  v.dirty_rows = load_gptr(&ap->dirty_rows[which]);
  v.dirty_chunk0 = load_gptr(&ap->dirty_chunk0[which]);
  v.dirty_small = load_gptr(&ap->dirty_small[which]);
  v.wide_rows = load_gptr(&ap->wide_rows[which]);
  v.wmerge = load_gptr(&ap->wmerge[which]);
  v.add_keep = load_gptr(&ap->add_keep[which]);
  v.n = ap->n;
  v.n_ins = ap->n_ins;
  v.hadd_cap = ap->hadd_cap;
  v.hash_mask = ap->hash_mask;
  v.iu = load_gptr(&ap->iu);
  v.iv = load_gptr(&ap->iv);
  v.ins_qw = load_gptr(&ap->ins_qw);
  v.iw = load_gptr(&ap->iw);
  v.ins_rinv = load_gptr(&ap->ins_rinv);
  v.hadd = load_gptr(&ap->hadd);
  v.hash = load_gptr(&ap->hash2);
  return v;
}

// List row r (final length len > kHub) for a weight-tree rebuild, once per
// phase 4: one atomic claims its list slot and its chunks of kTreeChunk
// entries, so first chunks grow with the slot.  The row's mark counts its
// finished chunks in k_hub_tree.
__device__ __forceinline__ void mark_dirty4(const P4& a, uint32_t which, uint32_t r,
                                            uint32_t len) {
  if (atomicExch(&a.X.mark[r], 1u) == 0u) {
    if (len <= kTreeSmall) {
      a.dirty_small[atomicAdd(&a.ctl->tsmall[which], 1ull)] = r;
      return;
    }
    const uint32_t chunks = (len + kTreeChunk - 1) / kTreeChunk;
    const unsigned long long claim =
        atomicAdd(&a.ctl->tpack[which], (static_cast<unsigned long long>(chunks) << 32) | 1ull);
    a.dirty_rows[static_cast<uint32_t>(claim)] = r;
    a.dirty_chunk0[static_cast<uint32_t>(claim)] = static_cast<uint32_t>(claim >> 32);
  }
}

// A claim on a shared 64-bit counter by a whole wavefront with one atomic:
// every lane calls it with its amount (0 for none) and gets the counter's
// value plus the amounts of the lanes below it.
__device__ unsigned long long wave_claim(unsigned long long* ctr, unsigned long long v) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  unsigned long long incl = v;
  for (uint32_t d = 1; d < kWave; d <<= 1) {
    const unsigned long long o = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += o;
  }
  const unsigned long long total = __shfl(incl, kWave - 1, kWave);
  unsigned long long base = 0;
  if (lane == kWave - 1 && total != 0) base = atomicAdd(ctr, total);
  base = __shfl(base, kWave - 1, kWave);
  return base + incl - v;
}

// mark_dirty4 for the rows of a whole wavefront (every lane calls it; `want`
// says whether its row r, of final length len, is listed), with one claim
// per wavefront; also raises the hub flag.
__device__ void mark_dirty_wave(const P4& a, uint32_t which, bool want, uint32_t r,
                                uint32_t len) {
  const bool fresh = want && atomicExch(&a.X.mark[r], 1u) == 0u;
  const bool small = len <= kTreeSmall;
  const unsigned long long chunks = (len + kTreeChunk - 1) / kTreeChunk;
  const unsigned long long slot =
      wave_claim(&a.ctl->tpack[which], fresh && !small ? (chunks << 32) | 1ull : 0ull);
  const unsigned long long sslot = wave_claim(&a.ctl->tsmall[which], fresh && small ? 1ull : 0ull);
  if (fresh && small) {
    a.dirty_small[static_cast<uint32_t>(sslot)] = r;
  } else if (fresh) {
    a.dirty_rows[static_cast<uint32_t>(slot)] = r;
    a.dirty_chunk0[static_cast<uint32_t>(slot)] = static_cast<uint32_t>(slot >> 32);
  }
  if (__ballot(want) != 0 && (threadIdx.x & (kWave - 1)) == 0) a.ctl->hubs = 1u;
}

struct AddEntry {
  uint32_t r, c, qw;
  double rinv, w;
  bool valid;
};

// Directed entry e of the additions to graph `which`: two per undirected edge.
__device__ __forceinline__ AddEntry add_entry(const P4& a, uint32_t which, uint32_t e) {
  const uint32_t i = e >> 1;
  const bool flip = e & 1u;
  if (which == 0) {
    const uint32_t u = a.iu[i], v = a.iv[i];
    return AddEntry{flip ? v : u, flip ? u : v, a.ins_qw[i], a.ins_rinv[i], a.iw[i], true};
  }
  const AddRec rec = a.hadd[i];
  if (rec.a >= a.n || rec.b >= a.n) return AddEntry{0, 0, 0, 0.0, 0.0, false};  // unused slot
  return AddEntry{flip ? rec.b : rec.a, flip ? rec.a : rec.b, rec.qw, rec.rinv, rec.w, true};
}

__device__ __forceinline__ uint32_t add_count(const P4& a, uint32_t which) {
  return which == 0 ? 2u * a.n_ins : 2u * a.hadd_cap;
}

// H additions are taken from the slots [h_lo, h_hi) only (two-stage
// batches add the deletions' recoveries and the kept insertions apart).
__device__ __forceinline__ bool in_window(uint32_t which, uint32_t e, uint32_t h_lo,
                                          uint32_t h_hi) {
  return which == 0 || ((e >> 1) >= h_lo && (e >> 1) < h_hi);
}

__global__ void k_add_prepare(const BatchArgs* const* __restrict__ argv, uint32_t which0,
                              uint32_t h_lo, uint32_t h_hi) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (batch_failed(a.ctl)) return;
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= add_count(a, which)) return;
  a.add_keep[e] = 0;
  if (!in_window(which, e, h_lo, h_hi)) return;
  const AddEntry d = add_entry(a, which, e);
  if (!d.valid) return;
  const RowHdr row = row_hdr(X, d.r);
  const Seg seg = seg_of(X, d.r, row.off);
  const int k = find_nbr(seg, row.len, d.c);
  if (k >= 0) {
    // a tombstone of the same edge: revive it in place (once)
    const uint32_t old = atomicCAS(&seg.qw(k), 0u, d.qw);
    if (old == 0u) {
      seg.r(k) = d.rinv;
      seg.w[k] = d.w;
      atomicSub(&row_hdr_ref(X, d.r).dead, 1u);
      if (row.len > kHub) tree_add(X, d.r, row.off, row.len, static_cast<uint32_t>(k), d.qw);
    }
    return;
  }
  if (which == 1 &&
      !hash_insert_first(a.hash, a.hash_mask,
                         (static_cast<unsigned long long>(d.r) << 32) | d.c))
    return;  // the same edge recovered by another deletion
  const uint32_t slot = atomicAdd(&X.pending[d.r], 1u);
  if (slot == 0u) {
    const uint32_t t = atomicAdd(&a.ctl->touched[which], 1u);
    a.touched_rows[t] = d.r;
  }
  a.add_keep[e] = 1;
}

__device__ __forceinline__ uint32_t grown_cap(uint32_t live) {
  const uint32_t extra = live / 2 > 2u ? live / 2 : 2u;
  return live + extra;
}

// touched_k packs the number of appended entries with three decisions taken
// here, once, from the segment as it stands before phase 4 moves anything:
// whether the segment is relocated by a workgroup, merged by a workgroup, and
// relocated to a start aligned for a weight tree.
constexpr uint32_t kAlignHub = 1u << 29;
constexpr uint32_t kWideRelocate = 1u << 30;
constexpr uint32_t kWideMerge = 1u << 31;
constexpr uint32_t kCountMask = kAlignHub - 1u;

// A segment of more than kHub entries must start at a multiple of kHubAlign
// and own a multiple of kFan slots (its weight tree's layout).
__device__ __forceinline__ bool tree_ready(const RowHdr& row) {
  return row.off != kInlineOff && row.off % kHubAlign == 0 && row.cap % kFan == 0;
}

// First slot of a relocated segment whose reservation starts at `raw` (an
// aligned segment reserves kHubAlign slots more than its capacity).
__device__ __forceinline__ uint32_t relocated_off(unsigned long long raw, bool align) {
  return static_cast<uint32_t>(align ? (raw + kHubAlign - 1) / kHubAlign * kHubAlign : raw);
}

__global__ void k_rows_plan(const BatchArgs* const* __restrict__ argv, uint32_t which0) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (batch_failed(a.ctl)) return;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.ctl->touched[which]) return;
  const uint32_t r = a.touched_rows[t];
  const uint32_t k = X.pending[r];
  const RowHdr row = row_hdr(X, r);
  uint32_t need = 0, flags = 0, merged_from = row.len;
  // relocated when the slack cannot take the k new entries, or when the
  // merged segment becomes long and its place does not suit a weight tree
  if (row.len + k > row.cap || (row.len + k > kHub && !tree_ready(row))) {
    const uint32_t live = row.len - row.dead + k;  // relocation drops the tombstones
    const bool align = live > kHub;
    // even capacities keep every segment start even (two pairs per load)
    need = align ? round_fan(grown_cap(live)) : (grown_cap(live) + 1u) & ~1u;
    // an aligned start may skip up to kHubAlign - 2 slots (reserved: kHubAlign)
    const uint32_t reserve = align ? need + kHubAlign : need;
    atomicAdd(&a.ctl->need[which], static_cast<unsigned long long>(reserve));
    if (row.len > kHub) flags |= kWideRelocate;
    if (align) flags |= kAlignHub;
    merged_from = row.len - row.dead;
  }
  if (merged_from + k > kHub) {
    flags |= kWideMerge;
    // the merge stages its new and old entries past the pool top (not kept)
    atomicAdd(&a.ctl->need[which], static_cast<unsigned long long>(merged_from) + k);
  }
  a.touched_k[t] = k | flags;
  a.touched_need[t] = need;
  if (flags) a.wide_rows[atomicAdd(&a.ctl->wide[which], 1u)] = t;  // rare: long rows only
}

__global__ void k_pool_check(const BatchArgs* const* __restrict__ argv, uint32_t which0) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const uint64_t pool_cap = a.X.pool_cap;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (batch_failed(a.ctl)) return;
  if (a.ctl->pool_top[which] + a.ctl->need[which] > pool_cap) a.ctl->nomem[which] = 1;
}

__device__ __forceinline__ void rows_relocate_narrow(const BatchArgs* const* __restrict__ argv,
                                                     uint32_t which0, uint32_t bx) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (batch_failed(a.ctl) || a.ctl->nomem[which]) return;
  const uint32_t t = bx * blockDim.x + threadIdx.x;
  if (t >= a.ctl->touched[which]) return;
  const uint32_t need = a.touched_need[t];
  if (need == 0) return;
  if (a.touched_k[t] & kWideRelocate) return;  // moved by rows_relocate_wide
  const uint32_t r = a.touched_rows[t];
  const RowHdr row = row_hdr(X, r);
  const Seg src = seg_of(X, r, row.off);
  const bool align = (a.touched_k[t] & kAlignHub) != 0;
  const uint32_t off = relocated_off(
      atomicAdd(&a.ctl->pool_top[which],
                static_cast<unsigned long long>(align ? need + kHubAlign : need)),
      align);
  uint32_t o = 0;
  for (uint32_t i = 0; i < row.len; ++i) {
    const Ent e = src.get(i);
    if (e.qw == 0u) continue;  // drop tombstones while moving
    X.ent[off + o] = Pair{e.nbr, e.qw};
    X.prinv[off + o] = e.rinv;
    X.w[off + o] = src.w[i];
    ++o;
  }
  row_hdr_ref(X, r) = RowHdr{off, o, need, 0u};
}

// Relocation of long segments: one workgroup per segment, tombstones dropped
// through a block-wide scan of the live flags.
__device__ __forceinline__ void rows_relocate_wide(const BatchArgs* const* __restrict__ argv,
                                                   uint32_t which0, uint32_t bx, uint32_t nbx) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (batch_failed(a.ctl) || a.ctl->nomem[which]) return;
  __shared__ uint32_t s_off;
  const uint32_t count = a.ctl->wide[which];
  for (uint32_t wi = bx; wi < count; wi += nbx) {
    const uint32_t t = a.wide_rows[wi];
    const uint32_t need = a.touched_need[t];
    if (need == 0 || !(a.touched_k[t] & kWideRelocate)) continue;  // block-uniform
    const uint32_t r = a.touched_rows[t];
    const RowHdr row = row_hdr(X, r);  // len > kHub: a pool segment
    const bool align = (a.touched_k[t] & kAlignHub) != 0;
    if (threadIdx.x == 0)
      s_off = relocated_off(
          atomicAdd(&a.ctl->pool_top[which],
                    static_cast<unsigned long long>(align ? need + kHubAlign : need)),
          align);
    __syncthreads();
    const uint32_t off = s_off;
    unsigned long long out = 0;
    for (uint32_t base = 0; base < row.len; base += kBlock) {
      const uint32_t i = base + threadIdx.x;
      Pair e{0, 0};
      double er = 0.0, we = 0.0;
      if (i < row.len) {
        e = X.ent[row.off + i];
        er = X.prinv[row.off + i];
        we = X.w[row.off + i];
      }
      const unsigned long long live = (i < row.len && e.qw != 0u) ? 1u : 0u;
      unsigned long long excl;
      const unsigned long long total = block_excl_scan(live, excl);
      if (live) {
        X.ent[off + out + excl] = e;
        X.prinv[off + out + excl] = er;
        X.w[off + out + excl] = we;
      }
      out += total;
    }
    if (threadIdx.x == 0) row_hdr_ref(X, r) = RowHdr{off, static_cast<uint32_t>(out), need, 0u};
    __syncthreads();
  }
}

// Relocations of the touched rows that need more room: the first
// narrow_blocks workgroups move short rows (a thread per row), the others
// long ones (a workgroup per row); the two sets of rows are disjoint.
__global__ __launch_bounds__(kBlock) void k_rows_relocate(const BatchArgs* const* __restrict__ argv,
                                                          uint32_t which0, uint32_t narrow_blocks) {
  if (blockIdx.x < narrow_blocks) rows_relocate_narrow(argv, which0, blockIdx.x);
  else rows_relocate_wide(argv, which0, blockIdx.x - narrow_blocks, gridDim.x - narrow_blocks);
}

__global__ void k_add_place(const BatchArgs* const* __restrict__ argv, uint32_t which0,
                            uint32_t h_lo, uint32_t h_hi) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (batch_failed(a.ctl) || a.ctl->nomem[which]) return;
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= add_count(a, which)) return;
  if (!in_window(which, e, h_lo, h_hi) || !a.add_keep[e]) return;
  const AddEntry d = add_entry(a, which, e);
  const RowHdr row = row_hdr(X, d.r);
  const uint32_t slot = atomicSub(&X.pending[d.r], 1u) - 1u;  // leaves pending at 0
  const uint32_t pos = row.len + slot;
  seg_of(X, d.r, row.off).put(pos, Ent{d.c, d.qw, d.rinv}, d.w);
}

// Merge the k appended entries (unsorted tail) into the sorted segment; one
// thread per short segment (insertion of each new entry).
__device__ __forceinline__ void rows_merge_narrow(const BatchArgs* const* __restrict__ argv,
                                                  uint32_t which0, uint32_t bx) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (batch_failed(a.ctl) || a.ctl->nomem[which]) return;
  const uint32_t t = bx * blockDim.x + threadIdx.x;
  uint32_t packed = kWideMerge;  // rows merged by rows_merge_wide are skipped
  if (t < a.ctl->touched[which]) packed = a.touched_k[t];
  const bool mine = !(packed & kWideMerge);
  uint32_t r = 0, len = 0;
  if (mine) {
    r = a.touched_rows[t];
    const uint32_t k = packed & kCountMask;
    const RowHdr row = row_hdr(X, r);
    const Seg seg = seg_of(X, r, row.off);
    for (uint32_t j = row.len; j < row.len + k; ++j) {
      const Ent e = seg.get(j);
      const double we = seg.w[j];
      uint32_t i = j;
      while (i > 0 && seg.nbr(i - 1) > e.nbr) {
        seg.put(i, seg.get(i - 1), seg.w[i - 1]);
        --i;
      }
      seg.put(i, e, we);
    }
    len = row.len + k;
    row_hdr_ref(X, r).len = len;
  }
  mark_dirty_wave(a, which, mine && len > kHub, r, len);  // weight tree rebuilt next
}

constexpr uint32_t kTailChunk = 1024;  // appended entries merged per pass (12 KB LDS)

// Merges for long segments (the appended entries of a touched row into its
// sorted prefix), in three forms by the number k of appended entries.
// * k <= kWaveKeys (nearly every row): a wavefront sorts the keys across its
//   lanes and stages the new entries; k_wide_copy_out and k_wide_place then
//   move the row in units of kMergeChunk old entries, the units of all rows
//   spread over the grid.
// * k <= kTailChunk: the same, with the sort and staging by a workgroup.
// * larger k (one workgroup per row, in place): each pass takes up to
//   kTailChunk appended entries, copies them past the pool top, sorts their
//   keys in LDS (bitonic), computes every entry's final position (old entries
//   shift right by the number of new entries below them; new entries sit
//   after the old entries below them), moves the old entries right to left
//   in block-sized chunks, so no entry is overwritten before it is read, and
//   finally writes the new entries from their staging copy.
// Staging slots lie past the pool top, reserved by the phase-4 pool check and
// given back at the end of the batch.
constexpr uint32_t kMergePer = 8;  // old entries per thread and chunk of a wide merge

// Bitonic sort of P (a power of two) keys in LDS by the whole block.
__device__ __forceinline__ void block_sort_keys(unsigned long long* key, uint32_t P) {
  for (uint32_t size = 2; size <= P; size <<= 1)
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < P; i += kBlock) {
        const uint32_t l = i ^ stride;
        if (l > i) {
          const bool up = (i & size) == 0;
          const unsigned long long x = key[i], y = key[l];
          if ((x > y) == up) {
            key[i] = y;
            key[l] = x;
          }
        }
      }
      __syncthreads();
    }
}

// Whether a touched row's merge is spread over many workgroups: a wide merge
// of at most kTailChunk appended entries (a longer tail takes the in-place
// passes below).
__device__ __forceinline__ bool parallel_merge(uint32_t packed) {
  return (packed & kWideMerge) && (packed & kCountMask) <= kTailChunk;
}

// Parallel wide merges of at most kWaveKeys appended entries are prepared by
// one wavefront (keys sorted across its lanes), the others by a workgroup.
constexpr uint32_t kWaveKeys = kWave;
__device__ __forceinline__ bool wave_merge(uint32_t packed) {
  return (packed & kWideMerge) && (packed & kCountMask) <= kWaveKeys;
}

// First stage of the parallel wide merges of at most kWaveKeys appended
// entries (cur .. cur+k-1 of their rows), up to kWave of them by one
// wavefront, lane j holding merge j: its least new key, the first old entry
// that moves (stay, a binary search per lane), the row's final length and
// its listing for the weight-tree rebuild, then the staging slots and the
// merge's slot and chunks claimed with one atomic each for the wavefront
// (chunk numbers grow with the slot).  Then the new entries of each merge
// are sorted by neighbour (bitonic across a segment of lanes, several merges
// side by side) and staged past the pool top, in slots the pool check
// reserved.
__device__ void wave_prepare_group(const P4& a, uint32_t which, bool mine, uint32_t t,
                                   unsigned long long top) {
  const DevGraph& X = a.X;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t r = 0, k = 0, off = 0, cur = 0, stay = 0;
  if (mine) {
    r = a.touched_rows[t];
    k = a.touched_k[t] & kCountMask;
    const RowHdr row = row_hdr(X, r);  // relocated or long: a pool segment
    off = row.off;
    cur = row.len;
    const Pair* seg = X.ent + off;
    uint32_t least = ~0u;
    for (uint32_t i = 0; i < k; ++i) least = min(least, seg[cur + i].nbr);
    uint32_t lo = 0, hi = cur;  // old entries below the least new one
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (seg[mid].nbr < least) lo = mid + 1;
      else hi = mid;
    }
    stay = lo;
    row_hdr_ref(X, r).len = cur + k;  // the moves below read no header
  }
  mark_dirty_wave(a, which, mine, r, cur + k);  // cur + k > kHub for every wide merge
  const uint32_t moving = cur - stay;
  const unsigned long long chunks = moving ? (moving + kMergeChunk - 1) / kMergeChunk : 1u;
  const uint32_t at = static_cast<uint32_t>(
      top + wave_claim(&a.ctl->stage_used[which], mine ? k + moving : 0u));
  const unsigned long long claim =
      wave_claim(&a.ctl->wpack[which], mine ? (chunks << 32) | 1ull : 0ull);
  if (mine)
    a.wmerge[static_cast<uint32_t>(claim)] =
        WideMerge{r, k, stay, cur, off, at, static_cast<uint32_t>(claim >> 32),
                  static_cast<uint32_t>(chunks)};
  // the merges of each size class S (S/2 < k <= S), kWave / S at a time:
  // merge q of a pass sorts and stages on lanes qS .. qS + S - 1
  __shared__ uint32_t s_rows[kBlock];  // a wavefront's members of one class
  uint32_t* rows_of = s_rows + (threadIdx.x / kWave) * kWave;
  for (uint32_t S = 1; S <= kWave; S <<= 1) {
    const bool in_class = mine && k <= S && 2 * k > S;
    const unsigned long long cls = __ballot(in_class);
    if (cls == 0) continue;  // wavefront-uniform
    const uint32_t n = static_cast<uint32_t>(__popcll(cls));
    if (in_class) rows_of[__popcll(cls & ((1ull << lane) - 1ull))] = lane;
    wave_lds_order();
    const uint32_t per = kWave / S, q = lane / S, sub = lane % S;
    for (uint32_t p0 = 0; p0 < n; p0 += per) {
      const bool has = p0 + q < n;
      const int j = has ? static_cast<int>(rows_of[p0 + q]) : 0;
      const uint32_t kj = __shfl(k, j, kWave), offj = __shfl(off, j, kWave);
      const uint32_t curj = __shfl(cur, j, kWave), atj = __shfl(at, j, kWave);
      const bool live = has && sub < kj;
      uint32_t key = live ? X.ent[static_cast<uint64_t>(offj) + curj + sub].nbr : ~0u;
      uint32_t idx = sub;  // ids are below ~0u
      for (uint32_t size = 2; size <= S; size <<= 1)
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
          const uint32_t ok = __shfl_xor(key, stride, kWave);
          const uint32_t oi = __shfl_xor(idx, stride, kWave);
          const bool up = size == S || (lane & size) == 0;
          const bool lower = (lane & stride) == 0;
          if (lower == up ? ok < key : ok > key) {
            key = ok;
            idx = oi;
          }
        }
      if (live) {
        const uint64_t src = static_cast<uint64_t>(offj) + curj + idx;
        const uint64_t dst = static_cast<uint64_t>(atj) + sub;
        X.ent[dst] = X.ent[src];
        X.prinv[dst] = X.prinv[src];
        X.w[dst] = X.w[src];
      }
    }
    wave_lds_order();  // the list is rewritten for the next class
  }
}

// Entries of the sorted segment seg[0, n) whose neighbour is below key, by the
// whole block: rounds of kBlock evenly spaced probes narrow the range kBlock
// times per round (three rounds for the longest rows).
__device__ uint32_t block_lower_bound(const Pair* seg, uint32_t n, uint32_t key) {
  uint32_t lo = 0, hi = n;  // the answer is in [lo, hi]
  while (hi > lo) {
    const uint32_t step = (hi - lo + kBlock - 1) / kBlock;
    const uint32_t at = lo + threadIdx.x * step;
    const int below = __syncthreads_count(at < hi && seg[at].nbr < key);
    if (below == 0) return lo;
    const uint32_t nlo = lo + (below - 1) * step + 1;
    const uint32_t nhi = lo + below * step;
    if (step == 1) return nlo;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
  return lo;
}

// First stage of a parallel wide merge of the k appended entries [cur, cur+k):
// sort them by neighbour, find the first old entry that has to move (stay:
// the old entries below the least new one), claim the merge's slot and its
// chunks with one atomic (so chunk numbers grow with the slot), and stage the
// sorted new entries past the pool top, in slots the pool check reserved.
// k_wide_copy_out and k_wide_place finish the merge; the row itself is not
// written here.  One workgroup.
__device__ void wide_prepare(const P4& a, uint32_t which, uint32_t r, uint32_t k,
                             uint32_t seg_off, uint32_t cur, unsigned long long top,
                             unsigned long long* s_key, unsigned long long& s_stage) {
  const DevGraph& X = a.X;
  const Pair* seg = X.ent + seg_off;
  uint32_t P = 1;
  while (P < k) P <<= 1;
  for (uint32_t j = threadIdx.x; j < P; j += kBlock)
    s_key[j] = j < k ? (static_cast<unsigned long long>(seg[cur + j].nbr) << 32) | j : ~0ull;
  __syncthreads();
  block_sort_keys(s_key, P);
  const uint32_t stay = block_lower_bound(seg, cur, static_cast<uint32_t>(s_key[0] >> 32));
  if (threadIdx.x == 0) {
    const uint32_t moving = cur - stay;
    const uint32_t chunks = moving ? (moving + kMergeChunk - 1) / kMergeChunk : 1u;
    const unsigned long long at = top + atomicAdd(&a.ctl->stage_used[which], k + moving);
    const unsigned long long claim =
        atomicAdd(&a.ctl->wpack[which], (static_cast<unsigned long long>(chunks) << 32) | 1ull);
    a.wmerge[static_cast<uint32_t>(claim)] =
        WideMerge{r, k, stay, cur, seg_off, static_cast<uint32_t>(at),
                  static_cast<uint32_t>(claim >> 32), chunks};
    s_stage = at;
    row_hdr_ref(X, r).len = cur + k;  // the moves read no header
    mark_dirty4(a, which, r, cur + k);
    a.ctl->hubs = 1u;
  }
  __syncthreads();
  const unsigned long long at = s_stage;
  for (uint32_t j = threadIdx.x; j < k; j += kBlock) {
    const uint32_t src = seg_off + cur + static_cast<uint32_t>(s_key[j] & 0xFFFFFFFFull);
    X.ent[at + j] = X.ent[src];
    X.prinv[at + j] = X.prinv[src];
    X.w[at + j] = X.w[src];
  }
  __syncthreads();
}

__device__ __forceinline__ void rows_merge_wide(const BatchArgs* const* __restrict__ argv,
                                                uint32_t which0, uint32_t bx, uint32_t nbx) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (batch_failed(a.ctl) || a.ctl->nomem[which]) return;
  __shared__ unsigned long long s_key[kTailChunk];  // (nbr << 32) | local index
  __shared__ uint32_t s_pos[kTailChunk];
  __shared__ unsigned long long s_stage;
  __shared__ uint32_t s_list[kBlock];
  __shared__ uint32_t s_n;
  const uint32_t count = a.ctl->wide[which];
  const unsigned long long top = a.ctl->pool_top[which];  // final: relocations are done
  // merges of few appended entries: kWave rows per wavefront at a time
  constexpr uint32_t kWaves = kBlock / kWave;
  for (uint32_t g0 = (bx * kWaves + threadIdx.x / kWave) * kWave; g0 < count;
       g0 += nbx * kWaves * kWave) {  // wavefront-uniform
    const uint32_t wi = g0 + (threadIdx.x & (kWave - 1));
    uint32_t t = 0, packed = 0;
    if (wi < count) {
      t = a.wide_rows[wi];
      packed = a.touched_k[t];
    }
    wave_prepare_group(a, which, wi < count && wave_merge(packed), t, top);
  }
  // the others: a workgroup each, listed kBlock rows at a time
  for (uint32_t base = bx * kBlock; base < count; base += nbx * kBlock) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    if (base + threadIdx.x < count) {
      const uint32_t packed = a.touched_k[a.wide_rows[base + threadIdx.x]];
      if ((packed & kWideMerge) && !wave_merge(packed)) s_list[atomicAdd(&s_n, 1u)] = base + threadIdx.x;
    }
    __syncthreads();
    const uint32_t listed = s_n;
    for (uint32_t q = 0; q < listed; ++q) {
      const uint32_t t = a.wide_rows[s_list[q]];
      const uint32_t packed = a.touched_k[t];
      const uint32_t r = a.touched_rows[t];
      const uint32_t k = packed & kCountMask;
      const RowHdr row = row_hdr(X, r);  // relocated or long: a pool segment
      Pair* seg = X.ent + row.off;
      double* rseg = X.prinv + row.off;
      double* wseg = X.w + row.off;
      uint32_t cur = row.len;  // sorted prefix length
      if (parallel_merge(packed)) {
        wide_prepare(a, which, r, k, row.off, cur, top, s_key, s_stage);
        continue;
      }
      if (threadIdx.x == 0) s_stage = top + atomicAdd(&a.ctl->stage_used[which], k);
      __syncthreads();
      const unsigned long long stage = s_stage;  // k staging slots
      for (uint32_t c0 = 0; c0 < k; c0 += kTailChunk) {
        const uint32_t c = (k - c0) < kTailChunk ? (k - c0) : kTailChunk;
        uint32_t P = 1;
        while (P < c) P <<= 1;
        for (uint32_t j = threadIdx.x; j < P; j += kBlock) {
          if (j < c) {
            const Pair e = seg[cur + j];
            X.ent[stage + c0 + j] = e;
            X.prinv[stage + c0 + j] = rseg[cur + j];
            X.w[stage + c0 + j] = wseg[cur + j];
            s_key[j] = (static_cast<unsigned long long>(e.nbr) << 32) | j;
          } else {
            s_key[j] = ~0ull;
          }
        }
        __syncthreads();
        for (uint32_t size = 2; size <= P; size <<= 1)
          for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += kBlock) {
              const uint32_t l = i ^ stride;
              if (l > i) {
                const bool up = (i & size) == 0;
                const unsigned long long x = s_key[i], y = s_key[l];
                if ((x > y) == up) {
                  s_key[i] = y;
                  s_key[l] = x;
                }
              }
            }
            __syncthreads();
          }
        // final slot of each new entry: its rank plus the old entries below it
        for (uint32_t j = threadIdx.x; j < c; j += kBlock) {
          const uint32_t key = static_cast<uint32_t>(s_key[j] >> 32);
          uint32_t lo = 0, hi = cur;
          while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (seg[mid].nbr < key) lo = mid + 1;
            else hi = mid;
          }
          s_pos[j] = j + lo;
        }
        __syncthreads();
        // Old entries move right by the number of new entries below them, in
        // chunks from the right end (every thread reads its kMergePer entries
        // before any writes); entries below the first new one stay put.
        const uint32_t stay = s_pos[0];  // new entry of least id lands here
        for (uint32_t hi_i = cur; hi_i > stay;) {
          const uint32_t span = kBlock * kMergePer;
          const uint32_t lo_i = hi_i - stay > span ? hi_i - span : stay;
          // fields in separate arrays (registers; an array of structs written
          // under a condition would go to scratch)
          uint32_t en[kMergePer], eq[kMergePer], shift[kMergePer];
          double er[kMergePer], we[kMergePer];
  #pragma unroll
          for (uint32_t m = 0; m < kMergePer; ++m) {
            const uint32_t i = lo_i + m * kBlock + threadIdx.x;
            const uint32_t ii = i < hi_i ? i : lo_i;  // in range either way
            const Pair x = seg[ii];
            en[m] = x.nbr;
            eq[m] = x.qw;
            er[m] = rseg[ii];
            we[m] = wseg[ii];
            shift[m] = 0;
          }
  #pragma unroll
          for (uint32_t m = 0; m < kMergePer; ++m) {
            const uint32_t i = lo_i + m * kBlock + threadIdx.x;
            // new entries below e.nbr: a fixed-length search over the P sorted
            // keys (padding keys are ~0), so that the arrays stay in registers
            uint32_t below = 0;
  #pragma unroll
            for (uint32_t w = kTailChunk; w >= 1; w >>= 1)  // counts up to P = kTailChunk
              if (below + w <= P && static_cast<uint32_t>(s_key[below + w - 1] >> 32) < en[m])
                below += w;
            if (i < hi_i) shift[m] = below;
          }
          __syncthreads();
  #pragma unroll
          for (uint32_t m = 0; m < kMergePer; ++m) {
            const uint32_t i = lo_i + m * kBlock + threadIdx.x;
            if (i < hi_i && shift[m]) {
              seg[i + shift[m]] = Pair{en[m], eq[m]};
              rseg[i + shift[m]] = er[m];
              wseg[i + shift[m]] = we[m];
            }
          }
          __syncthreads();
          hi_i = lo_i;
        }
        for (uint32_t j = threadIdx.x; j < c; j += kBlock) {
          const uint64_t src = stage + c0 + static_cast<uint32_t>(s_key[j] & 0xFFFFFFFFull);
          seg[s_pos[j]] = X.ent[src];
          rseg[s_pos[j]] = X.prinv[src];
          wseg[s_pos[j]] = X.w[src];
        }
        __syncthreads();
        cur += c;
      }
      if (threadIdx.x == 0) {
        row_hdr_ref(X, r).len = cur;
        if (cur > kHub) {
          mark_dirty4(a, which, r, cur);
          a.ctl->hubs = 1u;
        }
      }
      __syncthreads();
    }
    __syncthreads();  // s_n is reset after every read
  }
}

// Merges of the appended tails into sorted order: the first narrow_blocks
// workgroups take short rows (a thread per row), the others long ones (a
// workgroup per row); the two sets of rows are disjoint.
__global__ __launch_bounds__(kBlock) void k_rows_merge(const BatchArgs* const* __restrict__ argv,
                                                       uint32_t which0, uint32_t narrow_blocks) {
  if (blockIdx.x < narrow_blocks) rows_merge_narrow(argv, which0, blockIdx.x);
  else rows_merge_wide(argv, which0, blockIdx.x - narrow_blocks, gridDim.x - narrow_blocks);
}

// The parallel wide merge that chunk c belongs to, by one wavefront: the
// last merge whose first chunk is at or below c (first chunks grow with the
// merge's slot, and merge 0 starts at chunk 0).
__device__ uint32_t wave_merge_of_chunk(const WideMerge* wm, uint32_t merges, uint32_t c,
                                        uint32_t lane) {
  uint32_t lo = 0, hi = merges;  // merges starting at or below c: in [lo, hi]
  while (hi > lo) {
    const uint32_t step = (hi - lo + kWave - 1) / kWave;
    const uint32_t at = lo + lane * step;
    const uint32_t below = static_cast<uint32_t>(__popcll(__ballot(at < hi && wm[at].chunk0 <= c)));
    if (below == 0) return lo - 1;
    const uint32_t nlo = lo + (below - 1) * step + 1;
    if (step == 1) return nlo - 1;
    const uint32_t nhi = lo + below * step;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
  return lo - 1;
}

// The chunks [begin, end) of a graph's parallel wide merges that wavefront
// gw of nw takes: a contiguous share, so that one search finds its first
// merge and the rest follow in order.
struct ChunkShare {
  uint32_t begin, end;
};
__device__ __forceinline__ ChunkShare chunk_share(uint32_t chunks) {
  const uint32_t nw = gridDim.x * (kBlock / kWave);
  const uint32_t gw = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const uint32_t per = (chunks + nw - 1) / nw;
  const uint64_t b = static_cast<uint64_t>(gw) * per;
  const uint64_t e = b + per < chunks ? b + per : chunks;
  return b < e ? ChunkShare{static_cast<uint32_t>(b), static_cast<uint32_t>(e)} : ChunkShare{0u, 0u};
}

// Second stage of the parallel wide merges: copy the moving old entries
// [stay, cur) of every merge to their staging slots (after its k new
// entries), kMergeChunk entries per wavefront unit.
__global__ __launch_bounds__(kBlock) void k_wide_copy_out(const BatchArgs* const* __restrict__ argv,
                                                          uint32_t which0) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (batch_failed(a.ctl) || a.ctl->nomem[which]) return;
  const unsigned long long pack = a.ctl->wpack[which];
  const ChunkShare sh = chunk_share(static_cast<uint32_t>(pack >> 32));
  if (sh.begin == sh.end) return;  // wavefront-uniform; no workgroup barriers here
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t p = wave_merge_of_chunk(a.wmerge, static_cast<uint32_t>(pack), sh.begin, lane);
  WideMerge m = a.wmerge[p];
  for (uint32_t c = sh.begin; c < sh.end; ++c) {
    while (c >= m.chunk0 + m.chunks) m = a.wmerge[++p];
    const uint32_t base = (c - m.chunk0) * kMergeChunk;
    const uint32_t moving = m.cur - m.stay;
    const uint32_t end = moving - base < kMergeChunk ? moving : base + kMergeChunk;
    const uint64_t src = static_cast<uint64_t>(m.seg_off) + m.stay;
    const uint64_t dst = static_cast<uint64_t>(m.new_off) + m.k;
    for (uint32_t i = base + lane; i < end; i += kWave) {
      X.ent[dst + i] = X.ent[src + i];
      X.prinv[dst + i] = X.prinv[src + i];
      X.w[dst + i] = X.w[src + i];
    }
  }
}

// New keys (sorted, in LDS) below a neighbour.
__device__ __forceinline__ uint32_t keys_below(const uint32_t* key, uint32_t k, uint32_t nbr) {
  uint32_t lo = 0, hi = k;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (key[mid] < nbr) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Last stage: write every staged entry to its merged slot, kMergeChunk old
// entries per wavefront unit.  The moving old entry i (i-th after stay) moves
// right by s_i, the new keys below it; the new entries j with
// s_{i-1} <= j < s_i (between old entries i-1 and i) land at stay + i + j and
// are written by the lane of old entry i, those above every old entry by the
// lane of the last one.  The slots are disjoint and fill [stay, cur + k);
// only staged copies are read, so the units of a row need no order.
__global__ __launch_bounds__(kBlock) void k_wide_place(const BatchArgs* const* __restrict__ argv,
                                                       uint32_t which0) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (batch_failed(a.ctl) || a.ctl->nomem[which]) return;
  __shared__ uint32_t s_new[kBlock / kWave][kTailChunk];  // a wavefront's merge's new keys
  const unsigned long long pack = a.ctl->wpack[which];
  const ChunkShare sh = chunk_share(static_cast<uint32_t>(pack >> 32));
  if (sh.begin == sh.end) return;  // wavefront-uniform; no workgroup barriers here
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t* keys = s_new[threadIdx.x / kWave];
  uint32_t p = wave_merge_of_chunk(a.wmerge, static_cast<uint32_t>(pack), sh.begin, lane);
  WideMerge m = a.wmerge[p];
  bool fresh = true;
  for (uint32_t c = sh.begin; c < sh.end; ++c) {
    while (c >= m.chunk0 + m.chunks) {
      m = a.wmerge[++p];
      fresh = true;
    }
    const uint64_t nw = m.new_off, od = static_cast<uint64_t>(m.new_off) + m.k;
    if (fresh) {
      wave_lds_order();  // the previous merge's keys are no longer read
      for (uint32_t j = lane; j < m.k; j += kWave) keys[j] = X.ent[nw + j].nbr;
      wave_lds_order();
      fresh = false;
    }
    const uint32_t base = (c - m.chunk0) * kMergeChunk;
    const uint32_t moving = m.cur - m.stay;
    const uint32_t end = moving - base < kMergeChunk ? moving : base + kMergeChunk;
    const uint64_t to0 = static_cast<uint64_t>(m.seg_off) + m.stay;  // slot of merged index 0
    if (moving == 0) {  // every new entry lands above the old ones
      for (uint32_t j = lane; j < m.k; j += kWave) {
        X.ent[to0 + j] = X.ent[nw + j];
        X.prinv[to0 + j] = X.prinv[nw + j];
        X.w[to0 + j] = X.w[nw + j];
      }
    }
    uint32_t last = 0;  // the lane's s_i of the previous pass
    for (uint32_t i0 = base; i0 < end; i0 += kWave) {  // wavefront-uniform
      const uint32_t i = i0 + lane;
      const bool valid = i < end;
      uint32_t below = 0;
      if (valid) {
        const Pair e = X.ent[od + i];
        below = keys_below(keys, m.k, e.nbr);
        X.ent[to0 + i + below] = e;
        X.prinv[to0 + i + below] = X.prinv[od + i];
        X.w[to0 + i + below] = X.w[od + i];
      }
      const uint32_t left = __shfl_up(below, 1, kWave);    // s_{i-1} within the pass
      const uint32_t carry = __shfl(last, kWave - 1, kWave);  // s_{i-1} for lane 0
      if (valid) {
        uint32_t from;
        if (lane > 0) from = left;
        else if (i0 > base) from = carry;
        else from = i > 0 ? keys_below(keys, m.k, X.ent[od + i - 1].nbr) : 0u;
        const uint32_t upto = i + 1 == moving ? m.k : below;
        for (uint32_t j = from; j < upto; ++j) {
          const uint64_t to = to0 + i + j + (j >= below ? 1u : 0u);
          X.ent[to] = X.ent[nw + j];
          X.prinv[to] = X.prinv[nw + j];
          X.w[to] = X.w[nw + j];
        }
      }
      last = below;
    }
  }
}

// After a pool shortfall: undo the per-row counters so phase 4 can run again
// once the pool has grown.
__global__ void k_phase4_reset(const BatchArgs* const* __restrict__ argv, uint32_t which0) {
  const uint32_t which = which0 + blockIdx.z;
  const P4 a = load_p4(argv, blockIdx.y, which);
  const DevGraph& X = a.X;
  if (which == 1) {
    // H's re-run deduplicates its additions afresh
    const uint64_t slots = args_of(argv, blockIdx.y)->hash_slots;
    for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < slots;
         i += uint64_t(gridDim.x) * blockDim.x) {
      a.hash[i].key = ~0ull;
      a.hash[i].minidx = ~0u;
    }
  }
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.ctl->touched[which]) return;
  X.pending[a.touched_rows[t]] = 0u;
}

__global__ void k_phase4_reset_ctl(const BatchArgs* const* __restrict__ argv, uint32_t which0) {
  const uint32_t which = which0 + blockIdx.z;
  BatchCtl* ctl = ctl_of(argv, blockIdx.y);
  if (threadIdx.x == 0) {
    ctl->touched[which] = 0;
    ctl->stage_used[which] = 0;
    ctl->wpack[which] = 0;
    ctl->need[which] = 0;
    ctl->nomem[which] = 0;
    ctl->wide[which] = 0;
    ctl->tpack[which] = 0;  // (rows listed by a finished phase 4 have their trees)
    ctl->tsmall[which] = 0;
  }
}

constexpr uint32_t kWideBlocks = 512;  // workgroups of the per-long-segment kernels
constexpr uint32_t kMergeBlocks = 2048;  // workgroups of the wide merges (latency-bound)
constexpr uint32_t kHubBlocks = 2048;  // workgroups of the prefix rebuild (memory-bound)

inline uint32_t blocks_for(uint64_t n, uint32_t per = kBlock) {
  return static_cast<uint32_t>((n + per - 1) / per);
}

}  // namespace

// ---- launchers ----------------------------------------------------------------------
// Per-batch kernels run on a grid of (x, F): blockIdx.y selects the batch, and
// x covers the largest batch of the launch.

namespace {
void launch_hub_tree(const Launch& L, uint32_t which0, uint32_t nw, hipStream_t st) {
  k_hub_tree_small<<<dim3(kHubBlocks, L.F, nw), kBlock, 0, st>>>(L.argv, which0);
  k_hub_tree<<<dim3(kHubBlocks, L.F, nw), kBlock, 0, st>>>(L.argv, which0);
}

inline dim3 grid_of(uint64_t n, uint32_t F, uint32_t per = kBlock) {
  const uint64_t b = (n + per - 1) / per;
  return dim3(static_cast<uint32_t>(b ? b : 1), F);
}

// Deferred fallbacks of the walk step (only deletions can have one).
void launch_fallback_wide(const Launch& L, hipStream_t st) {
  if (L.max_del == 0) return;
  const uint32_t nb = L.max_del < kWideBlocks ? L.max_del : kWideBlocks;
  k_fallback_wide<<<dim3(nb, L.F), kFbBlock, 0, st>>>(L.argv);
}
}  // namespace

void launch_batch_begin(const Launch& L, hipStream_t st) {
  const uint32_t nb = blocks_for(L.max_hash_slots) < 4096 ? blocks_for(L.max_hash_slots) : 4096;
  k_batch_begin<<<dim3(nb ? nb : 1, L.F), kBlock, 0, st>>>(L.argv);
}

void launch_validate(const Launch& L, hipStream_t st) {
  if (L.max_nu == 0) return;
  k_validate_a<<<grid_of(L.max_nu, L.F), kBlock, 0, st>>>(L.argv);
  k_validate_b<<<grid_of(L.max_nu, L.F), kBlock, 0, st>>>(L.argv);
}

void launch_phase1(const Launch& L, hipStream_t st) {
  if (L.max_del == 0) return;
  // long segments' weight trees are updated in place by the tombstones
  k_phase1<<<grid_of(L.max_del, L.F), kBlock, 0, st>>>(L.argv);
}

void launch_walks(const Launch& L, hipStream_t st) {
  if (L.max_nu == 0) return;
  const uint32_t sg = L.stage;
  if (L.hubs) {
    constexpr int B = kLockstepBlock<true>;
    const dim3 g = grid_of(L.max_nu, L.F, B / kWave);
    if (L.coop) k_walks<true, true><<<g, B, 0, st>>>(L.argv, sg);
    else k_walks<true, false><<<g, B, 0, st>>>(L.argv, sg);
  } else {
    constexpr int B = kLockstepBlock<false>;
    const dim3 g = grid_of(L.max_nu, L.F, B / kWave);
    if (L.coop) k_walks<false, true><<<g, B, 0, st>>>(L.argv, sg);
    else k_walks<false, false><<<g, B, 0, st>>>(L.argv, sg);
  }
}

void launch_walk_fallbacks(const Launch& L, hipStream_t st) {
  if (L.stage != kStageInsertions) launch_fallback_wide(L, st);  // only deletions have one
}

void launch_sum_counters(const Launch& L, hipStream_t st) {
  if (L.max_nu == 0) return;
  const uint32_t nb = blocks_for(L.max_nu) < 64 ? blocks_for(L.max_nu) : 64;
  k_sum_counters<<<dim3(nb, L.F), kBlock, 0, st>>>(L.argv);
}

void launch_queue_prepare(const Launch& L, hipStream_t st) {
  if (L.max_nu == 0) return;
  const uint32_t per = kWalkBlock / kWave;
  k_count_walkers<<<grid_of(L.max_nu, L.F), kBlock, 0, st>>>(L.argv);
  k_scan_tiles<<<grid_of(L.max_nu, L.F, kScanTile), kBlock, 0, st>>>(L.argv);
  k_scan_top<<<dim3(1, L.F), kBlock, 0, st>>>(L.argv);
  k_scan_add<<<grid_of(L.max_nu, L.F, kScanTile), kBlock, 0, st>>>(L.argv);
  if (L.upw == 0) k_expand_items<<<grid_of(L.max_nu, L.F, per), kBlock, 0, st>>>(L.argv);
}

void launch_walk_queue(const Launch& L, hipStream_t st) {
  if (L.max_nu == 0) return;
  if (L.tail_lanes > 0) {
    const uint32_t upw = L.upw < 1 ? 1u : (L.upw < kMaxUpw ? L.upw : kMaxUpw);
    const uint32_t waves = (L.max_nu + upw - 1) / upw;
    const dim3 gh = grid_of(L.max_nu, L.F, kWalkBlock / kWave);
    const dim3 gt = grid_of(waves, L.F, kBlock / kWave);
    if (L.hubs) {
      k_walk_head<true><<<gh, kWalkBlock, 0, st>>>(L.argv);
      k_walk_tail<true><<<gt, kBlock, 0, st>>>(L.argv, upw);
    } else {
      k_walk_head<false><<<gh, kWalkBlock, 0, st>>>(L.argv);
      k_walk_tail<false><<<gt, kBlock, 0, st>>>(L.argv, upw);
    }
  } else if (L.upw > 0) {
    const uint32_t upw = L.upw < kMaxUpw ? L.upw : kMaxUpw;
    const uint32_t waves = (L.max_nu + upw - 1) / upw;
    if (L.hubs) k_walk_range<true><<<grid_of(waves, L.F, kBlock / kWave), kBlock, 0, st>>>(L.argv, upw);
    else k_walk_range<false><<<grid_of(waves, L.F, kBlock / kWave), kBlock, 0, st>>>(L.argv, upw);
  } else if (L.F > 1) {
    k_walk_queue<true><<<L.walk_blocks, kBlock, 0, st>>>(L.argv);
  } else {
    k_walk_queue<false><<<L.walk_blocks, kBlock, 0, st>>>(L.argv);
  }
}

void launch_queue_finish(const Launch& L, hipStream_t st) {
  if (L.max_nu == 0) return;
  if (L.hubs) k_reduce_updates<true><<<grid_of(L.max_nu, L.F, kWalkBlock / kWave), kWalkBlock, 0, st>>>(L.argv);
  else k_reduce_updates<false><<<grid_of(L.max_nu, L.F, kWalkBlock / kWave), kWalkBlock, 0, st>>>(L.argv);
  launch_fallback_wide(L, st);
}

namespace {

// Phase 4 of graphs which0 .. which0 + nw - 1 (both graphs at once normally;
// one when a pool repair re-runs it).
void phase4_sequence(const Launch& L, uint32_t which0, uint32_t nw, hipStream_t st) {
  uint64_t cap = 0;  // upper bound of the directed entries and of the touched rows
  for (uint32_t w = which0; w < which0 + nw; ++w) {
    const uint64_t c = w == 0 ? 2ull * L.max_ins : 2ull * L.max_hadd_cap;
    cap = c > cap ? c : cap;
  }
  if (cap == 0) return;
  const dim3 g(static_cast<uint32_t>((cap + kBlock - 1) / kBlock), L.F, nw);
  k_add_prepare<<<g, kBlock, 0, st>>>(L.argv, which0, L.h_lo, L.h_hi);
  k_rows_plan<<<g, kBlock, 0, st>>>(L.argv, which0);
  k_pool_check<<<dim3(1, L.F, nw), 64, 0, st>>>(L.argv, which0);
  const dim3 both(g.x + kWideBlocks, L.F, nw);  // short rows, then long rows
  k_rows_relocate<<<both, kBlock, 0, st>>>(L.argv, which0, g.x);
  k_add_place<<<g, kBlock, 0, st>>>(L.argv, which0, L.h_lo, L.h_hi);
  k_rows_merge<<<dim3(g.x + kMergeBlocks, L.F, nw), kBlock, 0, st>>>(L.argv, which0, g.x);
  const dim3 wide(kMergeBlocks, L.F, nw);
  k_wide_copy_out<<<wide, kBlock, 0, st>>>(L.argv, which0);
  k_wide_place<<<wide, kBlock, 0, st>>>(L.argv, which0);
  launch_hub_tree(L, which0, nw, st);
}

}  // namespace

void launch_phase4(const Launch& L, int which, hipStream_t st) {
  phase4_sequence(L, static_cast<uint32_t>(which), 1, st);
}

void launch_phase4_both(const Launch& L, hipStream_t st) { phase4_sequence(L, 0, 2, st); }

void launch_phase4_clear(const Launch& L, int which, hipStream_t st) {
  k_phase4_reset_ctl<<<dim3(1, L.F, 1), 64, 0, st>>>(L.argv, static_cast<uint32_t>(which));
}

void launch_phase4_reset(const Launch& L, int which, hipStream_t st) {
  const uint64_t cap = which == 0 ? 2ull * L.max_ins : 2ull * L.max_hadd_cap;
  if (cap == 0) return;
  const dim3 g(static_cast<uint32_t>((cap + kBlock - 1) / kBlock), L.F, 1);
  k_phase4_reset<<<g, kBlock, 0, st>>>(L.argv, static_cast<uint32_t>(which));
  k_phase4_reset_ctl<<<dim3(1, L.F, 1), 64, 0, st>>>(L.argv, static_cast<uint32_t>(which));
}

}  // namespace dyg
