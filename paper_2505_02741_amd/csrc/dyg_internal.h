// Library-internal declarations shared by the HIP translation units of
// libdygrass.  Not installed; the public interface is include/dygrass.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dyg {

// ---------------------------------------------------------------------------
// Device adjacency of one graph (the original graph G or the sparsifier H).
//
// Every vertex has a 64-byte row: a header and room for kInline (neighbour,
// quantised weight) pairs.  A vertex with at most kInline neighbours keeps
// those pairs inside its row, so a walk step there reads one cache line; their
// resistances 1/w and weights sit in side arrays (rinl, winl) because a step
// needs only the chosen one.  A longer row owns a segment of the entry pool:
// `len` entries in ascending neighbour order followed by `cap - len` free
// slots (per-node slack).  A deleted edge stays in place as a tombstone
// (qw == 0) until its segment is relocated or compacted; a zero weight never
// wins the cumulative search, so walks skip tombstones without testing them.
// The inline slots of a row past its len also hold qw == 0 (rows are zeroed
// when laid out, and an inline row only grows until it moves to the pool).
// Neighbour ids are unique within a row (a re-inserted edge revives its
// tombstone).  Pool entries are stored as 8-byte (neighbour, weight) pairs
// (`ent`), with their resistances and weights in side arrays (`prinv`, `w`),
// so a walk step's scan reads only what the choice needs; every pool segment
// starts at an even slot, so a scan reads two pairs per 16-byte load.
// Ent is the value of one entry as the host and phase 4 handle it.
struct Ent {
  uint32_t nbr;  // neighbour id
  uint32_t qw;   // quantised weight, 0 = tombstone
  double rinv;   // resistance 1/w
};

constexpr uint32_t kInline = 6;              // pairs stored inside the row
constexpr uint32_t kInlineOff = 0xFFFFFFFFu;  // `off` of a row whose entries are inline

struct RowHdr {
  uint32_t off;   // first pool entry, or kInlineOff
  uint32_t len;   // entries in use, tombstones included
  uint32_t cap;   // slots owned (kInline for an inline row)
  uint32_t dead;  // tombstones among the len entries
};

struct Pair {
  uint32_t nbr, qw;
};

struct Row {
  RowHdr h;
  Pair inl[kInline];
};

static_assert(sizeof(RowHdr) == 16, "RowHdr layout");
static_assert(sizeof(Ent) == 16, "Ent layout");
static_assert(sizeof(Row) == 64, "Row layout");

constexpr uint32_t kNone = 0xFFFFFFFFu;
// Segments longer than this keep a weight tree (below), so a walker picks a
// neighbour with a few block reads instead of a scan.
constexpr uint32_t kHub = 64;
constexpr uint32_t kMaxWalkers = 1024;
constexpr uint32_t kMaxSteps = 1024;
constexpr uint32_t kMaxUpw = 8;  // updates per wavefront of the range walk
// While every quantised weight stays below this, the six-term running sums
// of an inline row fit 32 bits; the walks then use 32-bit sums.
constexpr uint32_t kHeavyQw = 1u << 29;


// ---------------------------------------------------------------------------
// Weight tree of a long segment (len > kHub).  Such a segment starts at a
// pool offset that is a multiple of kHubAlign and owns a multiple of kFan
// slots.  Level 0 is implicit: its value i (i < len) is the running sum of
// the quantised weights over entry i's block of kFan entries, from the
// block's first entry to i, which a walker sums from the block's pairs as it
// reads them.  Level l >= 1 has tree_n(len, l) values; value b is the running sum,
// over b's block of kFan values, of the totals of the level-(l-1) blocks
// (block b of level l-1 = values kFan*b .. kFan*b + kFan-1).  Levels 1.. are
// stored one after another from tree[off / 4] (tree_base gives each level's
// start), each padded to a multiple of kFan values.  The top level
// tree_top(len) is the first with at most kFan values; slot kFan-1 of its one
// block holds the segment total.  Every other slot past a level's last value
// (up to the next multiple of kFan) holds kTreePad.
// A walker finds the entry whose running total first exceeds a target with
// one 128-byte read per level (kFan values, or the leaf block's kFan pairs);
// changing one entry's weight adds the difference to the rest of its block
// on every stored level.
constexpr uint32_t kFan = 16;
constexpr uint32_t kHubAlign = 64;           // pool offset alignment of long segments
constexpr unsigned long long kTreePad = ~0ull;

__host__ __device__ inline uint32_t round_fan(uint32_t x) { return (x + kFan - 1) & ~(kFan - 1); }

// Levels above level 0 (len > kFan).
__host__ __device__ inline uint32_t tree_top(uint32_t len) {
  uint32_t bits = 0;
  for (uint32_t x = len - 1; x; x >>= 1) ++bits;  // bits of len - 1
  return (bits + 3) / 4 - 1;
}

// Values on level l.
__host__ __device__ inline uint32_t tree_n(uint32_t len, uint32_t l) {
  return ((len - 1) >> (4 * l)) + 1;
}

// Start of level l >= 1 within the segment's tree slots (tree + off / 4).
__host__ __device__ inline uint32_t tree_base(uint32_t len, uint32_t l) {
  uint32_t b = 0;
  for (uint32_t m = 1; m < l; ++m) b += round_fan(tree_n(len, m));
  return b;
}

// The top block of a long segment's weight tree, when that level has at most
// kInlineTop values, is also kept in the row's 48 inline bytes (a pool row
// does not use them): its values 0 .. n-2 as 64-bit words 0 .. n-2 and the
// segment total as word kInline - 1, so that a walker has it with the row.
// (Value n-1, the running sum of the whole level, is the total again.)
constexpr uint32_t kInlineTop = kInline;
__host__ __device__ inline bool top_inline(uint32_t len) {
  return tree_n(len, tree_top(len)) <= kInlineTop;
}

struct DevGraph {
  Row* rows = nullptr;        // [n] 64-byte rows
  Pair* ent = nullptr;        // [pool_cap] (neighbour, quantised weight) of each pool entry
  double* prinv = nullptr;    // [pool_cap] 1/w of each pool entry
  double* w = nullptr;        // [pool_cap] weight of each pool entry (cold)
  double* rinl = nullptr;     // [n * kInline] 1/w of each inline entry
  double* winl = nullptr;     // [n * kInline] weight of each inline entry (cold)
  uint32_t* pending = nullptr;  // [n] per-row counter, zero between batches
  unsigned long long* tree = nullptr; // [pool_cap / 4 + kFan] weight tree levels 1.. (rows with len > kHub)
  uint32_t* mark = nullptr;     // [n] "prefix needs rebuilding" flag, zero between uses
  uint64_t pool_cap = 0;      // entries
};

// Edge to be added to a graph in phase 4 (one record per undirected edge).
struct AddRec {
  uint32_t a, b;
  uint32_t qw, pad;
  double rinv;
  double w;
};
static_assert(sizeof(AddRec) == 32, "AddRec layout");

// Walker index bits of WalkItem::walker; the bits above hold the batch (0..63)
// when several batches share one queue.
// Variants of the update rule (the paper's alternatives, off by default):
// odd walkers start at the second endpoint and aim at the first (Sec. III-C
// deploys walkers from p or from q); a hitting deletion recovers the loop
// erasure of its winner's path; the deletions and their recoveries enter H
// before the insertion walks (Sec. III-F otherwise defers every update to the
// batch end).
constexpr uint32_t kVarBothEnds = 1u;
constexpr uint32_t kVarLoopErased = 2u;
constexpr uint32_t kVarTwoStage = 4u;

constexpr uint32_t kWalkerBits = 10;
constexpr uint32_t kMaxFused = 64;

// One walker of the batched form's work queue.
struct WalkItem {
  uint32_t p, q;    // start vertex, target
  uint32_t upd;     // update index in the batch (insertions first)
  uint16_t walker;  // walker index within the update | batch << kWalkerBits
  uint16_t L;       // step limit
  double w_pq;      // inserted edge weight (threshold test), 0 for deletions
};
static_assert(sizeof(WalkItem) == 24, "WalkItem layout");

// Per-update result, layout identical to dyg_update_result.
struct UpdRes {
  uint8_t kind, flag, any_hit, reserved;
  uint16_t winner, n_rec;
  uint32_t steps;
  uint32_t reserved2;
  double Rmin;
};
static_assert(sizeof(UpdRes) == 24, "UpdRes layout");

struct WalkerRec {
  uint8_t hit, pad;
  uint16_t steps;
  uint32_t end;
  double R;
};
static_assert(sizeof(WalkerRec) == 16, "WalkerRec layout");

// Outcome of one queued walker (batched form): the public record plus the
// algorithmic bytes its steps gathered.
struct WalkOut {
  uint32_t end;
  uint16_t steps;
  uint8_t hit, pad;
  uint32_t bytes;
  uint32_t pad2;
  double R;
};
static_assert(sizeof(WalkOut) == 24, "WalkOut layout");

// A walker handed from the head walk to the tail walk (batched form, head/tail
// schedule): its state after `t` steps.
struct TailState {
  uint32_t x, prev, t, bytes;
  uint32_t qprev, walker;
  double R;
  const double* rpend;  // 1/w of the last edge taken, not yet added to R
};
static_assert(sizeof(TailState) == 40, "TailState layout");

// Device-resident control block of one batch.
struct BatchCtl {
  unsigned long long err_key;   // min over (phase, update, code); ~0 = valid
  uint32_t touched[2];          // touched rows, per graph (0 = G, 1 = H)
  unsigned long long need[2];   // pool slots needed by relocations, per graph
  uint32_t nomem[2];            // phase-4 pool shortfall, per graph
  uint32_t wide[2];             // touched rows moved or merged by a workgroup, per graph
  uint32_t hubs;                // set when phase 4 leaves a row longer than kHub
  uint32_t fb_count;            // deletions whose fallback scan is left to k_fallback_wide
  unsigned long long pool_top[2];  // next free pool slot, per graph
  unsigned long long stage_used[2];  // pool slots past pool_top used to stage wide merges
  unsigned long long wpack[2];  // parallel wide merges: (chunks << 32) | merges, per graph
  unsigned long long tpack[2];  // weight trees to rebuild: (chunks << 32) | rows, per graph
  unsigned long long tsmall[2]; // those of rows of at most kTreeSmall entries, per graph
  unsigned long long walk_items;       // walkers queued (queue control only)
  unsigned long long queue_next;       // next queue item to hand out (queue control only)
  unsigned long long item_base;        // first queue item of this batch
  // cumulative over the context's life (never reset by a batch)
  unsigned long long steps_total;      // walker steps taken
  unsigned long long alg_bytes_total;  // algorithmic gathered bytes of those steps
  uint32_t heavy;  // some quantised weight of G or H is >= kHeavyQw (set, never cleared)
};

// A wide merge done by many workgroups: the row's k appended entries sorted
// and staged at new_off, its old entries [stay, cur) staged right after them
// (new_off + k); both are written back to their merged slots by chunks of
// kMergeChunk old entries, chunk0 .. chunk0 + chunks - 1 of the graph's list.
struct WideMerge {
  uint32_t r;        // row
  uint32_t k;        // appended entries
  uint32_t stay;     // first old entry that moves (the first new entry's final slot)
  uint32_t cur;      // old entries
  uint32_t seg_off;  // the row's pool segment
  uint32_t new_off;  // pool slot of the staged entries
  uint32_t chunk0;   // first chunk (increasing with the merge's index)
  uint32_t chunks;   // at least one
};
static_assert(sizeof(WideMerge) == 32, "WideMerge layout");
constexpr uint32_t kMergeChunk = 512;  // old entries per wavefront unit of a parallel wide merge

// Slot of the validation / dedup hash table.
struct HashSlot {
  unsigned long long key;  // ~0 = empty
  uint32_t minidx;
  uint32_t pad;
};

// Everything the kernels of one batch need.
struct BatchArgs {
  uint32_t n;
  uint32_t n_ins, n_del;
  const uint32_t *iu, *iv;
  const double* iw;
  const uint32_t *du, *dv;
  const uint16_t *s, *L;  // per update or null
  uint32_t s_def, L_def;
  uint32_t Lcap;           // >= every L of the batch, >= 2
  uint32_t scap;           // >= every s of the batch
  uint64_t uid_base;
  uint64_t seed;
  double K;
  int has_K;
  int bounce;
  uint32_t variant;  // kVar* bits (variants of the update rule)
  double w_ref;
  int Q;
  // work buffers
  uint32_t* ins_qw;     // [n_ins]
  double* ins_rinv;     // [n_ins]
  uint8_t* in_h;        // [n_del]
  UpdRes* res;          // [n_ins + n_del]
  WalkerRec* wrec;      // optional [sum s]
  const uint64_t* wofs; // optional [n_ins + n_del]
  AddRec* hadd;         // [hadd_cap]: slot i for insertion i, then Lcap slots per deletion
  uint32_t* ubytes;     // [n_ins + n_del] algorithmic bytes gathered by each update's walks
  uint32_t* fb_list;    // [n_del] updates whose no-hit fallback scans a long row (ctl->fb_count)
  uint32_t hadd_cap;
  HashSlot* hash;       // validation: repeats within the batch
  HashSlot* hash2;      // phase 4: edges recovered more than once
  uint32_t hash_mask;
  uint64_t hash_slots;
  DevGraph g[2];              // 0 = G, 1 = H
  BatchCtl* ctl;
  BatchCtl* qctl;  // work-queue control shared by the batches of one launch
  // per-graph phase-4 scratch
  uint32_t* touched_rows[2];  // [add capacity]
  uint32_t* touched_k[2];
  uint32_t* touched_need[2];
  uint8_t* add_keep[2];       // per directed add entry: 1 = needs a new slot
  uint32_t* dirty_rows[2];    // rows whose weight tree must be rebuilt, in claim order
  uint32_t* dirty_chunk0[2];  // first tree chunk of each (increasing)
  uint32_t* dirty_small[2];   // rows of at most kTreeSmall entries whose tree is rebuilt
  uint32_t* wide_rows[2];     // indices into touched_* of the rows with a wide flag
  WideMerge* wmerge[2];       // [add capacity] the parallel wide merges, in claim order
  // batched form: walker work queue
  uint32_t* qcount;              // [n_ins + n_del] walkers of each update
  unsigned long long* qofs;      // [n_ins + n_del] first item of each update
  unsigned long long* qtile;     // [tiles] scan carry
  WalkItem* items;               // [items] walker of each queue item
  uint32_t refill_min;           // idle lanes that trigger a refill (1..64)
  uint32_t upw;                  // updates per wavefront of the range walk (0 = queue)
  WalkOut* wres;                 // [items] outcome of each walker
  // head/tail schedule (tail_lanes > 0): a head wavefront per update stops
  // once at most tail_lanes of its lanes still walk and hands those walkers on
  uint32_t tail_lanes;
  TailState* tstate;             // [items] the survivors of update u from item qofs[u]
  uint32_t* tcount;              // [n_ins + n_del] survivors of each update
};

// One launch of F batches (F = 1 for a single context; up to kMaxFused when a
// serving round fuses batches of different graphs).
struct Launch {
  const BatchArgs* const* argv;  // device array of F pointers to device BatchArgs
  uint32_t F;
  uint32_t max_nu, max_ins, max_del;  // largest batch of the launch (grid sizes)
  uint64_t max_hadd_cap, max_hash_slots;
  uint32_t walk_blocks;               // persistent walk grid
  uint32_t upw;                       // updates per wavefront (0 = work queue)
  bool hubs;                          // some row of a graph may be longer than kHub
  bool coop;                          // plain walks: rows of the walked graphs are mostly pool rows
  uint32_t tail_lanes;                // batched form: head/tail schedule (0 = off)
  uint32_t stage = 0;                 // plain walks: all updates (0), deletions (1), insertions (2)
  uint32_t h_lo = 0, h_hi = ~0u;      // phase 4: H additions from these slots only
};

// Host-side checks of a graph given as CSR (defined in dyg_api.hip): returns
// DYG_OK or a DYG_E_* code; *wmax = the largest weight.
int validate_csr(uint32_t n, const uint64_t* rowptr, const uint32_t* col, const double* w,
                 double* wmax);

// Host-side launchers (defined in dyg_kernels.hip), all asynchronous on
// `stream`.
void launch_batch_begin(const Launch& L, hipStream_t stream);
void launch_validate(const Launch& L, hipStream_t stream);
void launch_phase1(const Launch& L, hipStream_t stream);
// Plain form: one wavefront per update.
void launch_walks(const Launch& L, hipStream_t stream);
// The no-hit fallbacks the walk kernel left to k_fallback_wide (long G rows).
void launch_walk_fallbacks(const Launch& L, hipStream_t stream);
// Batched form: count, scan and expand the walker items; one persistent
// queue walk over every walker of the F batches; per-update reduction.
void launch_queue_prepare(const Launch& L, hipStream_t stream);
void launch_walk_queue(const Launch& L, hipStream_t stream);
void launch_queue_finish(const Launch& L, hipStream_t stream);
// Either form, after the walks: batch totals of steps and algorithmic bytes.
void launch_sum_counters(const Launch& L, hipStream_t stream);
// Phase 4 on both graphs at once (G += insertions, H += hadd records), or on
// one graph (which = 0: G, 1: H) when a pool repair re-runs it.
void launch_phase4_both(const Launch& L, hipStream_t stream);
void launch_phase4(const Launch& L, int which, hipStream_t stream);
void launch_phase4_reset(const Launch& L, int which, hipStream_t stream);
// Phase-4 counters of graph `which` back to zero (between the two stages of
// a two-stage batch).
void launch_phase4_clear(const Launch& L, int which, hipStream_t stream);
// The walk launch of the plain form takes the updates L.stage names.
constexpr uint32_t kStageDeletions = 1, kStageInsertions = 2;

}  // namespace dyg
