/*
 * dygrass.h -- C ABI of libdygrass, an MI355X (gfx950) implementation of the
 * update path of dyGRASS (Yuan, Aghdaei, Feng, "dyGRASS: Dynamic Spectral
 * Graph Sparsification via Localized Random Walks on GPUs", arXiv 2505.02741).
 *
 * The library keeps an undirected weighted graph G and a spectral sparsifier
 * H (a subgraph of G with the same weights) resident in GPU memory and
 * updates H as batches of edge insertions and deletions arrive:
 *
 *  - insertion (p,q,w): s non-backtracking, weight-biased walkers start at p
 *    in H; each stops when w*R exceeds K (R = sum of 1/w along its path), after
 *    L steps, or at a leaf.  The edge enters H iff no walker reaches q
 *    (Sec. III-B; Algorithm 1, insertion branch).
 *  - deletion (u,v): if the edge is in H, s walkers start at u in G without
 *    the edge; the hitting walker with the least R (Eq. 12) has its path edges
 *    that are missing from H added back; with no hit, per endpoint the G edge
 *    of least resistance missing from H is added (Sec. III-C; Algorithm 1,
 *    deletion branch).
 *  - batches: every walk of a batch reads the state after the batch's
 *    deletions; insertions and recovered edges are applied at the end of the
 *    batch (Sec. III-F, batch processing on the GPU).
 *
 * Random numbers: Philox-4x32-10 (Salmon et al., SC'11) keyed by the 64-bit
 * seed, counter (step/2, walker, uid low, uid high); update i of a batch has
 * uid = uid_base + i with insertions numbered before deletions.  Results are
 * therefore independent of scheduling and bit-reproducible.
 *
 * Ownership: every pointer argument is owned by the caller and only read or
 * written during the call; the library copies what it keeps.  A context owns
 * its GPU memory until dyg_destroy.  Calls on one context must not overlap;
 * different contexts are independent.
 *
 * Errors: every int-returning call returns DYG_OK (0) or a negative dyg_status.
 * A failed dyg_apply_batch leaves G, H and uid_base unchanged.
 */
#ifndef DYGRASS_H
#define DYGRASS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dyg_ctx dyg_ctx;

typedef enum {
  DYG_OK = 0,
  DYG_E_INVALID_ARG = -1,        /* bad pointer, size, parameter or s/L bound   */
  DYG_E_SELF_LOOP = -2,          /* an edge (u,u)                               */
  DYG_E_VERTEX_RANGE = -3,       /* a vertex id >= n                            */
  DYG_E_BAD_WEIGHT = -4,         /* weight <= 0, NaN, infinite, or so small that
                                    its resistance 1/w overflows                 */
  DYG_E_EDGE_EXISTS = -5,        /* inserted edge already in G (Sec. III-B)     */
  DYG_E_EDGE_MISSING = -6,       /* deleted edge not in G (Sec. III-C)          */
  DYG_E_DUPLICATE_IN_BATCH = -7, /* the same edge twice in one list             */
  DYG_E_H_NOT_SUBSET = -8,       /* init: a sparsifier edge not in G            */
  DYG_E_NOMEM = -9,              /* device or host allocation failed            */
  DYG_E_DEVICE = -10,            /* a HIP runtime call failed                   */
  DYG_E_TOO_LARGE = -11,         /* dyg_apply_batch_dev_static: the batch needs
                                    more than DYG_STATIC_SCRATCH_BYTES         */
  DYG_E_BUSY = -12               /* dyg_apply_batch_dev_static: a batch not yet
                                    synced holds the context or the static array */
} dyg_status;

enum { DYG_DEAD_END_TERMINATE = 0, DYG_DEAD_END_BOUNCE = 1 };

/* dyg_params.flags */
#define DYG_FLAG_LEAN_POOLS 1u /* size entry pools to the live entries plus 64 spare
                                  slots (instead of twice the live entries plus 8
                                  per vertex) and grow on demand                 */
#define DYG_FLAG_TIMING 2u     /* time the walk kernel and each batch with HIP
                                  events on the launch stream (dyg_stats)        */
#define DYG_FLAG_BATCHED 4u    /* batched form: walker counts are scanned on the
                                  device and the walks run as one launch in which
                                  a lane takes a new walker as soon as its own
                                  stops (schedule in dyg_tuning; same results as
                                  the plain one-wavefront-per-update form)       */
#define DYG_FLAG_GRAPH 8u      /* run each batch's launch sequence as a captured
                                  HIP graph, one per power-of-two size class of
                                  (insertions, deletions), replayed for every
                                  batch of that class                            */
#define DYG_FLAG_AUTOTUNE 16u  /* batched form: the first batches each try one
                                  walk schedule from a fixed candidate list, the
                                  lockstep walk among them (launched directly,
                                  walks and per-update decisions timed with HIP
                                  events); the schedule with the least such time
                                  per walker step is then kept (dyg_get_tuning
                                  reports it)                                     */
#define DYG_FLAG_TIMING_WALK 32u /* time the walk kernel alone: two HIP events per
                                  batch around it (dyg_stats walk_ms_*), none
                                  around the batch (batch_ms_last stays 0), so
                                  that timing disturbs the stream least          */
#define DYG_FLAG_FAIL_POOL_GROWTH 64u /* for tests of the failure paths: growing a
                                  pool that ran short fails as if the device had
                                  no memory left (the batch reports DYG_E_NOMEM
                                  and the context takes no further batches)      */
/* Variants of the update rule (the paper's alternatives; off by default): */
#define DYG_FLAG_BOTH_ENDS 128u  /* walker k starts at the second endpoint and aims
                                    at the first when k is odd (Sec. III-C lets
                                    walkers start at either endpoint)               */
#define DYG_FLAG_LOOP_ERASED 256u /* a hitting deletion recovers the edges of the
                                    chronological loop erasure of its winner's path
                                    (those not in H) instead of every edge the path
                                    traversed (Sec. III-C)                          */
#define DYG_FLAG_TWO_STAGE 512u  /* a batch's deletion walks and their recovered
                                    edges enter H before its insertion walks, which
                                    then read the repaired H (Sec. III-F otherwise
                                    defers every update to the batch end).  The
                                    host checks H's pool between the stages, so a
                                    two-stage batch is launched directly (no
                                    captured graph) with the lockstep walk in
                                    either form.  INVALID_ARG with
                                    DYG_FLAG_AUTOTUNE; refused by the serving
                                    engine and dyg_apply_batch_dev_static         */

#define DYG_MAX_WALKERS 1024 /* per update */
#define DYG_MAX_STEPS 1024   /* per walker */

typedef struct {
  uint64_t seed;      /* Philox key                                              */
  double K;           /* distortion threshold; +INFINITY disables it (Sec. III-B) */
  uint16_t s_default; /* walkers per update when the batch gives none            */
  uint16_t L_default; /* step limit T per walker when the batch gives none       */
  uint8_t Q;          /* bits of the quantised weights, 1..31; 24 recommended    */
  uint8_t dead_end;   /* DYG_DEAD_END_TERMINATE (the paper's leaf rule) or BOUNCE */
  uint16_t reserved0;
  double w_ref;       /* weight that maps to 2^Q; 0 = largest weight of G0       */
  double slack;       /* spare slots per vertex segment, as a fraction (>= 0)    */
  uint64_t uid_base;  /* uid of the first update of the next batch               */
  uint32_t flags;     /* DYG_FLAG_* bits                                         */
  uint32_t reserved1;
} dyg_params;

/* Per-update result (24 bytes), insertions first, then deletions. */
typedef struct {
  uint8_t kind;     /* 0 insertion, 1 deletion                                   */
  uint8_t flag;     /* insertion: edge added to H; deletion: edge was in H       */
  uint8_t any_hit;  /* some walker reached the other endpoint                    */
  uint8_t reserved;
  uint16_t winner;  /* walker index of the least-R hit, 0xFFFF if none           */
  uint16_t n_rec;   /* deletion: edges recovered into H (path or fallback)      */
  uint32_t steps;   /* steps taken by all walkers of the update                  */
  uint32_t reserved2;
  double Rmin;      /* least resistance sum over hitting walkers, +inf if none   */
} dyg_update_result;

/* Per-walker record (16 bytes), for verification. */
typedef struct {
  uint8_t hit;
  uint8_t reserved;
  uint16_t steps; /* edges traversed                                            */
  uint32_t end;   /* vertex where the walker stopped                            */
  double R;       /* resistance sum of its path                                 */
} dyg_walker_record;

typedef struct {
  uint32_t n;
  uint32_t reserved;
  uint64_t g_edges, h_edges;     /* live undirected edges                       */
  uint64_t g_pool_used, g_pool_cap; /* directed entry slots                     */
  uint64_t h_pool_used, h_pool_cap;
  uint64_t g_dead, h_dead;       /* tombstoned directed entries                 */
  uint64_t uid_base;
  uint64_t batches;
  uint64_t compactions;
  double w_ref;
  /* walk work since dyg_init: steps taken and the bytes those steps must
   * gather (per step at a vertex of live degree d: 16 + 8d for d <= 64,
   * 32 + 12 ceil(log2 d) above) */
  uint64_t walk_steps;
  uint64_t walk_alg_bytes;
  /* with DYG_FLAG_TIMING or DYG_FLAG_TIMING_WALK: walk-kernel launches timed,
   * their total and last duration (ms); with DYG_FLAG_TIMING also the device
   * time of the last batch (ms) */
  uint64_t walk_launches;
  double walk_ms_total;
  double walk_ms_last;
  double batch_ms_last;
} dyg_stats_t;

void dyg_default_params(dyg_params* p);

/*
 * Create a context from G0 and H0 (Algorithm 1 inputs G(0), H(0)).
 *   n        vertices, 1 <= n < 2^31
 *   rowptr   host, n+1 entries; col/w host, rowptr[n] entries: symmetric CSR of
 *            G0, each row ascending by neighbour, no self loops, weights > 0
 *            and finite, (u,v) and (v,u) with equal weights
 *   h_u/h_v  host, h_m edges of H0; each must be an edge of G0 (its weight is
 *            taken from G0), no repeats
 * Errors: INVALID_ARG, VERTEX_RANGE, SELF_LOOP, BAD_WEIGHT, H_NOT_SUBSET,
 * DUPLICATE_IN_BATCH (H0 repeats an edge), NOMEM, DEVICE.  *out is set only
 * on success.
 */
int dyg_init(dyg_ctx** out, uint32_t n, const uint64_t* rowptr, const uint32_t* col,
             const double* w, uint64_t h_m, const uint32_t* h_u, const uint32_t* h_v,
             const dyg_params* params);

/*
 * Apply one batch (Algorithm 1 over the batch, Sec. III-F deferral).
 *   iu/iv/iw  host, n_ins insertions (p,q,w): p is where the walkers start
 *   du/dv     host, n_del deletions (u,v): u is where the walkers start
 *   s, L      host, NULL or n_ins+n_del entries (insertions first): walkers and
 *             step limit per update, each <= 1024; NULL means the defaults
 *   results   host, NULL or n_ins+n_del records
 *   walkers   host, NULL or sum-of-s records in update order, walker order
 * Validation order: insertions in order (range, self loop, weight, already in
 * G, repeated earlier in the batch), then deletions in order (range, self
 * loop, not in G, repeated), then s/L bounds; the first failure is returned.
 */
int dyg_apply_batch(dyg_ctx* ctx, uint64_t n_ins, const uint32_t* iu, const uint32_t* iv,
                    const double* iw, uint64_t n_del, const uint32_t* du, const uint32_t* dv,
                    const uint16_t* s, const uint16_t* L, dyg_update_result* results,
                    dyg_walker_record* walkers);

/*
 * Device-resident batch for callers that keep inputs in GPU memory (PyTorch
 * tensors, a serving loop).  All pointers are device pointers; s, L and
 * results may be NULL.  An L or s above its stated bound fails validation.
 */
typedef struct {
  uint64_t n_ins, n_del;
  const uint32_t *iu, *iv;
  const double* iw;
  const uint32_t *du, *dv;
  const uint16_t *s, *L;
  uint32_t L_max; /* >= every L of the batch (<= 1024); ignored when L is NULL */
  uint32_t s_max; /* >= every s of the batch (<= 1024); ignored when s is NULL */
  dyg_update_result* results;
} dyg_batch_dev;

/*
 * Enqueue one batch on `stream` (a hipStream_t; NULL = the null stream)
 * without host synchronisation.  The call returns once the work is queued;
 * dyg_sync(ctx) waits for it and returns the batch status.  Inputs must stay
 * valid until then.
 */
int dyg_apply_batch_dev(dyg_ctx* ctx, const dyg_batch_dev* batch, void* stream);
int dyg_sync(dyg_ctx* ctx);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): dyg_apply_batch_dev
 * without any allocation.  Same arguments, same results and the same
 * asynchronous contract (dyg_sync reports the batch's status), but every
 * per-batch working buffer (hash tables, H-addition slots, phase-4 lists,
 * walker outcomes of the batched form, and the results when batch->results
 * is NULL) lives in one static device array of DYG_STATIC_SCRATCH_BYTES per
 * GPU, held by the library until the process ends, and the launch sequence
 * is never captured into a graph.  The caller still owns the inputs and the
 * results.
 * Limits and errors:
 *   DYG_E_TOO_LARGE  the batch's working memory exceeds the array (roughly
 *                    64 B per insertion plus 100 B per deletion and step of
 *                    its largest L, plus 24 B per walker in the batched form)
 *   DYG_E_BUSY       this context still has a batch in flight (call dyg_sync
 *                    first: completing a batch may grow a pool, which
 *                    allocates), or another context on the same GPU has a
 *                    static batch not yet synced (the array is shared by
 *                    every context on that GPU and keeps the last batch's
 *                    contents; the library clears what must start empty)
 * Calls that overlap on one GPU would race for the array; the library
 * refuses the second with DYG_E_BUSY instead.  dyg_sync and the pool growth
 * it may do are outside this no-allocation promise.
 */
#define DYG_STATIC_SCRATCH_BYTES (64ull << 20)
int dyg_apply_batch_dev_static(dyg_ctx* ctx, const dyg_batch_dev* batch, void* stream);

/*
 * Canonical edge list of H (Algorithm 1 output H(t)) or of G: u < v, sorted by
 * (u, v).  Two-call protocol: with cap < the edge count only *m is written.
 * u, v, w are host arrays of cap entries.
 */
int dyg_query_sparsifier(dyg_ctx* ctx, uint64_t cap, uint64_t* m, uint32_t* u, uint32_t* v,
                         double* w);
int dyg_query_graph(dyg_ctx* ctx, uint64_t cap, uint64_t* m, uint32_t* u, uint32_t* v,
                    double* w);

int dyg_stats(dyg_ctx* ctx, dyg_stats_t* out);

/*
 * Initial sparsifier H(0) of a graph G(0) -- the input Algorithm 1 starts
 * from (the experiments take it from GRASS, Sec. IV-A; here a spanning forest
 * plus off-tree edges of the same kind), computed on the current GPU:
 *   1. the maximum spanning forest of G(0), edges ordered by decreasing
 *      weight with ties to the smaller canonical index (a strict order, so
 *      the forest is unique; Boruvka rounds on the device);
 *   2. plus the n_extra edges outside the forest with the smallest 64-bit
 *      keys, ties to the smaller index, where the key of edge e is words 0-1
 *      (low first) of Philox-4x32-10 with key (seed low, seed high) and
 *      counter (e low, e high, 0, 0x53504152): a uniform sample without
 *      replacement (all of them if there are fewer).
 * Canonical edges are the pairs (u, v), u < v, of the CSR in ascending
 * (u, v) order; edge e is the e-th.  Arguments:
 *   n, rowptr, col, w   host CSR of G(0), as for dyg_init (same checks and
 *                       error codes; at most 2^32 - 1 edges)
 *   cap, m, h_u, h_v    host output: *m = the edge count of H(0); when cap >=
 *                       *m, h_u[i] < h_v[i] list H(0) in canonical order
 *                       (two-call protocol: cap = 0 asks for the count)
 * Allocates and frees its device memory within the call; synchronous.
 */
int dyg_initial_sparsifier(uint32_t n, const uint64_t* rowptr, const uint32_t* col,
                           const double* w, uint64_t n_extra, uint64_t seed, uint64_t cap,
                           uint64_t* m, uint32_t* h_u, uint32_t* h_v);

/* Launch schedule of the batched form (results never depend on it).
 * Defaults: walk_blocks_per_cu 8, refill_min 1, updates_per_wave 4,
 * tail_lanes 8, lockstep 0. */
typedef struct {
  uint32_t walk_blocks_per_cu; /* persistent walk grid = CUs x this (1..64)       */
  uint32_t refill_min;         /* idle lanes of a wavefront that trigger a refill
                                  from its item pool (1..64)                       */
  uint32_t updates_per_wave;   /* 0: one persistent work queue over every walker of
                                  the launch; 1..8: each wavefront walks the walkers
                                  of this many consecutive updates, a lane whose
                                  walker stops taking the next one of that range   */
  uint32_t tail_lanes;         /* 0: off.  1..64: head/tail schedule (single
                                  contexts): a head wavefront per update walks its
                                  walkers in lockstep until at most this many (and
                                  at most a quarter of them) still walk, then the
                                  tail walk packs those of updates_per_wave (at
                                  least 1) consecutive updates per wavefront      */
  uint32_t lockstep;           /* 1: single contexts walk one wavefront per update,
                                  lanes in lockstep, each update decided inside
                                  the walk kernel (the plain form's walk, inside
                                  the batched form's captured launch sequence);
                                  the fields above then apply to serving only    */
  uint32_t reserved[3];
} dyg_tuning;

int dyg_get_tuning(dyg_ctx* ctx, dyg_tuning* out);
int dyg_set_tuning(dyg_ctx* ctx, const dyg_tuning* t); /* INVALID_ARG if out of range */

/* Rewrite both pools without tombstones, with fresh slack (also done
 * automatically when a pool runs short). */
int dyg_compact(dyg_ctx* ctx);

/* Size the per-batch device buffers (staging, hash tables, H-addition slots,
 * per-walker records) for batches of up to max_ins insertions and max_del
 * deletions with at most max_s walkers and max_L steps per update, so that
 * later batches within these bounds allocate nothing.  Optional: buffers
 * otherwise grow on demand (a growth frees device memory, which waits for
 * the device).  INVALID_ARG beyond DYG_MAX_WALKERS / DYG_MAX_STEPS or 2^30
 * updates; NOMEM if the device cannot hold them. */
int dyg_reserve(dyg_ctx* ctx, uint64_t max_ins, uint64_t max_del, uint32_t max_s,
                uint32_t max_L);

/*
 * Consistency check of the device state (for tests and failure detection):
 * every segment sorted with unique neighbour ids inside its slots and the
 * pool, segments disjoint, the tombstone count of each row exact, the weight
 * prefix of every segment longer than 64 exact, G and H symmetric, H a
 * subgraph of G with equal weights.  Returns DYG_OK, or DYG_E_DEVICE with a
 * description of the first violation in msg (NUL-terminated, msg_len bytes).
 */
int dyg_check_state(dyg_ctx* ctx, char* msg, uint64_t msg_len);

void dyg_destroy(dyg_ctx* ctx);
const char* dyg_error_string(int code);

/*
 * Serving: one process keeps many graphs' G and H resident and applies update
 * batches as they arrive.  Batches of one graph are sequential (a batch reads
 * the state its predecessor left); batches of different graphs are
 * independent.  Each round admits the oldest waiting batches of graphs that
 * have none in flight, up to max_fused of them and within mem_budget bytes of
 * batch working memory, and runs them as one fused launch sequence (one
 * persistent walk launch over all their walkers).  Up to max_inflight rounds
 * run at once on separate streams, so batches that arrive while others are on
 * the GPU start as soon as slots and memory free up.  A batch's results are
 * bit-identical to applying it alone with dyg_apply_batch.
 */
typedef struct dyg_server dyg_server;

typedef struct {
  uint64_t mem_budget;   /* bytes of batch working memory held by rounds in flight   */
  uint32_t max_fused;    /* batches per round, 1..64                                  */
  uint32_t max_inflight; /* rounds in flight, 1..8                                    */
  uint32_t walk_blocks_per_cu; /* persistent walk grid per round, 1..64              */
  uint32_t reserved[3];
} dyg_server_params;

typedef struct {
  uint64_t request_id;
  uint32_t graph_id;
  int32_t status;        /* DYG_OK or the batch's error (state of that graph unchanged) */
  uint64_t n_updates;
  double t_submit;       /* seconds on the server's monotonic clock                  */
  double t_start;        /* round launched                                           */
  double t_done;         /* round observed complete                                  */
} dyg_request_done;

void dyg_server_default_params(dyg_server_params* p);
int dyg_server_create(dyg_server** out, const dyg_server_params* p);
/* Register a context (not owned; it must outlive the server and must not be
 * used directly while the server holds work for it). */
int dyg_server_add_graph(dyg_server* s, dyg_ctx* ctx, uint32_t* graph_id);
/* Queue a batch (host arrays copied at the call).  results: NULL or n_ins+n_del
 * records filled by the time the request is reported done. */
int dyg_server_submit(dyg_server* s, uint32_t graph_id, uint64_t n_ins, const uint32_t* iu,
                      const uint32_t* iv, const double* iw, uint64_t n_del, const uint32_t* du,
                      const uint32_t* dv, dyg_update_result* results, uint64_t* request_id);
/* Retire finished rounds, admit and launch new ones; never blocks on the GPU.
 * Writes up to cap finished requests to done and their number to *n_done. */
int dyg_server_poll(dyg_server* s, dyg_request_done* done, uint32_t cap, uint32_t* n_done);
/* Number of requests submitted but not yet reported by dyg_server_poll. */
uint64_t dyg_server_pending(const dyg_server* s);
double dyg_server_now(const dyg_server* s);
void dyg_server_destroy(dyg_server* s);

#ifdef __cplusplus
}
#endif

#endif /* DYGRASS_H */
