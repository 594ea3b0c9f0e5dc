/*
 * dyg_oracle.c -- plain, slow CPU oracle for the dyGRASS batched walk path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the HIP
 * library: every formula below is written out again from the paper
 * (Yuan, Aghdaei, Feng, "dyGRASS: Dynamic Spectral Graph Sparsification via
 * Localized Random Walks on GPUs", arXiv 2505.02741) and, for the random
 * numbers, from Salmon, Moraes, Dror and Shaw, "Parallel Random Numbers: As
 * Easy as 1, 2, 3" (SC'11).
 *
 * Data structures are deliberately naive: one sorted, malloc'd neighbour array
 * per vertex, insertions and deletions by memmove.  Walk trajectories are kept
 * whole, so the minimum-resistance path of a deletion is read back from the
 * stored trajectory rather than replayed.
 *
 * Floating point: the only FP operations are 1/w, w/w_ref*2^Q (host, once per
 * edge), R += r (strictly sequential per walker) and w*R > K.  Build with
 * -ffp-contract=off and without fast-math.
 *
 * Readings of what the paper leaves open:
 *  - neighbour choice is weight-biased, P(c) proportional to w(x,c), through
 *    integer weights qw = round-half-even(w / w_ref * 2^Q) and an exact
 *    integer cumulative search in ascending neighbour order; the 64-bit random
 *    number r picks target = floor(r * total / 2^64) and the first neighbour
 *    whose running sum exceeds target;
 *  - random numbers are Philox-4x32-10 keyed by the seed, counter
 *    (t/2, walker, uid), one block serving two steps;
 *  - a walker entering a vertex whose only neighbour is the previous one stops
 *    (the leaf condition of Sec. III-B); an optional policy steps back instead;
 *  - when the arriving step both reaches q and makes w*R exceed K, the walker
 *    misses: q must be reached within K; equality is within;
 *  - all walkers start at the first endpoint as given;
 *  - deletions walk only when the edge is in H (Sec. III-C, Algorithm 1);
 *  - batch order: deletions leave G and H first, then every walk reads that
 *    snapshot, then insertions, accepted edges and recovered edges are added;
 *  - the recovered path is the winner's edges in path order, first
 *    occurrence, without loop erasure, those not in H; the winner is the
 *    hitting walker of least R, ties to the lower walker index (a hit whose
 *    sum overflowed to +inf still counts: with every hit at +inf the first
 *    hitting walker wins);
 *  - a weight must be positive and finite with a finite 1/w;
 *  - with no hit, per endpoint the least-resistance G edge not in H (ties to
 *    the smaller neighbour id) is recovered, a reading of the local fallback
 *    of Sec. III-C.  The paper gives no rule to check this reading against;
 *    the tests pin the reading itself on hand-computed cases.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Error codes (kept equal by name and value to the library's, the tests    */
/* compare them; the numbers are restated here, not included).              */
enum {
  ORC_OK = 0,
  ORC_INVALID_ARG = -1,
  ORC_SELF_LOOP = -2,
  ORC_VERTEX_RANGE = -3,
  ORC_BAD_WEIGHT = -4,
  ORC_EDGE_EXISTS = -5,
  ORC_EDGE_MISSING = -6,
  ORC_DUPLICATE_IN_BATCH = -7,
  ORC_H_NOT_SUBSET = -8,
  ORC_NOMEM = -9
};

/* Variants (all off by default):
 *  BOTH_ENDS    walker k starts at the second endpoint and aims at the first
 *               when k is odd (Sec. III-C lets deletion walkers start at
 *               either endpoint; insertions alike);
 *  LOOP_ERASED  a hitting deletion recovers the edges of the chronological
 *               loop erasure of the winner's path (not in H) instead of
 *               every traversed edge;
 *  TWO_STAGE    the batch's deletion walks and their recoveries come first
 *               and enter H before the insertion walks, which then read the
 *               repaired H (the updates stay deferred to the batch end
 *               otherwise, Sec. III-F). */
#define ORC_VAR_BOTH_ENDS 1
#define ORC_VAR_LOOP_ERASED 2
#define ORC_VAR_TWO_STAGE 4

#define ORC_MAX_WALKERS 1024u
#define ORC_MAX_STEPS 1024u

/* ------------------------------------------------------------------------ */
/* Philox-4xW-10 (SC'11, Sec. 4).  One round maps counter (c0,c1,c2,c3) with */
/* round key (k0,k1) to (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1,        */
/* lo(M0*c0)); the key is bumped by the Weyl constants between rounds.       */

static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, c[0], &hi0, &lo0);
    mulhilo32(M1, c[2], &hi1, &lo1);
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    uint32_t n3 = lo0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
  }
  memcpy(out, c, sizeof c);
}

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2],
                       uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c[0], &hi0, &lo0);
    mulhilo64(M1, c[2], &hi1, &lo1);
    uint64_t n0 = hi1 ^ c[1] ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c[3] ^ k1;
    uint64_t n3 = lo0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
  }
  memcpy(out, c, sizeof c);
}

/* The 64-bit random number a walker draws at step t.  Counter words are     */
/* (t/2, walker, uid low, uid high), key words (seed low, seed high); even   */
/* steps take output words 0,1 and odd steps words 2,3 (low word first).     */
uint64_t orc_step_random(uint64_t seed, uint64_t uid, uint32_t walker,
                         uint32_t t) {
  uint32_t ctr[4] = {t >> 1, walker, (uint32_t)uid, (uint32_t)(uid >> 32)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  orc_philox4x32_10(ctr, key, x);
  uint32_t lo = x[2 * (t & 1u)], hi = x[2 * (t & 1u) + 1];
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

/* Quantised weight used for the weight-biased neighbour choice:             */
/* round-half-even(w / w_ref * 2^Q), clamped to [1, 2^32-1].                 */
uint32_t orc_quantize(double w, double w_ref, int Q) {
  double y = nearbyint((w / w_ref) * ldexp(1.0, Q));
  if (!(y >= 1.0)) return 1u;
  if (y > 4294967295.0) return 4294967295u;
  return (uint32_t)y;
}

/* ------------------------------------------------------------------------ */
/* Graph: per-vertex sorted neighbour arrays.                               */

typedef struct {
  uint32_t nbr;
  uint32_t qw;
  double w;
  double r; /* 1/w */
} oent;

typedef struct {
  oent *e;
  uint32_t len, cap;
} orow;

typedef struct {
  uint32_t n;
  orow *rows;
} ograph;

static int og_init(ograph *g, uint32_t n) {
  g->n = n;
  g->rows = (orow *)calloc(n ? n : 1, sizeof(orow));
  return g->rows ? 0 : -1;
}

static void og_free(ograph *g) {
  if (!g->rows) return;
  for (uint32_t i = 0; i < g->n; ++i) free(g->rows[i].e);
  free(g->rows);
  g->rows = NULL;
}

/* index of nbr v in row u, or -1 */
static long og_find(const ograph *g, uint32_t u, uint32_t v) {
  const orow *r = &g->rows[u];
  long lo = 0, hi = (long)r->len - 1;
  while (lo <= hi) {
    long mid = (lo + hi) / 2;
    if (r->e[mid].nbr == v) return mid;
    if (r->e[mid].nbr < v) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

static int og_has(const ograph *g, uint32_t u, uint32_t v) {
  return og_find(g, u, v) >= 0;
}

static int og_add_half(ograph *g, uint32_t u, const oent *x) {
  orow *r = &g->rows[u];
  if (r->len == r->cap) {
    uint32_t nc = r->cap ? 2 * r->cap : 4;
    oent *ne = (oent *)realloc(r->e, (size_t)nc * sizeof(oent));
    if (!ne) return -1;
    r->e = ne;
    r->cap = nc;
  }
  /* first position whose neighbour id exceeds the new one */
  uint32_t lo = 0, hi = r->len;
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (r->e[mid].nbr < x->nbr) lo = mid + 1;
    else hi = mid;
  }
  uint32_t pos = lo;
  memmove(&r->e[pos + 1], &r->e[pos], (size_t)(r->len - pos) * sizeof(oent));
  r->e[pos] = *x;
  r->len++;
  return 0;
}

static int og_add(ograph *g, uint32_t u, uint32_t v, double w, double r,
                  uint32_t qw) {
  oent a = {v, qw, w, r}, b = {u, qw, w, r};
  if (og_add_half(g, u, &a)) return -1;
  if (og_add_half(g, v, &b)) return -1;
  return 0;
}

static void og_remove_half(ograph *g, uint32_t u, uint32_t v) {
  long i = og_find(g, u, v);
  if (i < 0) return;
  orow *r = &g->rows[u];
  memmove(&r->e[i], &r->e[i + 1], (size_t)(r->len - (uint32_t)i - 1) * sizeof(oent));
  r->len--;
}

static void og_remove(ograph *g, uint32_t u, uint32_t v) {
  og_remove_half(g, u, v);
  og_remove_half(g, v, u);
}

/* ------------------------------------------------------------------------ */
/* One non-backtracking, weight-biased walker (Sec. III-B; Sec. III-C for    */
/* the deletion mode, Sec. III-F for the per-step procedure).               */

typedef struct {
  uint8_t hit;
  uint16_t steps;
  uint32_t end;
  double R;
  uint64_t bytes; /* gathered bytes the steps must read (measurement only) */
} owalk;

/* Bytes a step must read at a vertex with d live neighbours: offset and
 * degree (8), an (id, weight) pair per neighbour (8 each), the chosen edge's
 * resistance (8); above 64 neighbours a cumulative-weight binary search:
 * 32 plus 12 per halving, ceil(log2 d) halvings. */
static uint64_t o_step_bytes(uint32_t d) {
  if (d <= 64) return 16u + 8u * (uint64_t)d;
  uint32_t halvings = 0;
  while ((1ull << halvings) < d) halvings++;
  return 32u + 12u * (uint64_t)halvings;
}

/* traj (optional) receives x_0..x_steps (steps+1 vertices). */
static void o_walk_one(const ograph *X, uint32_t p, uint32_t q, int has_K,
                       double w_pq, double K, uint32_t L, uint64_t seed,
                       uint64_t uid, uint32_t walker, int bounce, owalk *res,
                       uint32_t *traj) {
  uint32_t x = p;
  long prev = -1; /* no previous vertex before the first step */
  double R = 0.0;
  uint8_t hit = 0;
  uint32_t steps = 0;
  uint64_t bytes = 0;
  if (traj) traj[0] = p;
  for (uint32_t t = 0; t < L; ++t) {
    const orow *row = &X->rows[x];
    /* candidates: every neighbour except the vertex we just came from */
    uint64_t tot = 0;
    for (uint32_t i = 0; i < row->len; ++i)
      if ((long)row->e[i].nbr != prev) tot += row->e[i].qw;
    int forced_back = 0;
    if (tot == 0) {
      /* leaf / dead end: stop, or (optional policy) step back */
      if (bounce && prev >= 0) forced_back = 1;
      else break;
    }
    uint32_t chosen = 0;
    double r = 0.0;
    if (forced_back) {
      long i = og_find(X, x, (uint32_t)prev);
      chosen = (uint32_t)prev;
      r = row->e[i].r;
    } else {
      uint64_t rnd = orc_step_random(seed, uid, walker, t);
      uint64_t target =
          (uint64_t)(((unsigned __int128)rnd * (unsigned __int128)tot) >> 64);
      uint64_t run = 0;
      int found = 0;
      for (uint32_t i = 0; i < row->len; ++i) {
        if ((long)row->e[i].nbr == prev) continue;
        run += row->e[i].qw;
        if (run > target) {
          chosen = row->e[i].nbr;
          r = row->e[i].r;
          found = 1;
          break;
        }
      }
      if (!found) abort(); /* impossible: target < tot */
    }
    bytes += o_step_bytes(row->len);
    R = R + r;
    prev = (long)x;
    x = chosen;
    steps++;
    if (traj) traj[steps] = x;
    if (has_K && w_pq * R > K) break; /* distortion threshold exceeded */
    if (x == q) {
      hit = 1;
      break;
    }
  }
  res->hit = hit;
  res->steps = (uint16_t)steps;
  res->end = x;
  res->R = R;
  res->bytes = bytes;
}

/* ------------------------------------------------------------------------ */
/* Standalone walk on a static graph given as a symmetric CSR (used by the   */
/* pins on tiny graphs).  rowptr has n+1 entries; col/w hold both directions */
/* of every edge, each row sorted ascending.                                */

int orc_walk_csr(uint32_t n, const uint64_t *rowptr, const uint32_t *col,
                 const double *w, double w_ref, int Q, uint32_t p, uint32_t q,
                 int has_K, double w_pq, double K, uint32_t s, uint32_t L,
                 uint64_t seed, uint64_t uid, int bounce, uint8_t *hit,
                 uint16_t *steps, uint32_t *end, double *R, uint32_t *traj) {
  ograph g;
  if (p >= n || q >= n) return ORC_VERTEX_RANGE;
  if (og_init(&g, n)) return ORC_NOMEM;
  for (uint32_t u = 0; u < n; ++u) {
    for (uint64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
      oent e = {col[k], orc_quantize(w[k], w_ref, Q), w[k], 1.0 / w[k]};
      if (og_add_half(&g, u, &e)) {
        og_free(&g);
        return ORC_NOMEM;
      }
    }
  }
  for (uint32_t k = 0; k < s; ++k) {
    owalk res;
    o_walk_one(&g, p, q, has_K, w_pq, K, L, seed, uid, k, bounce, &res,
               traj ? traj + (size_t)k * (L + 1) : NULL);
    hit[k] = res.hit;
    steps[k] = res.steps;
    end[k] = res.end;
    R[k] = res.R;
  }
  og_free(&g);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Full oracle state and Algorithm 1 with batch-deferred updates (Sec. III-F: */
/* the GPU version applies the updates of a batch at the end of the batch).  */

typedef struct {
  uint32_t n;
  ograph G, H;
  uint64_t seed;
  double K;
  int has_K;
  uint16_t s_def, L_def;
  int Q;
  double w_ref;
  int bounce;
  int variant; /* ORC_VAR_* bits: the alternatives of Sec. III-C and III-F */
  uint64_t uid_base;
  uint64_t steps_total;     /* walker steps taken since creation */
  uint64_t alg_bytes_total; /* bytes those steps must gather */
  /* edges each deletion of the last batch recovered into H, in the order
   * they were taken (path order, or the endpoints' fallback edges) */
  uint64_t last_ndel;
  uint64_t *last_rofs; /* [last_ndel + 1] */
  uint32_t *last_nrec; /* [last_ndel] */
  uint32_t *last_rec_a, *last_rec_b;
} oracle_t;

/* A usable weight is positive and finite with a finite resistance 1/w
 * (a subnormal weight's 1/w overflows). */
static int weight_ok(double w) { return w > 0.0 && !isinf(w) && !isinf(1.0 / w); }

static uint64_t ekey(uint32_t u, uint32_t v) {
  uint32_t a = u < v ? u : v, b = u < v ? v : u;
  return ((uint64_t)a << 32) | b;
}

typedef struct {
  uint64_t key;
  uint64_t idx;
} okeyidx;

static int cmp_keyidx(const void *a, const void *b) {
  const okeyidx *x = (const okeyidx *)a, *y = (const okeyidx *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

/* dup[i] = 1 iff an earlier entry of u/v (lower index) is the same edge */
static int o_mark_repeats(uint64_t cnt, const uint32_t *u, const uint32_t *v,
                          uint8_t *dup) {
  okeyidx *a = (okeyidx *)malloc((cnt + 1) * sizeof(okeyidx));
  if (!a) return -1;
  for (uint64_t i = 0; i < cnt; ++i) {
    a[i].key = ekey(u[i], v[i]);
    a[i].idx = i;
    dup[i] = 0;
  }
  qsort(a, cnt, sizeof(okeyidx), cmp_keyidx);
  for (uint64_t i = 1; i < cnt; ++i)
    if (a[i].key == a[i - 1].key) dup[a[i].idx] = 1;
  free(a);
  return 0;
}

/* params: seed, K (+inf => no threshold), s_def, L_def, Q, w_ref (0 => max
 * weight of G0), dead_end (0 terminate, 1 bounce), uid_base. */
oracle_t *orc_create(uint32_t n, const uint64_t *rowptr, const uint32_t *col,
                     const double *w, uint64_t h_m, const uint32_t *hu,
                     const uint32_t *hv, uint64_t seed, double K,
                     uint32_t s_def, uint32_t L_def, int Q, double w_ref,
                     int dead_end, uint64_t uid_base, int *err) {
  *err = ORC_OK;
  if (n == 0 || Q < 1 || Q > 31 || s_def > ORC_MAX_WALKERS ||
      L_def > ORC_MAX_STEPS || dead_end < 0 || dead_end > 1 || isnan(K) ||
      !(w_ref >= 0.0) || isinf(w_ref)) {
    *err = ORC_INVALID_ARG;
    return NULL;
  }
  /* validate the CSR: symmetric, sorted, no loops, positive finite weights */
  if (rowptr[0] != 0) {
    *err = ORC_INVALID_ARG;
    return NULL;
  }
  double wmax = 0.0;
  for (uint32_t u = 0; u < n; ++u) {
    if (rowptr[u + 1] < rowptr[u]) {
      *err = ORC_INVALID_ARG;
      return NULL;
    }
    for (uint64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
      if (col[k] >= n) {
        *err = ORC_VERTEX_RANGE;
        return NULL;
      }
      if (col[k] == u) {
        *err = ORC_SELF_LOOP;
        return NULL;
      }
      if (!weight_ok(w[k])) {
        *err = ORC_BAD_WEIGHT;
        return NULL;
      }
      if (k > rowptr[u] && col[k] <= col[k - 1]) {
        *err = ORC_INVALID_ARG; /* unsorted or repeated neighbour */
        return NULL;
      }
      if (w[k] > wmax) wmax = w[k];
    }
  }
  oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
  if (!o || og_init(&o->G, n) || og_init(&o->H, n)) {
    if (o) {
      og_free(&o->G);
      og_free(&o->H);
      free(o);
    }
    *err = ORC_NOMEM;
    return NULL;
  }
  o->n = n;
  o->seed = seed;
  o->has_K = !(isinf(K) && K > 0); /* K = +inf disables the threshold */
  o->K = K;
  o->s_def = (uint16_t)s_def;
  o->L_def = (uint16_t)L_def;
  o->Q = Q;
  o->w_ref = (w_ref > 0.0) ? w_ref : (wmax > 0.0 ? wmax : 1.0);
  o->bounce = dead_end;
  o->variant = 0;
  o->uid_base = uid_base;
  for (uint32_t u = 0; u < n; ++u) {
    uint32_t d = (uint32_t)(rowptr[u + 1] - rowptr[u]);
    orow *row = &o->G.rows[u];
    row->e = (oent *)malloc((size_t)(d ? d : 1) * sizeof(oent));
    row->cap = d ? d : 1;
    row->len = d;
    for (uint32_t i = 0; i < d; ++i) {
      uint64_t k = rowptr[u] + i;
      oent e = {col[k], orc_quantize(w[k], o->w_ref, Q), w[k], 1.0 / w[k]};
      row->e[i] = e;
    }
  }
  /* symmetry: every (u,v) must have (v,u) with the same weight */
  for (uint32_t u = 0; u < n; ++u) {
    for (uint32_t i = 0; i < o->G.rows[u].len; ++i) {
      const oent *e = &o->G.rows[u].e[i];
      long j = og_find(&o->G, e->nbr, u);
      if (j < 0 || o->G.rows[e->nbr].e[j].w != e->w) {
        *err = ORC_INVALID_ARG;
        og_free(&o->G);
        og_free(&o->H);
        free(o);
        return NULL;
      }
    }
  }
  /* sparsifier edges: must be distinct edges of G; copied with G's weight */
  for (uint64_t k = 0; k < h_m; ++k) {
    uint32_t a = hu[k], b = hv[k];
    int e = ORC_OK;
    if (a >= n || b >= n) e = ORC_VERTEX_RANGE;
    else if (a == b) e = ORC_SELF_LOOP;
    else if (!og_has(&o->G, a, b)) e = ORC_H_NOT_SUBSET;
    else if (og_has(&o->H, a, b)) e = ORC_DUPLICATE_IN_BATCH;
    if (e != ORC_OK) {
      *err = e;
      og_free(&o->G);
      og_free(&o->H);
      free(o);
      return NULL;
    }
    const oent *ge = &o->G.rows[a].e[og_find(&o->G, a, b)];
    og_add(&o->H, a, b, ge->w, ge->r, ge->qw);
  }
  return o;
}

static void o_free_last(oracle_t *o) {
  free(o->last_rofs);
  free(o->last_nrec);
  free(o->last_rec_a);
  free(o->last_rec_b);
  o->last_rofs = NULL;
  o->last_nrec = NULL;
  o->last_rec_a = o->last_rec_b = NULL;
  o->last_ndel = 0;
}

void orc_destroy(oracle_t *o) {
  if (!o) return;
  og_free(&o->G);
  og_free(&o->H);
  o_free_last(o);
  free(o);
}

/* Edges deletion j of the last successful batch recovered (path or
 * fallback), in the order taken: writes up to cap of them to a/b and
 * returns their number, or -1 if j is out of range. */
long orc_last_recovered(const oracle_t *o, uint64_t j, uint32_t cap, uint32_t *a,
                        uint32_t *b) {
  if (j >= o->last_ndel) return -1;
  uint32_t cnt = o->last_nrec[j];
  for (uint32_t z = 0; z < cnt && z < cap; ++z) {
    a[z] = o->last_rec_a[o->last_rofs[j] + z];
    b[z] = o->last_rec_b[o->last_rofs[j] + z];
  }
  return (long)cnt;
}

int orc_set_variant(oracle_t *o, int variant) {
  if (variant & ~(ORC_VAR_BOTH_ENDS | ORC_VAR_LOOP_ERASED | ORC_VAR_TWO_STAGE))
    return ORC_INVALID_ARG;
  o->variant = variant;
  return ORC_OK;
}

uint64_t orc_uid_base(const oracle_t *o) { return o->uid_base; }
uint64_t orc_steps_total(const oracle_t *o) { return o->steps_total; }
uint64_t orc_alg_bytes_total(const oracle_t *o) { return o->alg_bytes_total; }
double orc_w_ref(const oracle_t *o) { return o->w_ref; }

/* Threads of the loop over a batch's updates (a timing control: phase 2
 * reads only the batch snapshot, so results never depend on it).  k <= 0
 * leaves the count unchanged; returns the count now in use. */
int orc_set_threads(int k) {
  if (k > 0) omp_set_num_threads(k);
  return omp_get_max_threads();
}

/* Validation precedence: insertions in order (range, self loop, weight,
 * already in G, repeated in batch), then deletions in order (range, self
 * loop, not in G, repeated in batch), then per-update s and L bounds. */
static int o_validate(const oracle_t *o, uint64_t n_ins, const uint32_t *iu,
                      const uint32_t *iv, const double *iw, uint64_t n_del,
                      const uint32_t *du, const uint32_t *dv,
                      const uint16_t *s, const uint16_t *L) {
  uint8_t *dupi = (uint8_t *)malloc(n_ins + 1);
  uint8_t *dupd = (uint8_t *)malloc(n_del + 1);
  if (!dupi || !dupd || o_mark_repeats(n_ins, iu, iv, dupi) ||
      o_mark_repeats(n_del, du, dv, dupd)) {
    free(dupi);
    free(dupd);
    return ORC_NOMEM;
  }
  int err = ORC_OK;
  for (uint64_t i = 0; i < n_ins && err == ORC_OK; ++i) {
    if (iu[i] >= o->n || iv[i] >= o->n) err = ORC_VERTEX_RANGE;
    else if (iu[i] == iv[i]) err = ORC_SELF_LOOP;
    else if (!weight_ok(iw[i])) err = ORC_BAD_WEIGHT;
    else if (og_has(&o->G, iu[i], iv[i])) err = ORC_EDGE_EXISTS;
    else if (dupi[i]) err = ORC_DUPLICATE_IN_BATCH;
  }
  for (uint64_t j = 0; j < n_del && err == ORC_OK; ++j) {
    if (du[j] >= o->n || dv[j] >= o->n) err = ORC_VERTEX_RANGE;
    else if (du[j] == dv[j]) err = ORC_SELF_LOOP;
    else if (!og_has(&o->G, du[j], dv[j])) err = ORC_EDGE_MISSING;
    else if (dupd[j]) err = ORC_DUPLICATE_IN_BATCH;
  }
  for (uint64_t i = 0; i < n_ins + n_del && err == ORC_OK; ++i) {
    if (s && s[i] > ORC_MAX_WALKERS) err = ORC_INVALID_ARG;
    if (L && L[i] > ORC_MAX_STEPS) err = ORC_INVALID_ARG;
  }
  free(dupi);
  free(dupd);
  return err;
}

/*
 * One batch.  Per-update outputs (arrays of length n_ins+n_del, insertions
 * first, may be NULL): flag = accepted (insertion) / in H (deletion);
 * any_hit; winner (deletion, walker of the minimum (R, index) hit, 0xFFFF if
 * none); n_rec (deletion, edges recovered or taken by the fallback); steps
 * (sum over walkers); Rmin (+inf if no hit).
 * Per-walker outputs (optional, length sum of s over updates, in update
 * order; deletions whose edge is not in H report zero steps at u).
 */
/* Walks and decision of update i of the batch (phase 2), on the current
 * G and H; writes its results, its acceptance flag or recovered edges. */
static void o_update(oracle_t *o, uint64_t i, uint64_t n_ins, const uint32_t *iu,
                     const uint32_t *iv, const double *iw, const uint32_t *du,
                     const uint32_t *dv, const uint16_t *s, const uint16_t *L,
                     const uint8_t *inH, uint8_t *acc, const uint64_t *wofs,
                     const uint64_t *rofs, uint32_t *rec_a, uint32_t *rec_b, uint32_t *nrec,
                     uint8_t *flag, uint8_t *any_hit, uint16_t *winner, uint16_t *n_rec,
                     uint32_t *steps, double *Rmin, uint8_t *w_hit, uint16_t *w_steps,
                     uint32_t *w_end, double *w_R) {
  uint64_t uid = o->uid_base + i;
  uint32_t si = s ? s[i] : o->s_def;
  uint32_t Li = L ? L[i] : o->L_def;
  int is_ins = i < n_ins;
  uint64_t j = i - n_ins;
  uint32_t p = is_ins ? iu[i] : du[j];
  uint32_t q = is_ins ? iv[i] : dv[j];
  uint8_t fl = 0, anyh = 0;
  uint16_t win = 0xFFFF, nr = 0;
  uint32_t st = 0;
  uint64_t by = 0;
  double rmin = INFINITY;
  if (is_ins || inH[j]) {
    const ograph *X = is_ins ? &o->H : &o->G; /* H_mid / G_mid */
    uint32_t *traj = (uint32_t *)malloc((size_t)si * (Li + 1) * sizeof(uint32_t) + 4);
    owalk *res = (owalk *)malloc((size_t)si * sizeof(owalk) + 1);
    for (uint32_t k = 0; k < si; ++k) {
      /* odd walkers from the second endpoint towards the first (variant) */
      const int flip = (o->variant & ORC_VAR_BOTH_ENDS) && (k & 1u);
      o_walk_one(X, flip ? q : p, flip ? p : q, is_ins && o->has_K, is_ins ? iw[i] : 0.0,
                 o->K, Li, o->seed, uid, k, o->bounce, &res[k],
                 traj + (size_t)k * (Li + 1));
      st += res[k].steps;
      by += res[k].bytes;
      if (res[k].hit) {
        anyh = 1;
        /* minimum resistance over hitting walkers, ties to the lower index
         * (a sum that overflowed to +inf still names a walker) */
        if (win == 0xFFFF || res[k].R < rmin) {
          rmin = res[k].R;
          win = (uint16_t)k;
        }
      }
      if (w_hit) {
        w_hit[wofs[i] + k] = res[k].hit;
        w_steps[wofs[i] + k] = res[k].steps;
        w_end[wofs[i] + k] = res[k].end;
        w_R[wofs[i] + k] = res[k].R;
      }
    }
    if (is_ins) {
      fl = (uint8_t)!anyh; /* keep the new edge iff no walker reached q */
      acc[i] = fl;
    } else {
      fl = 1;
      uint32_t *ra = rec_a + rofs[j], *rb = rec_b + rofs[j];
      if (anyh) {
        /* edges of the winning path, first occurrence, not already in H;
         * with LOOP_ERASED the path is first loop-erased in time order:
         * a vertex met again cuts the loop back to its first visit */
        const uint32_t *path = traj + (size_t)win * (Li + 1);
        uint32_t plen = res[win].steps + 1;
        uint32_t *le = NULL;
        if (o->variant & ORC_VAR_LOOP_ERASED) {
          le = (uint32_t *)malloc(sizeof(uint32_t) * plen);
          uint32_t len = 0;
          for (uint32_t t = 0; t < plen; ++t) {
            uint32_t z = 0;
            while (z < len && le[z] != path[t]) ++z;
            if (z < len) len = z + 1;
            else le[len++] = path[t];
          }
          path = le;
          plen = len;
        }
        for (uint32_t t = 0; t + 1 < plen; ++t) {
          uint32_t a = path[t], b = path[t + 1];
          if (og_has(&o->H, a, b)) continue;
          int seen = 0;
          for (uint32_t z = 0; z < nr; ++z)
            if (ekey(ra[z], rb[z]) == ekey(a, b)) seen = 1;
          if (seen) continue;
          ra[nr] = a;
          rb[nr] = b;
          nr++;
        }
        free(le);
      } else {
        /* no hit: per endpoint, the least-resistance G edge not in H,
         * ties to the smaller neighbour id */
        uint32_t ends[2] = {p, q};
        for (int z = 0; z < 2; ++z) {
          const orow *row = &o->G.rows[ends[z]];
          long best = -1;
          for (uint32_t t = 0; t < row->len; ++t) {
            if (og_has(&o->H, ends[z], row->e[t].nbr)) continue;
            if (best < 0 || row->e[t].r < row->e[best].r) best = (long)t;
          }
          if (best >= 0) {
            ra[nr] = ends[z];
            rb[nr] = row->e[best].nbr;
            nr++;
          }
        }
      }
      nrec[j] = nr;
    }
    free(traj);
    free(res);
  } else if (w_hit) {
    for (uint32_t k = 0; k < si; ++k) {
      w_hit[wofs[i] + k] = 0;
      w_steps[wofs[i] + k] = 0;
      w_end[wofs[i] + k] = p;
      w_R[wofs[i] + k] = 0.0;
    }
  }
#pragma omp atomic
  o->steps_total += st;
#pragma omp atomic
  o->alg_bytes_total += by;
  if (flag) flag[i] = fl;
  if (any_hit) any_hit[i] = anyh;
  if (winner) winner[i] = win;
  if (n_rec) n_rec[i] = nr;
  if (steps) steps[i] = st;
  if (Rmin) Rmin[i] = rmin;
}

/* H += the recovered and fallback edges of the batch's deletions (a set
 * union; their weights are G's). */
static void o_add_recovered(oracle_t *o, uint64_t n_del, const uint64_t *rofs,
                            const uint32_t *rec_a, const uint32_t *rec_b,
                            const uint32_t *nrec) {
  for (uint64_t j = 0; j < n_del; ++j) {
    for (uint32_t z = 0; z < nrec[j]; ++z) {
      uint32_t a = rec_a[rofs[j] + z], b = rec_b[rofs[j] + z];
      if (og_has(&o->H, a, b)) continue;
      const oent *ge = &o->G.rows[a].e[og_find(&o->G, a, b)];
      og_add(&o->H, a, b, ge->w, ge->r, ge->qw);
    }
  }
}

int orc_apply_batch(oracle_t *o, uint64_t n_ins, const uint32_t *iu,
                    const uint32_t *iv, const double *iw, uint64_t n_del,
                    const uint32_t *du, const uint32_t *dv, const uint16_t *s,
                    const uint16_t *L, uint8_t *flag, uint8_t *any_hit,
                    uint16_t *winner, uint16_t *n_rec, uint32_t *steps,
                    double *Rmin, uint8_t *w_hit, uint16_t *w_steps,
                    uint32_t *w_end, double *w_R) {
  int err = o_validate(o, n_ins, iu, iv, iw, n_del, du, dv, s, L);
  if (err != ORC_OK) return err;
  const uint64_t nu = n_ins + n_del;
  uint64_t *wofs = (uint64_t *)malloc((nu + 1) * sizeof(uint64_t));
  uint8_t *inH = (uint8_t *)calloc(n_del + 1, 1);
  uint8_t *acc = (uint8_t *)calloc(n_ins + 1, 1);
  if (!wofs || !inH || !acc) {
    free(wofs);
    free(inH);
    free(acc);
    return ORC_NOMEM;
  }
  wofs[0] = 0;
  for (uint64_t i = 0; i < nu; ++i)
    wofs[i + 1] = wofs[i] + (s ? s[i] : o->s_def);

  /* Phase 1: membership of each deleted edge in H; remove D from G and H. */
  for (uint64_t j = 0; j < n_del; ++j) inH[j] = (uint8_t)og_has(&o->H, du[j], dv[j]);
  for (uint64_t j = 0; j < n_del; ++j) {
    og_remove(&o->G, du[j], dv[j]);
    if (inH[j]) og_remove(&o->H, du[j], dv[j]);
  }

  /* recovered edges per deletion: at most L path edges or 2 fallback edges */
  uint64_t *rofs = (uint64_t *)malloc((n_del + 1) * sizeof(uint64_t));
  rofs[0] = 0;
  for (uint64_t j = 0; j < n_del; ++j) {
    uint32_t Lj = L ? L[n_ins + j] : o->L_def;
    rofs[j + 1] = rofs[j] + (Lj > 2 ? Lj : 2);
  }
  uint32_t *rec_a = (uint32_t *)malloc((rofs[n_del] + 1) * sizeof(uint32_t));
  uint32_t *rec_b = (uint32_t *)malloc((rofs[n_del] + 1) * sizeof(uint32_t));
  uint32_t *nrec = (uint32_t *)calloc(n_del + 1, sizeof(uint32_t));

  /* Phase 2: walks, deletions first.  Within a stage every update reads
   * only that stage's snapshot, so the loop order is immaterial.  Single
   * stage: the insertions also read H_mid.  TWO_STAGE: the deletions'
   * recovered edges enter H before the insertion walks. */
  const int two = o->variant & ORC_VAR_TWO_STAGE;
#pragma omp parallel for schedule(dynamic, 16)
  for (long long ii = (long long)n_ins; ii < (long long)nu; ++ii)
    o_update(o, (uint64_t)ii, n_ins, iu, iv, iw, du, dv, s, L, inH, acc, wofs, rofs, rec_a,
             rec_b, nrec, flag, any_hit, winner, n_rec, steps, Rmin, w_hit, w_steps, w_end, w_R);
  if (two) o_add_recovered(o, n_del, rofs, rec_a, rec_b, nrec);
#pragma omp parallel for schedule(dynamic, 16)
  for (long long ii = 0; ii < (long long)n_ins; ++ii)
    o_update(o, (uint64_t)ii, n_ins, iu, iv, iw, du, dv, s, L, inH, acc, wofs, rofs, rec_a,
             rec_b, nrec, flag, any_hit, winner, n_rec, steps, Rmin, w_hit, w_steps, w_end, w_R);

  /* Phase 4: G += I; H += accepted insertions, recovered and fallback edges
   * (a set union: an edge already present is not added twice). */
  for (uint64_t i = 0; i < n_ins; ++i) {
    double r = 1.0 / iw[i];
    uint32_t qw = orc_quantize(iw[i], o->w_ref, o->Q);
    og_add(&o->G, iu[i], iv[i], iw[i], r, qw);
    if (acc[i]) og_add(&o->H, iu[i], iv[i], iw[i], r, qw);
  }
  if (!two) o_add_recovered(o, n_del, rofs, rec_a, rec_b, nrec);
  o->uid_base += nu;
  o_free_last(o);
  o->last_ndel = n_del;
  o->last_rofs = rofs;
  o->last_nrec = nrec;
  o->last_rec_a = rec_a;
  o->last_rec_b = rec_b;
  free(wofs);
  free(inH);
  free(acc);
  return ORC_OK;
}

/* Canonical edge list (u < v, sorted by (u, v)) of G (which=0) or H (1).
 * With cap smaller than the edge count only *m is written. */
int orc_query(const oracle_t *o, int which, uint64_t cap, uint64_t *m,
              uint32_t *u, uint32_t *v, double *w) {
  const ograph *g = which ? &o->H : &o->G;
  uint64_t cnt = 0;
  for (uint32_t a = 0; a < g->n; ++a)
    for (uint32_t i = 0; i < g->rows[a].len; ++i)
      if (g->rows[a].e[i].nbr > a) cnt++;
  *m = cnt;
  if (cap < cnt) return ORC_OK;
  uint64_t k = 0;
  for (uint32_t a = 0; a < g->n; ++a)
    for (uint32_t i = 0; i < g->rows[a].len; ++i)
      if (g->rows[a].e[i].nbr > a) {
        u[k] = a;
        v[k] = g->rows[a].e[i].nbr;
        w[k] = g->rows[a].e[i].w;
        k++;
      }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Initial sparsifier (the step before the update path: H(0) of Algorithm  */
/* 1, built here the way the experiments' synthetic stand-ins build it).    */
/* Edges are the pairs (u,v), u < v, of the symmetric CSR in ascending      */
/* (u,v) order; edge e is the e-th of them.                                 */
/*  1. Maximum spanning forest: Kruskal over the edges by decreasing        */
/*     weight, ties to the smaller edge index; an edge is kept iff its ends */
/*     are in different components so far.  The order is strict, so the    */
/*     forest is unique.                                                    */
/*  2. Off-tree sample: of the edges left out, the n_extra with the         */
/*     smallest 64-bit key, ties to the smaller edge index, where key(e) is */
/*     output words 0-1 of Philox-4x32-10 with key (seed low, seed high)    */
/*     and counter (e low, e high, 0, 0x53504152); i.i.d. uniform keys make */
/*     this a uniform sample without replacement.                           */
/* in_h[e] = 1 for the edges of H(0).  Returns the edge count of H(0), or a */
/* negative error code.                                                     */

typedef struct {
  double w;
  uint64_t e;
} o_wedge;

static int cmp_wdesc_idx(const void *a, const void *b) {
  const o_wedge *x = (const o_wedge *)a, *y = (const o_wedge *)b;
  if (x->w != y->w) return x->w > y->w ? -1 : 1;
  return x->e < y->e ? -1 : (x->e > y->e ? 1 : 0);
}

typedef struct {
  uint64_t key;
  uint64_t e;
} o_kedge;

static int cmp_key_idx(const void *a, const void *b) {
  const o_kedge *x = (const o_kedge *)a, *y = (const o_kedge *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->e < y->e ? -1 : (x->e > y->e ? 1 : 0);
}

static uint32_t uf_find(uint32_t *parent, uint32_t x) {
  uint32_t r = x;
  while (parent[r] != r) r = parent[r];
  while (parent[x] != r) {
    uint32_t nx = parent[x];
    parent[x] = r;
    x = nx;
  }
  return r;
}

uint64_t orc_sample_key(uint64_t seed, uint64_t e) {
  uint32_t ctr[4] = {(uint32_t)e, (uint32_t)(e >> 32), 0u, 0x53504152u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  orc_philox4x32_10(ctr, key, x);
  return (uint64_t)x[0] | ((uint64_t)x[1] << 32);
}

long orc_initial_sparsifier(uint32_t n, const uint64_t *rowptr, const uint32_t *col,
                            const double *w, uint64_t n_extra, uint64_t seed,
                            uint8_t *in_h) {
  if (!rowptr || (rowptr[n] && (!col || !w))) return ORC_INVALID_ARG;
  uint64_t m = 0;
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t k = rowptr[u]; k < rowptr[u + 1]; ++k)
      if (col[k] > u) ++m;
  uint32_t *eu = malloc(sizeof(uint32_t) * (m ? m : 1));
  uint32_t *ev = malloc(sizeof(uint32_t) * (m ? m : 1));
  o_wedge *order = malloc(sizeof(o_wedge) * (m ? m : 1));
  uint32_t *parent = malloc(sizeof(uint32_t) * (n ? n : 1));
  if (!eu || !ev || !order || !parent) {
    free(eu); free(ev); free(order); free(parent);
    return ORC_NOMEM;
  }
  uint64_t e = 0;
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t k = rowptr[u]; k < rowptr[u + 1]; ++k)
      if (col[k] > u) {
        eu[e] = u;
        ev[e] = col[k];
        order[e].w = w[k];
        order[e].e = e;
        ++e;
      }
  qsort(order, m, sizeof(o_wedge), cmp_wdesc_idx);
  for (uint32_t x = 0; x < n; ++x) parent[x] = x;
  memset(in_h, 0, m);
  long count = 0;
  for (uint64_t i = 0; i < m; ++i) {
    const uint64_t f = order[i].e;
    const uint32_t a = uf_find(parent, eu[f]), b = uf_find(parent, ev[f]);
    if (a == b) continue;
    parent[a] = b;
    in_h[f] = 1;
    ++count;
  }
  free(order);
  free(parent);
  o_kedge *off = malloc(sizeof(o_kedge) * ((m - (uint64_t)count) ? (m - (uint64_t)count) : 1));
  if (!off) {
    free(eu); free(ev);
    return ORC_NOMEM;
  }
  uint64_t n_off = 0;
  for (uint64_t f = 0; f < m; ++f)
    if (!in_h[f]) {
      off[n_off].key = orc_sample_key(seed, f);
      off[n_off].e = f;
      ++n_off;
    }
  qsort(off, n_off, sizeof(o_kedge), cmp_key_idx);
  for (uint64_t i = 0; i < n_off && i < n_extra; ++i) {
    in_h[off[i].e] = 1;
    ++count;
  }
  free(off);
  free(eu);
  free(ev);
  return count;
}
