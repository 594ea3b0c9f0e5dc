"""Literal oracle: a second, pure-Python reading of the dyGRASS batch update.

TEST INFRASTRUCTURE ONLY.  Only ``tests/`` imports this module.  It is the
second of the two oracles: the tests run it beside the C oracle
(``dyg_oracle.c``) on the same seeded streams and require the two to agree on
every output, integers and resistance sums bit for bit.  The two share no
code: this file has its own Philox, its own graph structure (a dict of
neighbour dicts), and its own walk, decision and batch logic.  It never
calls the ctypes wrappers of this package, and it uses nothing from the
product library.  It is slow (pure Python loops) and meant for graphs of a
few thousand vertices.

The method (Yuan, Aghdaei, Feng, "dyGRASS: Dynamic Spectral Graph
Sparsification via Localized Random Walks on GPUs", arXiv 2505.02741), in the
order Algorithm 1 takes its steps, with the batch deferral of Sec. III-F:

1. a deleted edge leaves G, and H when it is in H (Algorithm 1, deletion
   branch; Sec. III-C);
2. for a deleted edge (p, q) that was in H, s walkers start at p on the
   updated G.  When some walker reaches q, the hitting walker with the least
   resistance sum (Eq. 12) gives the path whose edges not in H are
   recovered.  When none does, a few edges near p and q are recovered
   (Sec. III-C, last paragraph);
3. for an inserted edge (p, q, w), s walkers start at p on H.  A walker
   stops when w times its resistance sum exceeds K, after L steps, or at a
   leaf.  The edge is kept iff no walker reaches q (Sec. III-B; Algorithm 1,
   insertion branch);
4. G gains the insertions and H gains the kept, recovered and fallback edges
   at the end of the batch (Sec. III-F).  Every walk of the batch therefore
   reads the graphs as they stand after step 1.

The walk is non-backtracking: it never steps straight back to the vertex it
came from.  It is biased by edge weight, and each step adds the chosen
edge's resistance 1/w to the walker's sum (Sec. III-B).

Readings of what the paper leaves open.  These are the same decisions as the
C oracle's, restated here rather than shared:

* a neighbour is chosen with probability proportional to an integer weight,
  qw = w / w_ref * 2^Q rounded half to even and clamped to [1, 2^32 - 1].
  A 64-bit random number r gives target = floor(r * total / 2^64), and the
  pick is the first neighbour, in ascending id order, whose running sum of
  qw exceeds target;
* r is drawn with Philox-4x32-10 (SC'11).  The key is the seed, and the
  counter is (step // 2, walker, uid low, uid high).  Even steps take output
  words 0 and 1, odd steps words 2 and 3, low word first;
* a walker at a vertex with no neighbour other than the one it came from
  stops there.  An optional policy steps back instead;
* the threshold test comes before the hit test, so a step that reaches q
  and also crosses K is a miss;
* the recovered path is the winner's edges in path order, each edge once,
  those not in H.  The winner is the least sum, ties to the lower walker
  index; a sum that overflowed to +inf still names a walker;
* with no hit, each endpoint (first p, then q) recovers its G edge of least
  resistance 1/w that is not in H, ties to the smaller neighbour id;
* a weight must be positive and finite with a finite 1/w.

Variants (all off by default), each an alternative the paper names or
leaves open:

* BOTH_ENDS: odd walkers start at q and aim at p (Sec. III-C lets the walkers
  start at either endpoint);
* LOOP_ERASED: a hitting deletion recovers the edges of the chronological
  loop erasure of the winner's path;
* TWO_STAGE: the deletions' walks and recoveries come first, and the
  recovered edges enter H before the insertion walks.
"""
from __future__ import annotations

import math

BOTH_ENDS = 1
LOOP_ERASED = 2
TWO_STAGE = 4

MAX_WALKERS = 1024
MAX_STEPS = 1024
NO_WINNER = 0xFFFF

_M32 = (1 << 32) - 1
_M64 = (1 << 64) - 1


class LiteralError(ValueError):
    """A batch or an initial state the rules refuse; .name is the reason."""

    def __init__(self, name: str):
        super().__init__(name)
        self.name = name


# --------------------------------------------------------------------------
# Philox (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two multiply-hi/lo
# S-boxes on a 4-word counter, the key bumped by the Weyl increments between
# rounds.


def _philox(counter, key, width: int, mult, weyl, rounds: int = 10):
    mask = (1 << width) - 1
    x0, x1, x2, x3 = (int(c) & mask for c in counter)
    k0, k1 = (int(k) & mask for k in key)
    for rnd in range(rounds):
        if rnd:
            k0 = (k0 + weyl[0]) & mask
            k1 = (k1 + weyl[1]) & mask
        a = mult[0] * x0
        b = mult[1] * x2
        x0, x1, x2, x3 = ((b >> width) ^ x1 ^ k0), b & mask, ((a >> width) ^ x3 ^ k1), a & mask
    return (x0, x1, x2, x3)


def philox4x32(counter, key, rounds: int = 10):
    return _philox(counter, key, 32, (0xD2511F53, 0xCD9E8D57), (0x9E3779B9, 0xBB67AE85), rounds)


def philox4x64(counter, key, rounds: int = 10):
    return _philox(counter, key, 64, (0xD2E7470EE14C6C93, 0xCA5A826395121157),
                   (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B), rounds)


def draw(seed: int, uid: int, walker: int, step: int) -> int:
    """The 64-bit random number walker `walker` of update `uid` uses at `step`."""
    out = philox4x32((step >> 1, walker, uid & _M32, (uid >> 32) & _M32),
                     (seed & _M32, (seed >> 32) & _M32))
    half = 2 * (step & 1)
    return out[half] | (out[half + 1] << 32)


def quantised(w: float, w_ref: float, Q: int) -> int:
    """Integer selection weight of an edge of weight w."""
    x = (w / w_ref) * float(1 << Q)
    if math.isnan(x) or x < 1.0:
        return 1
    if math.isinf(x) or x > float(_M32):
        return _M32
    return max(1, min(_M32, round(x)))


def usable_weight(w: float) -> bool:
    return w > 0.0 and not math.isinf(w) and not math.isinf(1.0 / w)


# --------------------------------------------------------------------------
# graphs: adj[x] maps each neighbour of x to (w, 1/w, qw)


class Graph:
    def __init__(self, n: int):
        self.adj = [dict() for _ in range(n)]

    def has(self, a: int, b: int) -> bool:
        return b in self.adj[a]

    def link(self, a: int, b: int, entry) -> None:
        self.adj[a][b] = entry
        self.adj[b][a] = entry

    def unlink(self, a: int, b: int) -> None:
        del self.adj[a][b]
        del self.adj[b][a]

    def edges(self):
        """(u, v, w) with u < v, ascending."""
        out = []
        for a, nb in enumerate(self.adj):
            for b in sorted(nb):
                if b > a:
                    out.append((a, b, nb[b][0]))
        return out


# --------------------------------------------------------------------------
# one walker (Sec. III-B; on G for a deletion, Sec. III-C)


class Walk:
    __slots__ = ("hit", "path", "R")

    def __init__(self, hit, path, R):
        self.hit = hit
        self.path = path
        self.R = R

    @property
    def steps(self) -> int:
        return len(self.path) - 1

    @property
    def end(self) -> int:
        return self.path[-1]


def walk(X: Graph, p: int, q: int, *, L: int, seed: int, uid: int, walker: int,
         threshold=None, step_back: bool = False) -> Walk:
    """threshold = (w_pq, K): stop once w_pq * R > K (insertions only)."""
    path = [p]
    came_from = None
    R = 0.0
    for t in range(L):
        here = path[-1]
        nb = X.adj[here]
        options = [c for c in sorted(nb) if c != came_from]
        if not options:
            if step_back and came_from is not None:
                nxt = came_from
            else:
                break
        else:
            total = sum(nb[c][2] for c in options)
            target = (draw(seed, uid, walker, t) * total) >> 64
            running = 0
            nxt = None
            for c in options:
                running += nb[c][2]
                if running > target:
                    nxt = c
                    break
            assert nxt is not None
        R = R + nb[nxt][1]
        came_from = here
        path.append(nxt)
        if threshold is not None and threshold[0] * R > threshold[1]:
            return Walk(False, path, R)
        if nxt == q:
            return Walk(True, path, R)
    return Walk(False, path, R)


def loop_erased(path):
    """Chronological loop erasure: meeting a vertex again cuts the path back
    to its first visit."""
    out = []
    where = {}
    for x in path:
        if x in where:
            cut = where[x] + 1
            for y in out[cut:]:
                del where[y]
            del out[cut:]
        else:
            where[x] = len(out)
            out.append(x)
    return out


# --------------------------------------------------------------------------
# the state and its batches


class LiteralOracle:
    def __init__(self, n, edges, h_edges, *, seed, K=math.inf, s=8, L=16, Q=24,
                 w_ref=0.0, dead_end=0, uid_base=0, variant=0):
        """edges: (u, v, w) of G, each edge once; h_edges: (u, v) of H(0)."""
        if (n <= 0 or not 1 <= Q <= 31 or s > MAX_WALKERS or L > MAX_STEPS
                or dead_end not in (0, 1) or math.isnan(K) or not w_ref >= 0.0
                or math.isinf(w_ref) or variant & ~(BOTH_ENDS | LOOP_ERASED | TWO_STAGE)):
            raise LiteralError("INVALID_ARG")
        for u, v, w in edges:
            if not (0 <= u < n and 0 <= v < n):
                raise LiteralError("VERTEX_RANGE")
            if u == v:
                raise LiteralError("SELF_LOOP")
            if not usable_weight(w):
                raise LiteralError("BAD_WEIGHT")
        wmax = max((w for _, _, w in edges), default=0.0)
        self.n = n
        self.seed = seed
        self.K = K
        self.use_K = not (math.isinf(K) and K > 0)
        self.s, self.L, self.Q = s, L, Q
        self.w_ref = w_ref if w_ref > 0.0 else (wmax if wmax > 0.0 else 1.0)
        self.step_back = dead_end == 1
        self.variant = variant
        self.uid_base = uid_base
        self.steps_total = 0
        self.G = Graph(n)
        self.H = Graph(n)
        for u, v, w in edges:
            if self.G.has(u, v):
                raise LiteralError("INVALID_ARG")
            self.G.link(u, v, self._entry(w))
        for a, b in h_edges:
            if not (0 <= a < n and 0 <= b < n):
                raise LiteralError("VERTEX_RANGE")
            if a == b:
                raise LiteralError("SELF_LOOP")
            if not self.G.has(a, b):
                raise LiteralError("H_NOT_SUBSET")
            if self.H.has(a, b):
                raise LiteralError("DUPLICATE_IN_BATCH")
            self.H.link(a, b, self.G.adj[a][b])
        self.recovered = []

    def _entry(self, w):
        return (w, 1.0 / w, quantised(w, self.w_ref, self.Q))

    def _check(self, ins, dels, s, L):
        seen = set()
        for u, v, w in ins:
            if not (0 <= u < self.n and 0 <= v < self.n):
                raise LiteralError("VERTEX_RANGE")
            if u == v:
                raise LiteralError("SELF_LOOP")
            if not usable_weight(w):
                raise LiteralError("BAD_WEIGHT")
            if self.G.has(u, v):
                raise LiteralError("EDGE_EXISTS")
            if (min(u, v), max(u, v)) in seen:
                raise LiteralError("DUPLICATE_IN_BATCH")
            seen.add((min(u, v), max(u, v)))
        seen = set()
        for u, v in dels:
            if not (0 <= u < self.n and 0 <= v < self.n):
                raise LiteralError("VERTEX_RANGE")
            if u == v:
                raise LiteralError("SELF_LOOP")
            if not self.G.has(u, v):
                raise LiteralError("EDGE_MISSING")
            if (min(u, v), max(u, v)) in seen:
                raise LiteralError("DUPLICATE_IN_BATCH")
            seen.add((min(u, v), max(u, v)))
        if any(x > MAX_WALKERS for x in s) or any(x > MAX_STEPS for x in L):
            raise LiteralError("INVALID_ARG")

    def _walkers(self, X, p, q, count, length, uid, threshold):
        out = []
        for k in range(count):
            a, b = (q, p) if (self.variant & BOTH_ENDS and k & 1) else (p, q)
            out.append(walk(X, a, b, L=length, seed=self.seed, uid=uid, walker=k,
                            threshold=threshold, step_back=self.step_back))
        return out

    @staticmethod
    def _winner(walks):
        best = None
        for k, wk in enumerate(walks):
            if wk.hit and (best is None or wk.R < walks[best].R):
                best = k
        return best

    def _repair(self, p, q, walks, best):
        """Edges a deletion recovers into H (Sec. III-C)."""
        taken = []
        if best is not None:
            path = walks[best].path
            if self.variant & LOOP_ERASED:
                path = loop_erased(path)
            keys = set()
            for a, b in zip(path, path[1:]):
                key = (min(a, b), max(a, b))
                if self.H.has(a, b) or key in keys:
                    continue
                keys.add(key)
                taken.append((a, b))
            return taken
        for x in (p, q):
            nb = self.G.adj[x]
            pick = None
            for c in sorted(nb):
                if self.H.has(x, c):
                    continue
                if pick is None or nb[c][1] < nb[pick][1]:
                    pick = c
            if pick is not None:
                taken.append((x, pick))
        return taken

    def _grow_H(self, edges):
        for a, b in edges:
            if not self.H.has(a, b):
                self.H.link(a, b, self.G.adj[a][b])

    def apply_batch(self, ins, dels, s=None, L=None):
        """ins: (u, v, w); dels: (u, v).  s, L: per update (insertions
        first) or None for the defaults.  Returns one dict per update and a
        list of walker records (hit, steps, end, R) per update."""
        n_ins, n_del = len(ins), len(dels)
        s = [self.s] * (n_ins + n_del) if s is None else [int(x) for x in s]
        L = [self.L] * (n_ins + n_del) if L is None else [int(x) for x in L]
        self._check(ins, dels, s, L)
        results = [None] * (n_ins + n_del)
        records = [None] * (n_ins + n_del)

        # step 1: deletions leave G, and H where they were in H
        was_in_H = [self.H.has(u, v) for u, v in dels]
        for (u, v), inH in zip(dels, was_in_H):
            self.G.unlink(u, v)
            if inH:
                self.H.unlink(u, v)

        # step 2: deletion walks on the updated G
        recovered = []
        for j, (u, v) in enumerate(dels):
            i = n_ins + j
            if not was_in_H[j]:
                results[i] = dict(flag=0, any_hit=0, winner=NO_WINNER, n_rec=0, steps=0,
                                  Rmin=math.inf)
                records[i] = [(0, 0, u, 0.0)] * s[i]
                recovered.append([])
                continue
            walks = self._walkers(self.G, u, v, s[i], L[i], self.uid_base + i, None)
            best = self._winner(walks)
            taken = self._repair(u, v, walks, best)
            recovered.append(taken)
            results[i] = dict(flag=1, any_hit=int(best is not None),
                              winner=NO_WINNER if best is None else best, n_rec=len(taken),
                              steps=sum(wk.steps for wk in walks),
                              Rmin=math.inf if best is None else walks[best].R)
            records[i] = [(int(wk.hit), wk.steps, wk.end, wk.R) for wk in walks]
        if self.variant & TWO_STAGE:
            for taken in recovered:
                self._grow_H(taken)

        # step 3: insertion walks on H
        keep = []
        for i, (u, v, w) in enumerate(ins):
            threshold = (w, self.K) if self.use_K else None
            walks = self._walkers(self.H, u, v, s[i], L[i], self.uid_base + i, threshold)
            best = self._winner(walks)
            keep.append(best is None)
            results[i] = dict(flag=int(best is None), any_hit=int(best is not None),
                              winner=NO_WINNER if best is None else best, n_rec=0,
                              steps=sum(wk.steps for wk in walks),
                              Rmin=math.inf if best is None else walks[best].R)
            records[i] = [(int(wk.hit), wk.steps, wk.end, wk.R) for wk in walks]

        # step 4: the batch's additions
        for (u, v, w), k in zip(ins, keep):
            e = self._entry(w)
            self.G.link(u, v, e)
            if k:
                self.H.link(u, v, e)
        if not self.variant & TWO_STAGE:
            for taken in recovered:
                self._grow_H(taken)

        self.uid_base += n_ins + n_del
        self.steps_total += sum(r["steps"] for r in results)
        self.recovered = recovered
        return results, records

    def query(self, which="H"):
        return (self.H if which == "H" else self.G).edges()


# --------------------------------------------------------------------------
# H(0): maximum spanning forest plus a keyed sample of the other edges


def initial_sparsifier(n, edges, n_extra, seed):
    """edges: (u, v, w) with u < v in ascending (u, v) order; returns the set
    of indices of the edges in H(0).  Kruskal over decreasing weight (ties to
    the lower index), then the n_extra left-out edges of least Philox key
    (counter (e low, e high, 0, 0x53504152), key the seed; words 0 and 1)."""
    root = list(range(n))

    def find(x):
        while root[x] != x:
            root[x] = root[root[x]]
            x = root[x]
        return x

    chosen = set()
    for e in sorted(range(len(edges)), key=lambda e: (-edges[e][2], e)):
        a, b = find(edges[e][0]), find(edges[e][1])
        if a != b:
            root[a] = b
            chosen.add(e)
    rest = []
    for e in range(len(edges)):
        if e not in chosen:
            out = philox4x32((e & _M32, e >> 32, 0, 0x53504152),
                             (seed & _M32, (seed >> 32) & _M32))
            rest.append((out[0] | (out[1] << 32), e))
    rest.sort()
    chosen.update(e for _, e in rest[:n_extra])
    return chosen
