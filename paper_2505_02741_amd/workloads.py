"""Seeded synthetic workloads for the dyGRASS update path.

The paper evaluates on SuiteSparse circuit, FEM and Delaunay matrices
(Sec. IV, Table II) which are not available here.  This module builds seeded
stand-ins of the same kind and size:

* ``grid2d``   -- circuit-like 2D power-grid mesh (4-neighbour lattice);
* ``mesh3d``   -- FEM-like 3D lattice, 6 axis neighbours plus one diagonal
                  per face orientation (+x+y, +y+z, +x+z);
* ``rmat``     -- power-law R-MAT graph (Chakrabarti, Zhan, Faloutsos 2004),
                  per-bit quadrant recursion, self loops dropped,
                  deduplicated, undirected, randomly relabelled.

The initial sparsifier H0 stands in for the GRASS output the paper starts
from (Sec. III-A): a maximum-weight spanning forest plus ``round(0.1 n)``
off-tree edges drawn uniformly without replacement, which matches the paper's
initial off-tree density d_H ~ 10% (Table II).

Update streams follow the paper's experiments (Sec. IV-A): batches of
insertions between nearby vertices (2-6 hops apart on the lattice) and
deletions drawn uniformly from the current graph.

This module is shared by the tests, the benchmark and the oracle's drivers.
It holds none of the method's arithmetic: no walks, no resistances, no
quantisation, no decisions.  Everything here is a pure function of its seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Graph",
    "Batch",
    "Workload",
    "grid2d",
    "mesh3d",
    "rmat",
    "draw_weights",
    "max_spanning_forest",
    "initial_sparsifier",
    "to_csr",
    "EdgeSet",
    "make_workload",
    "CONFIGS",
]


# --------------------------------------------------------------------------
# containers


@dataclass
class Graph:
    """Undirected simple graph as canonical edge arrays (u < v), sorted."""

    n: int
    u: np.ndarray  # uint32
    v: np.ndarray  # uint32
    w: np.ndarray  # float64

    @property
    def m(self) -> int:
        return int(self.u.size)


@dataclass
class Batch:
    """One batch of updates; insertions first, then deletions (uid order)."""

    iu: np.ndarray
    iv: np.ndarray
    iw: np.ndarray
    du: np.ndarray
    dv: np.ndarray
    s: np.ndarray | None = None  # uint16 per update or None for the default
    L: np.ndarray | None = None

    @property
    def n_ins(self) -> int:
        return int(self.iu.size)

    @property
    def n_del(self) -> int:
        return int(self.du.size)

    @property
    def size(self) -> int:
        return self.n_ins + self.n_del


@dataclass
class Workload:
    name: str
    G: Graph
    h_mask: np.ndarray  # bool per edge of G: edge is in H0
    batches: list
    seed_walk: int
    s: int
    L: int
    K: float = math.inf
    meta: dict = field(default_factory=dict)

    @property
    def hu(self) -> np.ndarray:
        return self.G.u[self.h_mask]

    @property
    def hv(self) -> np.ndarray:
        return self.G.v[self.h_mask]


# --------------------------------------------------------------------------
# graphs


def _canonical(n: int, u: np.ndarray, v: np.ndarray):
    """Drop self loops, orient u < v, deduplicate, sort by (u, v)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = np.unique(a * n + b)
    return (key // n).astype(np.uint32), (key % n).astype(np.uint32)


def grid2d(side: int):
    """side x side 4-neighbour lattice; vertex id = y*side + x."""
    n = side * side
    ids = np.arange(n, dtype=np.int64).reshape(side, side)
    hu = ids[:, :-1].ravel()
    hv = ids[:, 1:].ravel()
    vu = ids[:-1, :].ravel()
    vv = ids[1:, :].ravel()
    u, v = _canonical(n, np.concatenate([hu, vu]), np.concatenate([hv, vv]))
    return n, u, v


def mesh3d(side: int):
    """side^3 lattice, id = (z*side + y)*side + x; 6 axis neighbours plus the
    +x+y, +y+z and +x+z face diagonals."""
    n = side**3
    ids = np.arange(n, dtype=np.int64).reshape(side, side, side)  # [z, y, x]
    us, vs = [], []
    # axis neighbours
    us.append(ids[:, :, :-1].ravel()); vs.append(ids[:, :, 1:].ravel())   # x
    us.append(ids[:, :-1, :].ravel()); vs.append(ids[:, 1:, :].ravel())   # y
    us.append(ids[:-1, :, :].ravel()); vs.append(ids[1:, :, :].ravel())   # z
    # face diagonals
    us.append(ids[:, :-1, :-1].ravel()); vs.append(ids[:, 1:, 1:].ravel())  # +x+y
    us.append(ids[:-1, :-1, :].ravel()); vs.append(ids[1:, 1:, :].ravel())  # +y+z
    us.append(ids[:-1, :, :-1].ravel()); vs.append(ids[1:, :, 1:].ravel())  # +x+z
    u, v = _canonical(n, np.concatenate(us), np.concatenate(vs))
    return n, u, v


def rmat(scale: int, edge_factor: int, abcd=(0.57, 0.19, 0.19, 0.05), rng=None,
         chunk: int = 1 << 21, workers: int | None = None):
    """R-MAT by per-bit quadrant recursion, then random relabelling.

    Edge samples are drawn in chunks, each from its own generator seeded by
    (a base seed drawn from rng, chunk index), so the graph depends only on
    rng and not on how many threads draw the chunks.  Each bit of a sample
    takes 32 random bits: quadrant (0,0) below a*2^32, (0,1) below
    (a+b)*2^32, (1,0) below (a+b+c)*2^32, else (1,1)."""
    from concurrent.futures import ThreadPoolExecutor

    rng = np.random.default_rng(rng)
    n = 1 << scale
    total = edge_factor * n
    a, b, c, _ = abcd
    t_a = np.uint32(min(round(a * 2**32), 2**32 - 1))
    t_ab = np.uint32(min(round((a + b) * 2**32), 2**32 - 1))
    t_abc = np.uint32(min(round((a + b + c) * 2**32), 2**32 - 1))
    base = int(rng.integers(0, 2**63))
    counts = [min(chunk, total - s) for s in range(0, total, chunk)]

    def draw(k):
        cnt = counts[k]
        g = np.random.default_rng([base, k])
        src = np.zeros(cnt, dtype=np.uint32)
        dst = np.zeros(cnt, dtype=np.uint32)
        for bit in range(0, scale, 2):
            raw = g.bit_generator.random_raw(cnt)
            for half, bb in ((raw & 0xFFFFFFFF, bit), (raw >> 32, bit + 1)):
                if bb >= scale:
                    break
                r = half.astype(np.uint32)
                down = r >= t_ab
                right = (r >= t_abc) | ((r >= t_a) & ~down)
                src |= down.astype(np.uint32) << np.uint32(bb)
                dst |= right.astype(np.uint32) << np.uint32(bb)
        keep = src != dst
        src, dst = src[keep], dst[keep]
        lo = np.minimum(src, dst).astype(np.int64)
        hi = np.maximum(src, dst).astype(np.int64)
        return np.unique(lo * n + hi)

    import os

    workers = workers or max(1, min(os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(workers) as ex:
        keys = list(ex.map(draw, range(len(counts))))
    key = np.unique(np.concatenate(keys))
    perm = rng.permutation(n).astype(np.int64)
    u = perm[key // n]
    v = perm[key % n]
    u, v = _canonical(n, u, v)
    return n, u, v


def draw_weights(kind: str, m: int, rng) -> np.ndarray:
    rng = np.random.default_rng(rng)
    if kind == "uniform_1_10":
        return rng.uniform(1.0, 10.0, m)
    if kind == "uniform_0.5_2":
        return rng.uniform(0.5, 2.0, m)
    if kind == "lognormal_0_1":
        return rng.lognormal(0.0, 1.0, m)
    if kind == "unit":
        return np.ones(m)
    raise ValueError(kind)


def _stable_order(x: np.ndarray) -> np.ndarray:
    """Stable argsort of non-negative integers below 2^32: two stable passes
    on 16-bit digits (numpy sorts 16-bit keys by radix)."""
    o = np.argsort((x & 0xFFFF).astype(np.uint16), kind="stable")
    if x.size and int(x.max()) >= 1 << 16:
        o = o[np.argsort((x[o] >> 16).astype(np.uint16), kind="stable")]
    return o


def to_csr(n: int, u: np.ndarray, v: np.ndarray, w: np.ndarray):
    """Symmetric CSR (rowptr uint64[n+1], col uint32, w float64), rows
    ascending by neighbour id."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    m = u.size
    key = u * n + v
    if m and np.all(u < v) and np.all(key[1:] > key[:-1]):
        # canonical edges sorted by (u, v): row r is its smaller neighbours
        # (edges (x, r), in the order of x) followed by its larger ones
        # (edges (r, y), already in the order of y)
        lower = np.bincount(v, minlength=n)  # neighbours below r
        upper = np.bincount(u, minlength=n)  # neighbours above r
        rowptr = np.zeros(n + 1, dtype=np.uint64)
        rowptr[1:] = np.cumsum(lower + upper, dtype=np.uint64)
        start = rowptr[:-1].astype(np.int64)
        col = np.empty(2 * m, dtype=np.uint32)
        ww = np.empty(2 * m, dtype=np.float64)
        idx = np.arange(m, dtype=np.int64)
        first_u = np.cumsum(upper) - upper  # first edge (r, .) in input order
        pos = start[u] + lower[u] + (idx - first_u[u])
        col[pos] = v
        ww[pos] = w
        o = _stable_order(v)  # by v, then u (input order)
        vs = v[o]
        first_v = np.cumsum(lower) - lower
        pos = start[vs] + (idx - first_v[vs])
        col[pos] = u[o]
        ww[pos] = w[o]
        return rowptr, col, ww
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    ww = np.concatenate([w, w])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    counts = np.bincount(src, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.uint64)
    rowptr[1:] = np.cumsum(counts, dtype=np.uint64)
    return rowptr, dst.astype(np.uint32), ww


# --------------------------------------------------------------------------
# initial sparsifier (stand-in for GRASS)


class _DSU:
    def __init__(self, n):
        self.p = list(range(n))

    def find(self, x):
        p = self.p
        while p[x] != x:
            p[x] = p[p[x]]
            x = p[x]
        return x

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra == rb:
            return False
        self.p[ra] = rb
        return True


def max_spanning_forest(n: int, u: np.ndarray, v: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Boolean mask of a maximum-weight spanning forest: Kruskal over edges in
    order of decreasing weight, ties by canonical edge index."""
    m = u.size
    if m == 0:
        return np.zeros(0, dtype=bool)
    if np.unique(w).size == m and m > 50_000:
        # distinct weights: the maximum spanning forest is unique, so any
        # correct Kruskal gives the same edge set
        import scipy.sparse as sp
        from scipy.sparse.csgraph import minimum_spanning_tree

        idx = np.arange(m, dtype=np.int64)
        A = sp.csr_matrix((-w, (u.astype(np.int64), v.astype(np.int64))), shape=(n, n))
        T = minimum_spanning_tree(A).tocoo()
        key = np.minimum(T.row, T.col).astype(np.int64) * n + np.maximum(T.row, T.col)
        ekey = u.astype(np.int64) * n + v.astype(np.int64)
        pos = np.searchsorted(ekey, key)
        mask = np.zeros(m, dtype=bool)
        mask[idx[pos]] = True
        return mask
    order = np.lexsort((np.arange(m), -w))
    dsu = _DSU(n)
    mask = np.zeros(m, dtype=bool)
    uu = u.tolist()
    vv = v.tolist()
    for e in order.tolist():
        if dsu.union(uu[e], vv[e]):
            mask[e] = True
    return mask


def initial_sparsifier(G: Graph, rng, off_tree_frac: float = 0.10, with_forest: bool = False):
    """Forest + round(off_tree_frac * n) off-tree edges, uniform without
    replacement; with_forest: also the number of forest edges."""
    rng = np.random.default_rng(rng)
    mask = max_spanning_forest(G.n, G.u, G.v, G.w)
    n_forest = int(mask.sum())
    off = np.flatnonzero(~mask)
    extra = min(int(round(off_tree_frac * G.n)), off.size)
    pick = rng.choice(off, size=extra, replace=False) if extra else np.zeros(0, np.int64)
    mask[pick] = True
    return (mask, n_forest) if with_forest else mask


# --------------------------------------------------------------------------
# evolving edge set used to draw valid update streams


class EdgeSet:
    """The current edge set of G, kept as a fixed sorted base plus inserted
    keys, for membership tests and uniform deletion draws."""

    def __init__(self, G: Graph):
        self.n = G.n
        self.base = G.u.astype(np.int64) * G.n + G.v.astype(np.int64)
        self.alive = np.ones(self.base.size, dtype=bool)
        self.extra = np.zeros(0, dtype=np.int64)  # sorted

    def key(self, a, b):
        a = np.asarray(a, dtype=np.int64)
        b = np.asarray(b, dtype=np.int64)
        return np.minimum(a, b) * self.n + np.maximum(a, b)

    def contains(self, keys: np.ndarray) -> np.ndarray:
        keys = np.asarray(keys, dtype=np.int64)
        pos = np.searchsorted(self.base, keys)
        posc = np.minimum(pos, self.base.size - 1)
        inb = (self.base.size > 0) & (self.base[posc] == keys) & self.alive[posc]
        if self.extra.size:
            pe = np.minimum(np.searchsorted(self.extra, keys), self.extra.size - 1)
            ine = self.extra[pe] == keys
        else:
            ine = np.zeros(keys.size, dtype=bool)
        return inb | ine

    def current_keys(self) -> np.ndarray:
        return np.concatenate([self.base[self.alive], self.extra])

    def apply(self, ins_keys: np.ndarray, del_keys: np.ndarray):
        if del_keys.size:
            pos = np.searchsorted(self.base, del_keys)
            posc = np.minimum(pos, self.base.size - 1)
            hitb = self.base[posc] == del_keys
            self.alive[posc[hitb]] = False
            rest = del_keys[~hitb]
            if rest.size:
                self.extra = np.setdiff1d(self.extra, rest)
        if ins_keys.size:
            self.extra = np.union1d(self.extra, ins_keys)


def _lattice_offsets(dim: int, h: int):
    rng = range(-h, h + 1)
    if dim == 2:
        offs = [(dx, dy, 0) for dx in rng for dy in rng if abs(dx) + abs(dy) == h]
    else:
        offs = [(dx, dy, dz) for dx in rng for dy in rng for dz in rng
                if abs(dx) + abs(dy) + abs(dz) == h]
    return np.array(offs, dtype=np.int64)


def _first_unique(keys: np.ndarray) -> np.ndarray:
    """Mask keeping the first occurrence of every key."""
    _, first = np.unique(keys, return_index=True)
    mask = np.zeros(keys.size, dtype=bool)
    mask[first] = True
    return mask


def local_insertions_lattice(es: EdgeSet, side: int, dim: int, count: int, rng,
                             taken: np.ndarray, hmin=2, hmax=6):
    """count insertions (p, q): p uniform, h ~ U{hmin..hmax}, q = p + a
    lattice offset of L1 length h drawn uniformly, in bounds; an edge already
    in G or already drawn in this batch is redrawn."""
    if count == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    offs = {h: _lattice_offsets(dim, h) for h in range(hmin, hmax + 1)}
    n = es.n
    out_p, out_q = [], []
    have = 0
    taken = taken.copy()
    while have < count:
        M = max(2 * (count - have), 64)
        p = rng.integers(0, n, M)
        h = rng.integers(hmin, hmax + 1, M)
        q = np.full(M, -1, dtype=np.int64)
        for hh in range(hmin, hmax + 1):
            sel = np.flatnonzero(h == hh)
            if sel.size == 0:
                continue
            o = offs[hh][rng.integers(0, len(offs[hh]), sel.size)]
            x = p[sel] % side
            y = (p[sel] // side) % side
            z = p[sel] // (side * side) if dim == 3 else np.zeros(sel.size, np.int64)
            nx, ny, nz = x + o[:, 0], y + o[:, 1], z + o[:, 2]
            ok = (nx >= 0) & (nx < side) & (ny >= 0) & (ny < side)
            if dim == 3:
                ok &= (nz >= 0) & (nz < side)
            qq = (nz * side + ny) * side + nx if dim == 3 else ny * side + nx
            q[sel[ok]] = qq[ok]
        good = q >= 0
        p, q = p[good], q[good]
        k = es.key(p, q)
        good = ~es.contains(k) & ~np.isin(k, taken)
        p, q, k = p[good], q[good], k[good]
        fu = _first_unique(k)
        p, q, k = p[fu], q[fu], k[fu]
        need = count - have
        p, q, k = p[:need], q[:need], k[:need]
        out_p.append(p)
        out_q.append(q)
        taken = np.concatenate([taken, k])
        have += p.size
    return np.concatenate(out_p), np.concatenate(out_q)


def local_insertions_walk(es: EdgeSet, rowptr, col, count: int, rng, taken,
                          hmin=2, hmax=6):
    """For graphs without coordinates: p uniform over non-isolated vertices,
    q = end of an h-step uniform random walk on the initial graph,
    h ~ U{hmin..hmax}; self pairs, existing edges and repeats are redrawn."""
    if count == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    n = es.n
    deg = (rowptr[1:] - rowptr[:-1]).astype(np.int64)
    nz = np.flatnonzero(deg > 0)
    out_p, out_q = [], []
    have = 0
    taken = taken.copy()
    rp = rowptr.astype(np.int64)
    while have < count:
        M = max(2 * (count - have), 64)
        p = nz[rng.integers(0, nz.size, M)]
        h = rng.integers(hmin, hmax + 1, M)
        x = p.copy()
        for t in range(hmax):
            act = h > t
            d = deg[x]
            j = (rng.random(M) * d).astype(np.int64)
            nxt = col[rp[x] + np.minimum(j, np.maximum(d - 1, 0))].astype(np.int64)
            x = np.where(act & (d > 0), nxt, x)
        q = x
        k = es.key(p, q)
        good = (p != q) & ~es.contains(k) & ~np.isin(k, taken)
        p, q, k = p[good], q[good], k[good]
        fu = _first_unique(k)
        p, q, k = p[fu], q[fu], k[fu]
        need = count - have
        p, q, k = p[:need], q[:need], k[:need]
        out_p.append(p)
        out_q.append(q)
        taken = np.concatenate([taken, k])
        have += p.size
    return np.concatenate(out_p), np.concatenate(out_q)


def uniform_deletions(es: EdgeSet, count: int, rng):
    keys = es.current_keys()
    count = min(count, keys.size)
    pick = rng.choice(keys.size, size=count, replace=False)
    k = keys[pick]
    a = (k // es.n).astype(np.uint32)
    b = (k % es.n).astype(np.uint32)
    # random orientation: the first endpoint is where deletion walkers start
    flip = rng.random(count) < 0.5
    return np.where(flip, b, a), np.where(flip, a, b)


# --------------------------------------------------------------------------
# named configurations

CONFIGS = {
    # 64x64 grid, 10 x 100 insertions, s=8, L=16 (oracle finishes in seconds)
    "grid64": dict(kind="grid", side=64, weights="uniform_1_10", batches=10,
                   ins=100, dels=0, s=8, L=16),
    # 1024x1024 lognormal power grid, 10 x 20k insertions, s=64, L=32
    "grid1024": dict(kind="grid", side=1024, weights="lognormal_0_1", batches=10,
                     ins=20_000, dels=0, s=64, L=32),
    # 128^3 FEM-like mesh, 20 x (10k ins + 10k del), s=64, L=24
    "mesh128": dict(kind="mesh", side=128, weights="uniform_0.5_2", batches=20,
                    ins=10_000, dels=10_000, s=64, L=24),
    # R-MAT scale 22, 50 uneven batches (log-uniform 100..200k), 70/30 ins/del,
    # per-update s ~ U{16..128}, L ~ U{8..32}
    "rmat22": dict(kind="rmat", scale=22, ef=16, weights="uniform_1_10",
                   batches=50, size_lo=100, size_hi=200_000, ins_frac=0.7,
                   s_lo=16, s_hi=128, L_lo=8, L_hi=32, s=64, L=32),
}


def _seeds(seed: int):
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(5)
    graph, wts, spars, stream, walk = kids
    walk_seed = int(walk.generate_state(1, dtype=np.uint64)[0])
    return graph, wts, spars, stream, walk_seed


def make_workload(name: str, seed: int = 1, n_batches: int | None = None,
                  **overrides) -> Workload:
    """Build a named workload (see CONFIGS); keyword overrides change any
    field, e.g. make_workload("grid64", side=16, ins=20)."""
    if name not in CONFIGS:
        raise KeyError(name)
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    if n_batches is not None:
        cfg["batches"] = n_batches
    sg, sw, sh, sst, walk_seed = _seeds(seed)
    kind = cfg["kind"]
    if kind == "grid":
        n, u, v = grid2d(cfg["side"])
    elif kind == "mesh":
        n, u, v = mesh3d(cfg["side"])
    elif kind == "rmat":
        n, u, v = rmat(cfg["scale"], cfg["ef"], rng=np.random.default_rng(sg))
    else:
        raise ValueError(kind)
    w = draw_weights(cfg["weights"], u.size, np.random.default_rng(sw))
    G = Graph(n, u, v, w)
    h_mask, n_forest = initial_sparsifier(G, np.random.default_rng(sh), with_forest=True)
    rng = np.random.default_rng(sst)
    es = EdgeSet(G)
    batches = []
    rowptr = col = None
    if kind == "rmat":
        rowptr, col, _ = to_csr(n, u, v, w)
    for _ in range(cfg["batches"]):
        if "size_lo" in cfg:
            # uneven batches: size log-uniform in [size_lo, size_hi], each
            # update an insertion with probability ins_frac
            size = int(math.floor(math.exp(rng.uniform(math.log(cfg["size_lo"]),
                                                       math.log(cfg["size_hi"])))))
            n_ins = int((rng.random(size) < cfg["ins_frac"]).sum())
            n_del = size - n_ins
        else:
            n_ins, n_del = cfg["ins"], cfg["dels"]
        empty = np.zeros(0, dtype=np.int64)
        if kind == "rmat":
            p, q = local_insertions_walk(es, rowptr, col, n_ins, rng, empty)
        else:
            p, q = local_insertions_lattice(es, cfg["side"], 2 if kind == "grid" else 3,
                                            n_ins, rng, empty)
        iw = draw_weights(cfg["weights"], p.size, rng)
        du, dv = uniform_deletions(es, n_del, rng) if n_del else (empty, empty)
        b = Batch(p.astype(np.uint32), q.astype(np.uint32), iw.astype(np.float64),
                  np.asarray(du, dtype=np.uint32), np.asarray(dv, dtype=np.uint32))
        if cfg.get("s_lo") is not None:
            b.s = rng.integers(cfg["s_lo"], cfg["s_hi"] + 1, b.size).astype(np.uint16)
            b.L = rng.integers(cfg["L_lo"], cfg["L_hi"] + 1, b.size).astype(np.uint16)
        es.apply(es.key(b.iu, b.iv), es.key(b.du, b.dv))
        batches.append(b)
    return Workload(name=name, G=G, h_mask=h_mask, batches=batches,
                    seed_walk=walk_seed, s=cfg["s"], L=cfg["L"],
                    meta=dict(cfg=cfg, seed=seed, forest_edges=n_forest))


def make_fleet(n_graphs: int = 64, seed: int = 1, n_lo: int = 10_000, n_hi: int = 2_000_000,
               batches_per_graph: int = 32, size_lo: int = 1, size_hi: int = 50_000,
               ins_frac: float = 0.6, s: int = 64, L: int = 24) -> list:
    """Many graphs for the serving form: kinds cycled grid / mesh / R-MAT, n
    log-uniform in [n_lo, n_hi] (grid side sqrt(n), mesh side cbrt(n), R-MAT
    scale ceil(log2 n)), each with its own seed and its own stream of uneven
    batches (size log-uniform in [size_lo, min(size_hi, n/2)], ins_frac
    insertions)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5EED]))
    base = {"grid": "grid1024", "mesh": "mesh128", "rmat": "rmat22"}
    out = []
    for g in range(n_graphs):
        kind = ("grid", "mesh", "rmat")[g % 3]
        n = math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))
        # batches up to half the vertex count, so small graphs are not swamped
        hi = max(size_lo + 1, min(size_hi, int(n) // 2))
        over = dict(size_lo=size_lo, size_hi=hi, ins_frac=ins_frac, s=s, L=L)
        if kind == "grid":
            over["side"] = max(8, int(round(math.sqrt(n))))
        elif kind == "mesh":
            over["side"] = max(6, int(round(n ** (1.0 / 3.0))))
        else:
            over["scale"] = max(10, int(math.ceil(math.log2(n))))
            for k in ("s_lo", "s_hi", "L_lo", "L_hi"):
                over[k] = None
        wl = make_workload(base[kind], seed=seed * 1000 + g, n_batches=batches_per_graph, **over)
        wl.name = f"{kind}{g}"
        out.append(wl)
    return out
