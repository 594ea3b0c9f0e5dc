"""ctypes binding of libdygrass (include/dygrass.h).

Argument marshalling only: every step of a batch runs in the HIP kernels of
libdygrass.so.  The functions keep the C names; ``Dygrass`` is a small
convenience wrapper around a context.  Importing this module fails loudly if
the library has not been built (``python paper_2505_02741_amd/build.py``):
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DYGRASS_LIB") or os.path.join(_HERE, "libdygrass.so")

STATUS = {
    0: "OK",
    -1: "INVALID_ARG",
    -2: "SELF_LOOP",
    -3: "VERTEX_RANGE",
    -4: "BAD_WEIGHT",
    -5: "EDGE_EXISTS",
    -6: "EDGE_MISSING",
    -7: "DUPLICATE_IN_BATCH",
    -8: "H_NOT_SUBSET",
    -9: "NOMEM",
    -10: "DEVICE",
    -11: "TOO_LARGE",
    -12: "BUSY",
}

STATIC_SCRATCH_BYTES = 64 << 20  # the static working memory of dyg_apply_batch_dev_static

FLAG_LEAN_POOLS = 1
FLAG_TIMING = 2
FLAG_BATCHED = 4
FLAG_GRAPH = 8
FLAG_AUTOTUNE = 16
FLAG_TIMING_WALK = 32
FLAG_FAIL_POOL_GROWTH = 64
FLAG_BOTH_ENDS = 128
FLAG_LOOP_ERASED = 256
FLAG_TWO_STAGE = 512

DEAD_END_TERMINATE = 0
DEAD_END_BOUNCE = 1
MAX_WALKERS = 1024
MAX_STEPS = 1024

UPDATE_RESULT_DTYPE = np.dtype([("kind", "u1"), ("flag", "u1"), ("any_hit", "u1"),
                                ("reserved", "u1"), ("winner", "<u2"), ("n_rec", "<u2"),
                                ("steps", "<u4"), ("reserved2", "<u4"), ("Rmin", "<f8")])
WALKER_RECORD_DTYPE = np.dtype([("hit", "u1"), ("reserved", "u1"), ("steps", "<u2"),
                                ("end", "<u4"), ("R", "<f8")])
assert UPDATE_RESULT_DTYPE.itemsize == 24 and WALKER_RECORD_DTYPE.itemsize == 16


class dyg_params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("K", C.c_double), ("s_default", C.c_uint16),
                ("L_default", C.c_uint16), ("Q", C.c_uint8), ("dead_end", C.c_uint8),
                ("reserved0", C.c_uint16), ("w_ref", C.c_double), ("slack", C.c_double),
                ("uid_base", C.c_uint64), ("flags", C.c_uint32), ("reserved1", C.c_uint32)]


class dyg_stats_t(C.Structure):
    _fields_ = [("n", C.c_uint32), ("reserved", C.c_uint32), ("g_edges", C.c_uint64),
                ("h_edges", C.c_uint64), ("g_pool_used", C.c_uint64),
                ("g_pool_cap", C.c_uint64), ("h_pool_used", C.c_uint64),
                ("h_pool_cap", C.c_uint64), ("g_dead", C.c_uint64), ("h_dead", C.c_uint64),
                ("uid_base", C.c_uint64), ("batches", C.c_uint64),
                ("compactions", C.c_uint64), ("w_ref", C.c_double),
                ("walk_steps", C.c_uint64), ("walk_alg_bytes", C.c_uint64),
                ("walk_launches", C.c_uint64), ("walk_ms_total", C.c_double),
                ("walk_ms_last", C.c_double), ("batch_ms_last", C.c_double)]


class dyg_tuning(C.Structure):
    _fields_ = [("walk_blocks_per_cu", C.c_uint32), ("refill_min", C.c_uint32),
                ("updates_per_wave", C.c_uint32), ("tail_lanes", C.c_uint32),
                ("lockstep", C.c_uint32), ("reserved", C.c_uint32 * 3)]


class dyg_batch_dev(C.Structure):
    _fields_ = [("n_ins", C.c_uint64), ("n_del", C.c_uint64), ("iu", C.c_void_p),
                ("iv", C.c_void_p), ("iw", C.c_void_p), ("du", C.c_void_p),
                ("dv", C.c_void_p), ("s", C.c_void_p), ("L", C.c_void_p),
                ("L_max", C.c_uint32), ("s_max", C.c_uint32), ("results", C.c_void_p)]


class dyg_server_params(C.Structure):
    _fields_ = [("mem_budget", C.c_uint64), ("max_fused", C.c_uint32),
                ("max_inflight", C.c_uint32), ("walk_blocks_per_cu", C.c_uint32),
                ("reserved", C.c_uint32 * 3)]


class dyg_request_done(C.Structure):
    _fields_ = [("request_id", C.c_uint64), ("graph_id", C.c_uint32), ("status", C.c_int32),
                ("n_updates", C.c_uint64), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double)]


EXPORTS = ["dyg_default_params", "dyg_init", "dyg_apply_batch", "dyg_apply_batch_dev",
           "dyg_apply_batch_dev_static", "dyg_initial_sparsifier",
           "dyg_sync", "dyg_query_sparsifier", "dyg_query_graph", "dyg_stats", "dyg_compact",
           "dyg_destroy", "dyg_error_string", "dyg_get_tuning", "dyg_set_tuning", "dyg_reserve",
           "dyg_check_state", "dyg_server_default_params", "dyg_server_create",
           "dyg_server_add_graph", "dyg_server_submit", "dyg_server_poll", "dyg_server_pending",
           "dyg_server_now", "dyg_server_destroy"]


class DygError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = int(code)
        self.name = STATUS.get(self.code, "?")
        super().__init__(f"{where}: {self.name} ({self.code})")


def _load():
    # A process must hold one HIP runtime.  PyTorch ships its own copy; when it
    # is installed, load it first so that libdygrass binds to the same runtime
    # (its device pointers and streams are then valid here, and torch keeps
    # seeing the GPU after this library has used it).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_2505_02741_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.dyg_default_params.argtypes = [C.POINTER(dyg_params)]
    lib.dyg_default_params.restype = None
    lib.dyg_init.argtypes = [C.POINTER(C.c_void_p), C.c_uint32, P, P, P, C.c_uint64, P, P,
                             C.POINTER(dyg_params)]
    lib.dyg_init.restype = C.c_int
    lib.dyg_apply_batch.argtypes = [P, C.c_uint64, P, P, P, C.c_uint64, P, P, P, P, P, P]
    lib.dyg_apply_batch.restype = C.c_int
    lib.dyg_apply_batch_dev.argtypes = [P, C.POINTER(dyg_batch_dev), P]
    lib.dyg_apply_batch_dev.restype = C.c_int
    lib.dyg_apply_batch_dev_static.argtypes = [P, C.POINTER(dyg_batch_dev), P]
    lib.dyg_apply_batch_dev_static.restype = C.c_int
    lib.dyg_initial_sparsifier.argtypes = [C.c_uint32, P, P, P, C.c_uint64, C.c_uint64,
                                           C.c_uint64, C.POINTER(C.c_uint64), P, P]
    lib.dyg_initial_sparsifier.restype = C.c_int
    lib.dyg_sync.argtypes = [P]
    lib.dyg_sync.restype = C.c_int
    for fn in (lib.dyg_query_sparsifier, lib.dyg_query_graph):
        fn.argtypes = [P, C.c_uint64, C.POINTER(C.c_uint64), P, P, P]
        fn.restype = C.c_int
    lib.dyg_stats.argtypes = [P, C.POINTER(dyg_stats_t)]
    lib.dyg_stats.restype = C.c_int
    lib.dyg_server_default_params.argtypes = [C.POINTER(dyg_server_params)]
    lib.dyg_server_default_params.restype = None
    lib.dyg_server_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(dyg_server_params)]
    lib.dyg_server_create.restype = C.c_int
    lib.dyg_server_add_graph.argtypes = [P, P, C.POINTER(C.c_uint32)]
    lib.dyg_server_add_graph.restype = C.c_int
    lib.dyg_server_submit.argtypes = [P, C.c_uint32, C.c_uint64, P, P, P, C.c_uint64, P, P, P,
                                      C.POINTER(C.c_uint64)]
    lib.dyg_server_submit.restype = C.c_int
    lib.dyg_server_poll.argtypes = [P, C.POINTER(dyg_request_done), C.c_uint32,
                                    C.POINTER(C.c_uint32)]
    lib.dyg_server_poll.restype = C.c_int
    lib.dyg_server_pending.argtypes = [P]
    lib.dyg_server_pending.restype = C.c_uint64
    lib.dyg_server_now.argtypes = [P]
    lib.dyg_server_now.restype = C.c_double
    lib.dyg_server_destroy.argtypes = [P]
    lib.dyg_server_destroy.restype = None
    lib.dyg_check_state.argtypes = [P, C.c_char_p, C.c_uint64]
    lib.dyg_check_state.restype = C.c_int
    lib.dyg_get_tuning.argtypes = [P, C.POINTER(dyg_tuning)]
    lib.dyg_get_tuning.restype = C.c_int
    lib.dyg_reserve.argtypes = [P, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32]
    lib.dyg_reserve.restype = C.c_int
    lib.dyg_set_tuning.argtypes = [P, C.POINTER(dyg_tuning)]
    lib.dyg_set_tuning.restype = C.c_int
    lib.dyg_compact.argtypes = [P]
    lib.dyg_compact.restype = C.c_int
    lib.dyg_destroy.argtypes = [P]
    lib.dyg_destroy.restype = None
    lib.dyg_error_string.argtypes = [C.c_int]
    lib.dyg_error_string.restype = C.c_char_p
    return lib


_lib = _load()


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc: int, where: str):
    if rc != 0:
        raise DygError(rc, where)


# --------------------------------------------------------------------------
# C entry points


def dyg_default_params(**overrides) -> dyg_params:
    p = dyg_params()
    _lib.dyg_default_params(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def dyg_error_string(code: int) -> str:
    return _lib.dyg_error_string(int(code)).decode()


def dyg_init(n, rowptr, col, w, h_u, h_v, params: dyg_params) -> C.c_void_p:
    rowptr = _arr(rowptr, np.uint64)
    col = _arr(col, np.uint32)
    w = _arr(w, np.float64)
    h_u = _arr(h_u, np.uint32)
    h_v = _arr(h_v, np.uint32)
    # the library reads n + 1 row offsets, rowptr[n] entries of col and w, and
    # h_m entries of h_u and h_v
    if rowptr.size != int(n) + 1:
        raise ValueError(f"rowptr has {rowptr.size} entries for n = {int(n)}")
    if col.size != int(rowptr[-1]) or w.size != int(rowptr[-1]):
        raise ValueError(f"col and w need rowptr[n] = {int(rowptr[-1])} entries, "
                         f"got {col.size} and {w.size}")
    if h_v.size != h_u.size:
        raise ValueError(f"h_u, h_v differ in length ({h_u.size}, {h_v.size})")
    ctx = C.c_void_p()
    _check(_lib.dyg_init(C.byref(ctx), int(n), _ptr(rowptr), _ptr(col), _ptr(w), h_u.size,
                         _ptr(h_u), _ptr(h_v), C.byref(params)), "dyg_init")
    return ctx


def _check_host_batch(iu, iv, iw, du, dv, s=None, L=None):
    """The library reads n_ins entries of iu, iv, iw, n_del of du, dv and
    n_ins + n_del of s and L: refuse shorter arrays before it reads past
    their end."""
    if iv.size != iu.size or iw.size != iu.size:
        raise ValueError(f"iu, iv, iw differ in length ({iu.size}, {iv.size}, {iw.size})")
    if dv.size != du.size:
        raise ValueError(f"du, dv differ in length ({du.size}, {dv.size})")
    nu = iu.size + du.size
    for name, a in (("s", s), ("L", L)):
        if a is not None and a.size != nu:
            raise ValueError(f"{name} has {a.size} entries for {nu} updates")


def dyg_apply_batch(ctx, iu, iv, iw, du, dv, s=None, L=None, results=True, walkers=False,
                    s_default=None):
    iu = _arr(iu, np.uint32)
    iv = _arr(iv, np.uint32)
    iw = _arr(iw, np.float64)
    du = _arr(du, np.uint32)
    dv = _arr(dv, np.uint32)
    nu = iu.size + du.size
    s_arr = None if s is None else _arr(s, np.uint16)
    L_arr = None if L is None else _arr(L, np.uint16)
    _check_host_batch(iu, iv, iw, du, dv, s_arr, L_arr)
    res = np.zeros(nu, UPDATE_RESULT_DTYPE) if results else None
    wk = None
    if walkers:
        if s_arr is not None:
            tot = int(np.minimum(s_arr.astype(np.int64), MAX_WALKERS).sum())
        else:
            tot = nu * int(s_default)
        wk = np.zeros(tot, WALKER_RECORD_DTYPE)
    _check(_lib.dyg_apply_batch(ctx, iu.size, _ptr(iu), _ptr(iv), _ptr(iw), du.size, _ptr(du),
                                _ptr(dv), _ptr(s_arr), _ptr(L_arr), _ptr(res), _ptr(wk)),
           "dyg_apply_batch")
    return res, wk


def check_dev_batch(iu, iv, iw, du, dv, s=None, L=None, results=None, on_gpu=True):
    """Reject tensors the kernels would misread: iu, iv, du, dv with 4-byte
    elements, iw float64, s and L with 2-byte elements, one entry per update
    each, results at least 24 bytes per update, all contiguous and (on_gpu)
    in GPU memory.  s, L and results may be raw device addresses (ints),
    which are not checked."""
    n_ins, n_del = int(iu.numel()), int(du.numel())
    want = (("iu", iu, 4, n_ins), ("iv", iv, 4, n_ins), ("iw", iw, 8, n_ins),
            ("du", du, 4, n_del), ("dv", dv, 4, n_del), ("s", s, 2, n_ins + n_del),
            ("L", L, 2, n_ins + n_del))
    for name, t, size, n in want:
        if t is None or isinstance(t, int):
            continue
        if t.element_size() != size:
            raise ValueError(f"{name}: {size}-byte elements expected, got {t.dtype}")
        if int(t.numel()) != n:
            raise ValueError(f"{name}: {n} entries expected, got {int(t.numel())}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if on_gpu and not t.is_cuda:
            raise ValueError(f"{name} must be in GPU memory")
    if not iw.is_floating_point():
        raise ValueError(f"iw: float64 expected, got {iw.dtype}")
    if results is not None and not isinstance(results, int):
        if int(results.numel()) * results.element_size() < 24 * (n_ins + n_del):
            raise ValueError(f"results: {24 * (n_ins + n_del)} bytes needed")
        if not results.is_contiguous():
            raise ValueError("results must be contiguous")
        if on_gpu and not results.is_cuda:
            raise ValueError("results must be in GPU memory")


def _dev_batch(iu, iv, iw, du, dv, s, L, L_max, s_max, results, stream):
    check_dev_batch(iu, iv, iw, du, dv, s=s, L=L, results=results)

    def addr(t):
        if t is None:
            return None
        return t if isinstance(t, int) else t.data_ptr()

    def count(t):
        return 0 if t is None else int(t.numel())

    b = dyg_batch_dev(n_ins=count(iu), n_del=count(du), iu=addr(iu), iv=addr(iv), iw=addr(iw),
                      du=addr(du), dv=addr(dv), s=addr(s), L=addr(L), L_max=int(L_max),
                      s_max=int(s_max), results=addr(results))
    handle = None
    if stream is not None:
        handle = stream if isinstance(stream, int) else stream.cuda_stream
    return b, handle


def dyg_apply_batch_dev(ctx, iu, iv, iw, du, dv, s=None, L=None, L_max=0, s_max=0,
                        results=None, stream=None):
    """Device-resident batch: iu, iv, iw, du, dv are torch tensors on the GPU
    (checked by check_dev_batch); s, L and results are tensors or raw device
    addresses as ints; stream is a torch stream or a raw handle."""
    b, handle = _dev_batch(iu, iv, iw, du, dv, s, L, L_max, s_max, results, stream)
    _check(_lib.dyg_apply_batch_dev(ctx, C.byref(b), handle), "dyg_apply_batch_dev")


def dyg_apply_batch_dev_static(ctx, iu, iv, iw, du, dv, s=None, L=None, L_max=0, s_max=0,
                               results=None, stream=None):
    """dyg_apply_batch_dev whose working memory is the library's static device
    array (no allocation); the same arguments.  Sync the context's previous
    batch first."""
    b, handle = _dev_batch(iu, iv, iw, du, dv, s, L, L_max, s_max, results, stream)
    _check(_lib.dyg_apply_batch_dev_static(ctx, C.byref(b), handle),
           "dyg_apply_batch_dev_static")


def dyg_initial_sparsifier(n, rowptr, col, w, n_extra, seed):
    """H(0) of the CSR graph (maximum spanning forest + n_extra keyed off-tree
    edges, computed on the GPU): (h_u, h_v) in canonical order."""
    rowptr = _arr(rowptr, np.uint64)
    col = _arr(col, np.uint32)
    w = _arr(w, np.float64)
    m = C.c_uint64(0)
    _check(_lib.dyg_initial_sparsifier(int(n), _ptr(rowptr), _ptr(col), _ptr(w), int(n_extra),
                                       int(seed), 0, C.byref(m), None, None),
           "dyg_initial_sparsifier")
    u = np.zeros(max(m.value, 1), np.uint32)
    v = np.zeros(max(m.value, 1), np.uint32)
    cnt = m.value
    _check(_lib.dyg_initial_sparsifier(int(n), _ptr(rowptr), _ptr(col), _ptr(w), int(n_extra),
                                       int(seed), cnt, C.byref(m), _ptr(u), _ptr(v)),
           "dyg_initial_sparsifier")
    return u[:m.value], v[:m.value]


def dyg_sync(ctx):
    _check(_lib.dyg_sync(ctx), "dyg_sync")


def _query(fn, ctx):
    m = C.c_uint64(0)
    _check(fn(ctx, 0, C.byref(m), None, None, None), "query")
    u = np.zeros(m.value, np.uint32)
    v = np.zeros(m.value, np.uint32)
    w = np.zeros(m.value, np.float64)
    _check(fn(ctx, m.value, C.byref(m), _ptr(u), _ptr(v), _ptr(w)), "query")
    return u, v, w


def dyg_query_sparsifier(ctx):
    return _query(_lib.dyg_query_sparsifier, ctx)


def dyg_query_graph(ctx):
    return _query(_lib.dyg_query_graph, ctx)


def dyg_stats(ctx) -> dict:
    st = dyg_stats_t()
    _check(_lib.dyg_stats(ctx, C.byref(st)), "dyg_stats")
    return {name: getattr(st, name) for name, _ in dyg_stats_t._fields_ if "reserved" not in name}


def dyg_check_state(ctx) -> str:
    """'' if the device state is consistent, else a description of the first
    violation."""
    buf = C.create_string_buffer(512)
    rc = _lib.dyg_check_state(ctx, buf, 512)
    if rc == 0:
        return ""
    return buf.value.decode() or STATUS.get(rc, str(rc))


def dyg_get_tuning(ctx) -> dict:
    t = dyg_tuning()
    _check(_lib.dyg_get_tuning(ctx, C.byref(t)), "dyg_get_tuning")
    return {"walk_blocks_per_cu": t.walk_blocks_per_cu, "refill_min": t.refill_min,
            "updates_per_wave": t.updates_per_wave, "tail_lanes": t.tail_lanes,
            "lockstep": t.lockstep}


def dyg_set_tuning(ctx, walk_blocks_per_cu: int, refill_min: int, updates_per_wave: int = None,
                   tail_lanes: int = None, lockstep: int = None):
    """Fields left as None keep their current values."""
    cur = dyg_tuning()
    _check(_lib.dyg_get_tuning(ctx, C.byref(cur)), "dyg_get_tuning")
    t = dyg_tuning(walk_blocks_per_cu=int(walk_blocks_per_cu), refill_min=int(refill_min),
                   updates_per_wave=int(cur.updates_per_wave if updates_per_wave is None
                                        else updates_per_wave),
                   tail_lanes=int(cur.tail_lanes if tail_lanes is None else tail_lanes),
                   lockstep=int(cur.lockstep if lockstep is None else lockstep))
    _check(_lib.dyg_set_tuning(ctx, C.byref(t)), "dyg_set_tuning")


def dyg_compact(ctx):
    _check(_lib.dyg_compact(ctx), "dyg_compact")


def dyg_reserve(ctx, max_ins: int, max_del: int, max_s: int = 0, max_L: int = 0):
    _check(_lib.dyg_reserve(ctx, int(max_ins), int(max_del), int(max_s), int(max_L)),
           "dyg_reserve")


def dyg_destroy(ctx):
    _lib.dyg_destroy(ctx)


# --------------------------------------------------------------------------


class Dygrass:
    """One device-resident (G, H) pair."""

    def __init__(self, n, rowptr, col, w, h_u, h_v, *, seed, K=math.inf, s=64, L=32, Q=24,
                 w_ref=0.0, dead_end=DEAD_END_TERMINATE, slack=0.5, uid_base=0, flags=0):
        self.params = dyg_default_params(seed=int(seed), K=float(K), s_default=int(s),
                                         L_default=int(L), Q=int(Q), w_ref=float(w_ref),
                                         dead_end=int(dead_end), slack=float(slack),
                                         uid_base=int(uid_base), flags=int(flags))
        self.n = int(n)
        self.ctx = dyg_init(n, rowptr, col, w, h_u, h_v, self.params)

    def apply_batch(self, iu, iv, iw, du, dv, s=None, L=None, walkers=False):
        return dyg_apply_batch(self.ctx, iu, iv, iw, du, dv, s=s, L=L, walkers=walkers,
                               s_default=self.params.s_default)

    def apply_batch_dev(self, *args, **kw):
        return dyg_apply_batch_dev(self.ctx, *args, **kw)

    def sync(self):
        dyg_sync(self.ctx)

    def query(self, which="H"):
        return dyg_query_sparsifier(self.ctx) if which == "H" else dyg_query_graph(self.ctx)

    def stats(self):
        return dyg_stats(self.ctx)

    def check_state(self) -> str:
        return dyg_check_state(self.ctx)

    def compact(self):
        dyg_compact(self.ctx)

    def close(self):
        if self.ctx is not None and self.ctx.value:
            dyg_destroy(self.ctx)
        self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# serving


def dyg_server_default_params(**overrides) -> dyg_server_params:
    p = dyg_server_params()
    _lib.dyg_server_default_params(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


class DygServer:
    """Continuous batching over many resident graphs (dyg_server_*).

    submit() queues a batch of one graph and returns its request id; poll()
    launches rounds and returns finished requests as dicts; results of a
    request (a structured array of n_ins+n_del records) are complete once it
    is reported."""

    def __init__(self, mem_budget=8 << 30, max_fused=32, max_inflight=2, walk_blocks_per_cu=4):
        self.params = dyg_server_default_params(mem_budget=int(mem_budget),
                                                max_fused=int(max_fused),
                                                max_inflight=int(max_inflight),
                                                walk_blocks_per_cu=int(walk_blocks_per_cu))
        self.h = C.c_void_p()
        _check(_lib.dyg_server_create(C.byref(self.h), C.byref(self.params)), "dyg_server_create")
        self._keep = {}  # request id -> arrays the server writes or reads until done
        self._done = (dyg_request_done * 1024)()

    def add_graph(self, ctx: "Dygrass") -> int:
        gid = C.c_uint32(0)
        _check(_lib.dyg_server_add_graph(self.h, ctx.ctx, C.byref(gid)), "dyg_server_add_graph")
        return int(gid.value)

    def submit(self, graph_id, iu, iv, iw, du, dv, results=True) -> int:
        iu = _arr(iu, np.uint32)
        iv = _arr(iv, np.uint32)
        iw = _arr(iw, np.float64)
        du = _arr(du, np.uint32)
        dv = _arr(dv, np.uint32)
        _check_host_batch(iu, iv, iw, du, dv)
        res = np.zeros(iu.size + du.size, UPDATE_RESULT_DTYPE) if results else None
        rid = C.c_uint64(0)
        _check(_lib.dyg_server_submit(self.h, int(graph_id), iu.size, _ptr(iu), _ptr(iv),
                                      _ptr(iw), du.size, _ptr(du), _ptr(dv), _ptr(res),
                                      C.byref(rid)), "dyg_server_submit")
        self._keep[int(rid.value)] = res
        return int(rid.value)

    def poll(self):
        n = C.c_uint32(0)
        _check(_lib.dyg_server_poll(self.h, self._done, len(self._done), C.byref(n)),
               "dyg_server_poll")
        out = []
        for i in range(n.value):
            d = self._done[i]
            rid = int(d.request_id)
            out.append(dict(request_id=rid, graph_id=int(d.graph_id), status=int(d.status),
                            n_updates=int(d.n_updates), t_submit=d.t_submit,
                            t_start=d.t_start, t_done=d.t_done,
                            results=self._keep.pop(rid, None)))
        return out

    @property
    def pending(self) -> int:
        return int(_lib.dyg_server_pending(self.h))

    def now(self) -> float:
        return float(_lib.dyg_server_now(self.h))

    def drain(self, sleep_s=0.0):
        import time

        out = []
        while self.pending:
            out += self.poll()
            if sleep_s:
                time.sleep(sleep_s)
        return out

    def close(self):
        if self.h is not None and self.h.value:
            _lib.dyg_server_destroy(self.h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
