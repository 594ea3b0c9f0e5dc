"""Sparsifier quality at mid scale (test infrastructure only).

* Off-tree density d_H = |E_H| / |V| - 1, the density measure of the
  experiments (Sec. IV).
* Relative condition number kappa(L_G, L_H) = lambda_max / lambda_min of the
  pencil (L_G, L_H) on the complement of the all-ones vector (Sec. II-A,
  Eq. 1), for connected graphs of up to ~10^5 vertices: both Laplacians are
  grounded at one vertex (its row and column removed).  Every class x + c*1
  holds exactly one vector that is zero at that vertex, and the Rayleigh
  quotient x^T L_G x / x^T L_H x does not depend on c, so the grounded pencil
  (SPD on both sides) has the same eigenvalues.  lambda_max comes from ARPACK
  on (L_G, L_H), lambda_min as 1 / lambda_max of (L_H, L_G).
* Preconditioned conjugate gradients on L_G x = b with L_H as the
  preconditioner, stopped once the relative residual ||b - L_G x|| / ||b||
  falls below 1e-8 (Sec. IV, Table IV): the iteration count follows
  sqrt(kappa(L_G, L_H)).  Textbook PCG, both Laplacians grounded as above,
  the preconditioner applied through a sparse LU of grounded L_H.
* The trend of Tables II, III and IV on a synthetic stream: an insertion stream
  applied three ways -- H left alone, every inserted edge added to H (no
  filter), and the update rule of Algorithm 1 through the CPU oracle, both
  batched (updates applied at the end of each batch, Sec. III-F) and
  sequential (each update its own batch, so every one sees the previous
  ones, as in the per-update loop of Algorithm 1) -- with d_H, kappa and the
  PCG iteration count after the stream.

Plain scipy sparse linear algebra; shares nothing with the GPU library.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla


def off_tree_density(n: int, m_h: int) -> float:
    """d_H = |E_H| / |V| - 1 (Sec. IV)."""
    return m_h / n - 1.0


def grounded_laplacian(n: int, u, v, w, root: int = 0) -> sp.csc_matrix:
    """L = D - A (Sec. II-A) with row and column `root` removed."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    rows = np.concatenate([u, v, u, v])
    cols = np.concatenate([v, u, u, v])
    vals = np.concatenate([-w, -w, w, w])
    Lm = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    keep = np.flatnonzero(np.arange(n) != root)
    return Lm[keep][:, keep].tocsc()


def _lambda_max(A: sp.csc_matrix, B: sp.csc_matrix) -> float:
    """Largest eigenvalue of A x = lambda B x, A and B SPD."""
    lu = sla.splu(B)
    vals = sla.eigsh(A, k=1, M=B, Minv=sla.LinearOperator(B.shape, matvec=lu.solve),
                     which="LA", tol=1e-10, return_eigenvectors=False)
    return float(vals[0])


def pencil_extremes(n: int, G, H) -> tuple[float, float]:
    """(lambda_min, lambda_max) of the pencil (L_G, L_H), G and H given as
    (u, v, w) edge lists of connected graphs on the same n vertices."""
    LG = grounded_laplacian(n, *G)
    LH = grounded_laplacian(n, *H)
    lam_max = _lambda_max(LG, LH)
    lam_min = 1.0 / _lambda_max(LH, LG)
    return lam_min, lam_max


def relative_condition_number(n: int, G, H) -> float:
    lam_min, lam_max = pencil_extremes(n, G, H)
    return lam_max / lam_min


def pcg_iterations(n: int, G, H, b=None, rtol: float = 1e-8, max_iter: int = 100_000,
                   seed: int = 0) -> tuple[int, np.ndarray]:
    """Iterations of PCG on grounded L_G x = b preconditioned by grounded L_H
    until ||r|| <= rtol ||b|| (Sec. IV); returns (iterations, x).  b defaults
    to a seeded standard normal vector."""
    A = grounded_laplacian(n, *G).tocsr()
    P = sla.splu(grounded_laplacian(n, *H))
    if b is None:
        b = np.random.default_rng(seed).standard_normal(n - 1)
    x = np.zeros(n - 1)
    r = b.copy()
    z = P.solve(r)
    p = z.copy()
    rz = r @ z
    stop = rtol * np.linalg.norm(b)
    for it in range(1, max_iter + 1):
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        if np.linalg.norm(r) <= stop:
            return it, x
        z = P.solve(r)
        rz_next = r @ z
        p = z + (rz_next / rz) * p
        rz = rz_next
    raise RuntimeError("PCG did not converge")


def stream_trend(wl, K: float | None = None, s: int | None = None, L: int | None = None,
                 w_ref: float = 0.0):
    """d_H, kappa(L_G, L_H) and PCG iterations before and after an
    insertion-only stream, for H left alone, H given every insertion, and H
    updated by the oracle with threshold K (by default kappa of the initial
    pair, the distortion bound of Eq. 11), batched and one update per batch
    ("sequential").  w_ref is the oracle's reference weight (0: its default;
    a huge one quantises every weight to 1, i.e. unweighted selection).
    Returns a dict of (d_H, kappa, iterations) triples; the
    initial one is taken against G before the stream, the others against G
    after it."""
    import oracle
    from paper_2505_02741_amd import workloads as W

    n = wl.G.n
    G0 = (wl.G.u, wl.G.v, wl.G.w)
    H0 = (wl.hu, wl.hv, wl.G.w[wl.h_mask])
    kappa0 = relative_condition_number(n, G0, H0)
    K = kappa0 if K is None else K
    iu = np.concatenate([b.iu for b in wl.batches]).astype(np.int64)
    iv = np.concatenate([b.iv for b in wl.batches]).astype(np.int64)
    iw = np.concatenate([b.iw for b in wl.batches])
    if any(b.n_del for b in wl.batches):
        raise ValueError("stream_trend takes insertion-only streams")
    G1 = (np.concatenate([G0[0], iu]), np.concatenate([G0[1], iv]), np.concatenate([G0[2], iw]))
    rp, col, w = W.to_csr(n, *G0)
    o = oracle.Oracle(n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, K=K,
                      s=wl.s if s is None else s, L=wl.L if L is None else L, w_ref=w_ref)
    try:
        for b in wl.batches:
            o.apply_batch(b.iu, b.iv, b.iw, b.du, b.dv, s=b.s, L=b.L)
        Hd = o.query("H")
    finally:
        o.close()
    Ha = (np.concatenate([H0[0], iu]), np.concatenate([H0[1], iv]), np.concatenate([H0[2], iw]))
    out = {"initial": (off_tree_density(n, H0[0].size), kappa0, pcg_iterations(n, G0, H0)[0])}
    for name, H in (("no_update", H0), ("no_filter", Ha), ("dygrass", Hd)):
        out[name] = (off_tree_density(n, np.asarray(H[0]).size),
                     relative_condition_number(n, G1, H), pcg_iterations(n, G1, H)[0])
    # sequential semantics: the same updates, one per batch
    o = oracle.Oracle(n, rp, col, w, wl.hu, wl.hv, seed=wl.seed_walk, K=K,
                      s=wl.s if s is None else s, L=wl.L if L is None else L, w_ref=w_ref)
    try:
        z = np.zeros(0, np.uint32)
        for b in wl.batches:
            for i in range(b.n_ins):
                o.apply_batch(b.iu[i:i + 1], b.iv[i:i + 1], b.iw[i:i + 1], z, z,
                              s=None if b.s is None else b.s[i:i + 1],
                              L=None if b.L is None else b.L[i:i + 1])
        Hs = o.query("H")
    finally:
        o.close()
    out["sequential"] = (off_tree_density(n, Hs[0].size), relative_condition_number(n, G1, Hs),
                         pcg_iterations(n, G1, Hs)[0])
    out["K"] = K if math.isfinite(K) else float("inf")
    return out
