"""Dense spectral quantities on tiny graphs (test infrastructure only).

* Laplacian L = D - A (Sec. II-A).
* Effective resistance R_eff(p,q) = b_pq^T L^+ b_pq (Definition 1, Eq. 2).
* Relative condition number kappa(L_G, L_H) from the generalized eigenvalues
  of the pencil (L_G, L_H) restricted to the complement of the all-ones
  vector (Sec. II-A, Eq. 1; Sec. III-B, Eqs. 6-11).
* The K-eigenvalue spectral distortion Delta_K of Lemma 3.2 (Eq. 5).

Everything is plain numpy/scipy dense linear algebra, O(n^3): use on graphs
of a few hundred vertices at most.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def laplacian(n: int, u, v, w) -> np.ndarray:
    Lm = np.zeros((n, n))
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    np.add.at(Lm, (u, v), -w)
    np.add.at(Lm, (v, u), -w)
    np.add.at(Lm, (u, u), w)
    np.add.at(Lm, (v, v), w)
    return Lm


def effective_resistance(Lm: np.ndarray, p: int, q: int) -> float:
    b = np.zeros(Lm.shape[0])
    b[p] = 1.0
    b[q] = -1.0
    return float(b @ np.linalg.pinv(Lm, rcond=1e-12, hermitian=True) @ b)


def _reduced(Lm: np.ndarray) -> np.ndarray:
    """Project onto the complement of the all-ones vector (connected graphs)."""
    n = Lm.shape[0]
    # orthonormal basis of 1-perp
    Qm = sla.null_space(np.ones((1, n)))
    return Qm.T @ Lm @ Qm


def generalized_eigs(LG: np.ndarray, LH: np.ndarray) -> np.ndarray:
    """Eigenvalues of L_H^+ L_G on 1-perp (both graphs connected)."""
    A = _reduced(LG)
    B = _reduced(LH)
    return np.sort(sla.eigh(A, B, eigvals_only=True))


def relative_condition_number(LG: np.ndarray, LH: np.ndarray) -> float:
    lam = generalized_eigs(LG, LH)
    return float(lam[-1] / lam[0])


def spectral_distortion(LH: np.ndarray, p: int, q: int, w: float, K: int | None = None) -> float:
    """Delta_K = sum_{i=2..K} w (u_i^T b)^2 / lambda_i over the eigenpairs of L_H
    (Lemma 3.1 and Lemma 3.2); K=None uses all nonzero eigenpairs."""
    lam, U = np.linalg.eigh(LH)
    b = np.zeros(LH.shape[0])
    b[p] = 1.0
    b[q] = -1.0
    order = np.argsort(lam)
    lam, U = lam[order], U[:, order]
    last = LH.shape[0] if K is None else K
    tot = 0.0
    for i in range(1, last):  # skip the zero eigenvalue (connected graph)
        tot += w * (U[:, i] @ b) ** 2 / lam[i]
    return float(tot)
