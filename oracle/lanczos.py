"""Largest eigenvalue of S A (S = diag(A)^{-1}), needed by the Chebyshev smoothers.

The paper takes lambda_max as the largest eigenvalue of S_j A_j (Sec. 2) but
does not say how it is obtained. Here: the symmetric form
S^{1/2} A S^{1/2} (same spectrum) and plain Lanczos with full
re-orthogonalisation from a seeded random start, stopped when the largest Ritz
value changes by less than `tol` relative; small problems use a dense
eigensolver.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from workload import uniform_noise


def lambda_max_dense(Adense: np.ndarray, Sinv: np.ndarray) -> float:
    s = np.sqrt(Sinv)
    M = s[:, None] * Adense * s[None, :]
    return float(sla.eigvalsh(M)[-1])


def lambda_max_SA(A, Sinv: np.ndarray, n: int, seed: int = 7, tol: float = 1e-12,
                  maxit: int = 400, dense_limit: int = 600) -> float:
    """lambda_max(S A) for a symmetric operator A given as a callable."""
    if n <= dense_limit:
        Ad = np.column_stack([A(e) for e in np.eye(n)])
        return lambda_max_dense(Ad, Sinv)
    s = np.sqrt(Sinv)
    q = uniform_noise(n, seed)
    q /= np.linalg.norm(q)
    Q = [q]
    alpha, beta = [], []
    prev = None
    for it in range(maxit):
        w = s * A(s * Q[-1])
        a = float(np.dot(Q[-1], w))
        alpha.append(a)
        w = w - a * Q[-1] - (beta[-1] * Q[-2] if beta else 0.0)
        for v in Q:  # full re-orthogonalisation
            w = w - np.dot(v, w) * v
        b = float(np.linalg.norm(w))
        T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
        top = float(sla.eigvalsh(T)[-1])
        if prev is not None and abs(top - prev) <= tol * abs(top):
            return top
        prev = top
        if b == 0.0:
            return top
        beta.append(b)
        Q.append(w / b)
    return prev
