"""Smoother and cycle analysis quantities (paper, Sec. 2, Lemma multilevel-poly-bound).

* error polynomial p_k(lambda) of a smoother, obtained by running the smoother
  itself on a diagonal operator (S = I, lambda_max = 1, b = 0, x0 = 1);
* gamma = sup_{0 < lambda <= 1} lambda p^2 / (1 - p^2)  (eq. gamma-defn);
* V(C, k) = C / (C + gamma^{-1}(k))                      (eq. simple-multilevel-bound);
* the (m, n) objective of eq. optimal-mn and the critical C at which (2k, 0)
  beats (k, k);
* the approximation-property constant C_j (eq. C-def) as the largest
  eigenvalue of (A^{-1} - P A_c^{-1} P^T) v = C S v with S scaled so that
  rho(S A) = 1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.optimize as so

from . import chebyshev as cheb


def smoother_polynomial(kind: str, k: int, lam: np.ndarray) -> np.ndarray:
    """p_k(lam) for lambda_max = 1, by running the smoother on diag(lam)."""
    lam = np.asarray(lam, dtype=np.float64)
    if kind == "simple":
        raise ValueError("use simple_polynomial")
    A = lambda x: lam * x
    return cheb.smooth(kind, k, A, np.ones_like(lam), 1.0, np.zeros_like(lam), np.ones_like(lam))


def simple_polynomial(omega: float, k: int, lam):
    """(1 - omega lambda)^k, eq. simple-smoothing-iteration."""
    return (1.0 - omega * np.asarray(lam)) ** k


def gamma_inv_of(pfun) -> float:
    """1 / sup_{0<lam<=1} lam p(lam)^2 / (1 - p(lam)^2) for a scalar polynomial p."""
    def g(l):
        p = pfun(np.atleast_1d(l))
        return l * p ** 2 / (1.0 - p ** 2)
    lam = np.concatenate([np.geomspace(1e-7, 1e-2, 400), np.linspace(1e-2, 1.0, 20001)])
    vals = g(lam)
    i = int(np.argmax(vals))
    best = float(vals[i])
    lo = lam[max(i - 1, 0)]
    hi = lam[min(i + 1, len(lam) - 1)]
    if hi > lo:
        res = so.minimize_scalar(lambda l: -float(g(l)[0]), bounds=(lo, hi), method="bounded",
                                 options={"xatol": 1e-13})
        best = max(best, -float(res.fun))
    return 1.0 / best


def gamma_inv(kind: str, k: int) -> float:
    if k == 0:
        return 0.0
    return gamma_inv_of(lambda l: smoother_polynomial(kind, k, l))


def V(C: float, ginv: float) -> float:
    return C / (C + ginv)


def mn_objective(C: float, ginv_m: float, ginv_n: float) -> float:
    """C (g(m) + g(n)) + g(m) g(n): larger is better (eq. optimal-mn)."""
    return C * (ginv_m + ginv_n) + ginv_m * ginv_n


def critical_C(ginv_k: float, ginv_2k: float) -> float:
    """C above which (2k, 0) has the smaller bound than (k, k)."""
    return ginv_k ** 2 / (ginv_2k - 2.0 * ginv_k)


def approximation_constant(A: np.ndarray, P: np.ndarray, Ac: np.ndarray | None = None) -> float:
    """C of eq. C-def for dense A, interpolation P (Galerkin A_c by default), Jacobi S."""
    if Ac is None:
        Ac = P.T @ A @ P
    Sinv = 1.0 / np.diag(A)
    s = np.sqrt(Sinv)
    lmax = float(sla.eigvalsh(s[:, None] * A * s[None, :])[-1])
    S = Sinv / lmax  # rho(S A) = 1
    K = np.linalg.inv(A) - P @ np.linalg.solve(Ac, P.T)
    K = 0.5 * (K + K.T)
    # largest C with K v = C S v, S diagonal and positive
    t = 1.0 / np.sqrt(S)
    M = t[:, None] * K * t[None, :]
    return float(sla.eigvalsh(M)[-1])


def error_propagator(apply_M, A: np.ndarray) -> np.ndarray:
    """E = I - M^{-1} A, column by column (for tiny problems)."""
    n = A.shape[0]
    E = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        E[:, j] = e - apply_M(A[:, j])
    return E


def a_norm(E: np.ndarray, A: np.ndarray) -> float:
    """||E||_A = ||A^{1/2} E A^{-1/2}||_2."""
    w, U = sla.eigh(A)
    Ah = (U * np.sqrt(w)) @ U.T
    Aih = (U / np.sqrt(w)) @ U.T
    return float(np.linalg.norm(Ah @ E @ Aih, 2))
