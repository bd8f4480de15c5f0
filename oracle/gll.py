"""Gauss-Lobatto-Legendre (GLL) points, weights and the nodal derivative matrix.

The paper defers the spectral-element details to its reference on tuning
(Sec. 5, "High Order Cases"); these are the standard definitions:

* nodes: -1, 1 and the N-1 roots of L_N' (L_N the Legendre polynomial);
* weights: w_i = 2 / (N (N+1) L_N(x_i)^2);
* derivative of the Lagrange basis at the nodes:
  D_ij = L_N(x_i) / (L_N(x_j) (x_i - x_j)) for i != j,
  D_00 = -N(N+1)/4, D_NN = N(N+1)/4, otherwise 0.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as _leg


def legendre(N: int, x):
    """L_N(x)."""
    c = np.zeros(N + 1)
    c[N] = 1.0
    return _leg.legval(x, c)


def gll_nodes_weights(N: int):
    """GLL nodes (ascending) and weights for polynomial order N >= 1."""
    if N < 1:
        raise ValueError("N must be >= 1")
    c = np.zeros(N + 1)
    c[N] = 1.0
    dc = _leg.legder(c)
    if N == 1:
        inner = np.zeros(0)
    else:
        inner = np.sort(np.real(_leg.legroots(dc)))
        ddc = _leg.legder(dc)
        for _ in range(5):  # Newton polish of L_N'(x) = 0
            inner = inner - _leg.legval(inner, dc) / _leg.legval(inner, ddc)
    x = np.concatenate([[-1.0], inner, [1.0]])
    LN = legendre(N, x)
    w = 2.0 / (N * (N + 1) * LN ** 2)
    return x, w


def derivative_matrix(N: int) -> np.ndarray:
    """D[i, j] = d l_j / dx at x_i for the GLL Lagrange basis of order N."""
    x, _ = gll_nodes_weights(N)
    LN = legendre(N, x)
    D = np.zeros((N + 1, N + 1))
    for i in range(N + 1):
        for j in range(N + 1):
            if i != j:
                D[i, j] = LN[i] / (LN[j] * (x[i] - x[j]))
    D[0, 0] = -N * (N + 1) / 4.0
    D[N, N] = N * (N + 1) / 4.0
    return D


def lagrange_eval(nodes: np.ndarray, x) -> np.ndarray:
    """Matrix M[p, j] = l_j(x_p) for the Lagrange basis through `nodes` (product formula)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    M = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                M[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return M


def interpolation_matrix(Nc: int, Nf: int) -> np.ndarray:
    """J[i, j] = l_j^{(Nc)}(x_i^{(Nf)}): coarse GLL basis evaluated at the fine GLL nodes."""
    xc, _ = gll_nodes_weights(Nc)
    xf, _ = gll_nodes_weights(Nf)
    return lagrange_eval(xc, xf)
