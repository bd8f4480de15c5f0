"""Gradient of L = ||u - u_t||^2 where A(G) u = B f.

A depends on the geometric factors G through the local operator
sum_ab D_a^T G_ab D_b; B is the assembled diagonal mass. With the adjoint
lambda = A^{-1} 2 (u - u_t) (A is symmetric, so the adjoint operator is A):
  dL/df            = B lambda,
  dL/dG_aa(node)   = -(D_a lambda_L)(D_a u_L),
  dL/dG_ab(node)   = -[(D_a lambda_L)(D_b u_L) + (D_b lambda_L)(D_a u_L)]  (a != b,
                     the symmetric pair is stored once),
where lambda_L, u_L are the element-local copies Q R^T lambda, Q R^T u.
"""
from __future__ import annotations

import numpy as np

from .sem import SemBox, grad_local, _comp


def contract(box: SemBox, lam: np.ndarray, u: np.ndarray) -> np.ndarray:
    """dL/dG given the adjoint lam and the state u (global vectors); shape of box.G."""
    gl = grad_local(box.D, box.scatter(lam))
    gu = grad_local(box.D, box.scatter(u))
    out = np.empty_like(box.G)
    for a in range(3):
        for b in range(a, 3):
            if a == b:
                out[:, _comp(a, b)] = -gl[a] * gu[a]
            else:
                out[:, _comp(a, b)] = -(gl[a] * gu[b] + gl[b] * gu[a])
    return out


def loss_and_grad(box: SemBox, solve, f: np.ndarray, u_t: np.ndarray, G=None):
    """(L, u, dL/df, dL/dG). `solve(b, G)` returns A(G)^{-1} b."""
    B = box.mass()
    u = solve(B * f, G)
    res = u - u_t
    L = float(np.dot(res, res))
    lam = solve(2.0 * res, G)
    return L, u, B * lam, contract(box, lam, u)
