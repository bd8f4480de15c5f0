"""Preconditioned conjugate gradients (paper, Sec. 6.1 compares CG and GMRES).

x0 = 0, r0 = b, z0 = M(r0), p0 = z0; per iteration:
  w = A p, alpha = (r . z) / (p . w), x += alpha p, r -= alpha w;
  stop when ||r||_2 / ||b||_2 <= tol (recurrence residual);
  z_new = M(r);
  beta = (r . z_new) / (r_old . z_old)                  (PCG, Fletcher-Reeves)
  beta = (z_new . (r - r_old)) / (r_old . z_old)        (flexible CG, Polak-Ribiere)
  p = z_new + beta p.
The flexible form tolerates a preconditioner that is not symmetric or not
fixed (the one-sided V-cycle, a reduced-precision V-cycle).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    converged: bool
    history: list = field(default_factory=list)

    @property
    def relres(self) -> float:
        return self.history[-1] / self.history[0] if self.history[0] > 0 else 0.0

    def avg_rate(self) -> float:
        """rho = exp(log(||r_N|| / ||r_0||) / N), paper eq. avg-convergence-rate."""
        if self.iterations == 0:
            return 0.0
        return float(np.exp(np.log(self.history[-1] / self.history[0]) / self.iterations))


def pcg(A, b: np.ndarray, M, tol: float = 1e-8, maxit: int = 500,
        flexible: bool = False) -> SolveResult:
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = float(np.linalg.norm(b))
    hist = [bnorm]
    if bnorm == 0.0:
        return SolveResult(x, 0, True, hist)
    z = M(r)
    p = z.copy()
    rz = float(np.dot(r, z))
    for it in range(1, maxit + 1):
        w = A(p)
        alpha = rz / float(np.dot(p, w))
        x = x + alpha * p
        r_old = r
        r = r - alpha * w
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if rn <= tol * bnorm:
            return SolveResult(x, it, True, hist)
        z = M(r)
        if flexible:
            beta = float(np.dot(z, r - r_old)) / rz
        else:
            beta = float(np.dot(r, z)) / rz
        rz = float(np.dot(r, z))
        p = z + beta * p
    return SolveResult(x, maxit, False, hist)
