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


def fgmres(A, b: np.ndarray, M, tol: float = 1e-8, restart: int = 30,
           maxit: int = 500) -> SolveResult:
    """Restarted flexible GMRES(m) with classical Gram-Schmidt (paper, Sec. 6.1: GMRES(m)
    with classical Gram-Schmidt needs two reductions per iteration).

    Right preconditioning in the flexible form (the preconditioned directions z_j = M(v_j)
    are kept, so M may be non-symmetric or vary between applications). x0 = 0. One cycle:
      r = b - A x, beta = ||r||, v_0 = r / beta, g = beta e_0;
      for j = 0 .. m-1:
        z_j = M(v_j), w = A z_j,
        h_ij = v_i . w for all i <= j at once (classical Gram-Schmidt),
        w -= sum_i h_ij v_i, h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j},
        Givens rotations G_0 .. G_{j-1} applied to column j, then the rotation G_j that
        annihilates h_{j+1,j}; it also maps g, and |g_{j+1}| is ||b - A x_j||;
        stop when |g_{j+1}| <= tol ||b||;
      x += Z y with R y = g (R: the rotated, upper triangular H).
    history holds ||b|| and then |g_{j+1}| after every iteration (over all cycles).
    A rotation with c = h_jj / d, s = h_{j+1,j} / d, d = sqrt(h_jj^2 + h_{j+1,j}^2).
    """
    n = b.shape[0]
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    hist = [bnorm]
    if bnorm == 0.0:
        return SolveResult(x, 0, True, hist)
    it = 0
    while True:
        r = b - A(x) if it > 0 else b.copy()
        beta = float(np.linalg.norm(r))
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        done = False
        for j in range(restart):
            Z[j] = M(V[j])
            w = A(Z[j])
            h = V[: j + 1] @ w                       # reduction 1: all projections
            w = w - h @ V[: j + 1]
            hn = float(np.linalg.norm(w))            # reduction 2
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0.0:
                V[j + 1] = w / hn
            for i in range(j):                       # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = float(np.sqrt(H[j, j] * H[j, j] + H[j + 1, j] * H[j + 1, j]))
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(float(g[j + 1])))
            if abs(g[j + 1]) <= tol * bnorm or hn == 0.0:
                done = True
                break
            if it >= maxit:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):               # back substitution R y = g
            y[i] = (g[i] - H[i, i + 1: k] @ y[i + 1: k]) / H[i, i]
        x = x + y @ Z[:k]
        if done:
            return SolveResult(x, it, True, hist)
        if it >= maxit:
            return SolveResult(x, it, False, hist)


def mg_solver(A, b: np.ndarray, M, tol: float = 1e-6, maxit: int = 500) -> SolveResult:
    """Multigrid as the solver (paper, Sec. 3, where its observed convergence rate is set
    against Lemma multilevel-poly-bound): the stationary iteration
        x_i = x_{i-1} + M(b - A x_{i-1}),  x_0 = 0,
    with M one V-cycle. The residual b - A x_i is formed from the iterate every time;
    history holds ||b|| and ||b - A x_i||; stop when ||b - A x_i|| <= tol ||b||. The error
    obeys e_i = (I - M A) e_{i-1}, so the average rate of eq. avg-convergence-rate tends
    to the spectral radius of I - M A."""
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = float(np.linalg.norm(b))
    hist = [bnorm]
    if bnorm == 0.0:
        return SolveResult(x, 0, True, hist)
    for it in range(1, maxit + 1):
        x = x + M(r)
        r = b - A(x)
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if rn <= tol * bnorm:
            return SolveResult(x, it, True, hist)
    return SolveResult(x, maxit, False, hist)
