"""2D finite-difference Poisson with geometric multigrid (paper, Sec. 3).

Domain [0, Lx] x [0, Ly] with u = 0 on the boundary, a grid of (n+1) x (n+1)
points (n-1 interior unknowns per direction, x fastest), the 5-point operator
  (2/hx^2 + 2/hy^2) u_ij - (u_{i-1,j} + u_{i+1,j})/hx^2 - (u_{i,j-1} + u_{i,j+1})/hy^2.
Coarse grids have n_c = n/f intervals (f = 2 or 8, no semi-coarsening); coarse
point I coincides with fine point f*I. P is bilinear interpolation (1D hat
weights 1 - |i - f I| / f) and coarse operators are Galerkin,
A_{j+1} = P^T A_j P (eq. galerkin-coarse-grid).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import mg
from .lanczos import lambda_max_SA


def laplacian_5pt(n: int, Lx: float = 1.0, Ly: float = 1.0) -> sp.csr_matrix:
    m = n - 1
    hx, hy = Lx / n, Ly / n
    Tx = sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]) / hx ** 2
    Ty = sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]) / hy ** 2
    I = sp.identity(m)
    return (sp.kron(I, Tx) + sp.kron(Ty, I)).tocsr()


def bilinear_1d(n: int, f: int) -> sp.csr_matrix:
    """1D interpolation from n/f intervals to n intervals (interior points only)."""
    nc = n // f
    rows, cols, vals = [], [], []
    for I in range(1, nc):
        for i in range(max(1, f * I - f + 1), min(n - 1, f * I + f - 1) + 1):
            wgt = 1.0 - abs(i - f * I) / f
            if wgt > 0.0:
                rows.append(i - 1)
                cols.append(I - 1)
                vals.append(wgt)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n - 1, nc - 1))


def hierarchy_matrices(n: int, f: int, Lx: float = 1.0, Ly: float = 1.0,
                       coarsest_n: int = 2):
    """Operators and interpolations from n intervals down to coarsest_n intervals.

    Returns (As, Ps, ns) with As[j] the level-j operator, Ps[j] the
    interpolation level j+1 -> j and ns[j] the interval count of level j.
    """
    As = [laplacian_5pt(n, Lx, Ly)]
    Ps, ns = [], [n]
    while ns[-1] // f >= coarsest_n and ns[-1] % f == 0:
        nf = ns[-1]
        P1 = bilinear_1d(nf, f)
        P = sp.kron(P1, P1).tocsr()
        Ps.append(P)
        As.append((P.T @ As[-1] @ P).tocsr())
        ns.append(nf // f)
    return As, Ps, ns


def grid_complexity(As) -> float:
    """sum_j nnz(A_j) / nnz(A_0), eq. mg-cycle-complexity."""
    return sum(A.nnz for A in As) / As[0].nnz


def fd_hierarchy(n: int, f: int, kind: str, pre: int, post: int, Lx: float = 1.0,
                 Ly: float = 1.0, coarsest_n: int = 2, lmax=None) -> mg.Hierarchy:
    As, Ps, ns = hierarchy_matrices(n, f, Lx, Ly, coarsest_n)
    levels = []
    for j, A in enumerate(As):
        Sinv = 1.0 / A.diagonal()
        lev = mg.Level(A=(lambda x, A=A: A @ x), Sinv=Sinv, n=A.shape[0])
        if j < len(As) - 1:
            lev.lmax = float(lmax[j]) if lmax is not None else lambda_max_SA(
                lev.A, Sinv, A.shape[0])
        levels.append(lev)
    Ac = As[-1].toarray()
    Acinv = np.linalg.inv(Ac)
    return mg.Hierarchy(levels=levels,
                        prolong=[(lambda x, P=P: P @ x) for P in Ps],
                        restrict=[(lambda x, P=P: P.T @ x) for P in Ps],
                        coarse_solve=lambda b: np.linalg.solve(Ac, b),
                        kind=kind, pre=pre, post=post,
                        extra={"As": As, "Ps": Ps, "ns": ns, "Acinv": Acinv})
