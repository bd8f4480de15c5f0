"""Multigrid V-cycles (paper, Sec. 2).

The V-cycle on level j (eq. recursive-v-cycle-err-prop, with M_l^{-1} = A_l^{-1}
on the coarsest level l):

  1. j == l: return A_l^{-1} b;
  2. pre-smooth from a zero guess: x = Cheb_m(b, 0);
  3. residual r = b - A_j x;
  4. coarse-grid correction x += P V_{j+1}(P^T r);
  5. post-smooth x = Cheb_n(b, x) (symmetric cycle; the one-sided cycle of eq.
     recursive-ftc-err has n = 0 and m = 2k).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import chebyshev as cheb
from .sem import SemBox, SemTransfer
from .lanczos import lambda_max_SA


@dataclass
class Level:
    A: Callable[[np.ndarray], np.ndarray]
    Sinv: object              # diag(A)^{-1} (array), or a Schwarz smoother (callable)
    n: int
    lmax: float = 0.0         # lambda_max(S A)
    applies: int = 0          # operator applications performed on this level

    def apply(self, x):
        self.applies += 1
        return self.A(x)


@dataclass
class Hierarchy:
    levels: List[Level]
    prolong: List[Callable]   # prolong[j]: level j+1 -> level j
    restrict: List[Callable]  # restrict[j]: level j -> level j+1
    coarse_solve: Callable
    kind: str
    pre: int
    post: int
    extra: dict = field(default_factory=dict)

    def vcycle(self, b: np.ndarray, j: int = 0) -> np.ndarray:
        if j == len(self.levels) - 1:
            return self.coarse_solve(b)
        lev = self.levels[j]
        if self.pre > 0:
            x = cheb.smooth(self.kind, self.pre, lev.apply, lev.Sinv, lev.lmax, b, None)
            r = b - lev.apply(x)
        else:
            x = np.zeros_like(b)
            r = b.copy()
        x = x + self.prolong[j](self.vcycle(self.restrict[j](r), j + 1))
        if self.post > 0:
            x = cheb.smooth(self.kind, self.post, lev.apply, lev.Sinv, lev.lmax, b, x)
        return x

    def reset_counters(self):
        for lev in self.levels:
            lev.applies = 0


def exact_coarse(Ac: sp.spmatrix) -> Callable:
    """Exact solve with the assembled coarse matrix (sparse LU)."""
    lu = spla.splu(sp.csc_matrix(Ac))
    return lambda b: lu.solve(b)


def default_orders(N: int) -> list:
    """Schedule N -> floor(N/2) -> 1, duplicates removed."""
    out = [N]
    for o in (N // 2, 1):
        if o < out[-1] and o >= 1:
            out.append(o)
    return out


def lambda_max_nonsym(A, S, n: int) -> float:
    """Largest real part of the eigenvalues of S A for a non-symmetric smoother S (the
    Schwarz smoothers; Sec. 4.1 notes that their spectra have small imaginary parts),
    from the dense matrix S A."""
    SA = np.column_stack([S(A(e)) for e in np.eye(n)])
    return float(np.max(np.linalg.eigvals(SA).real))


def sem_hierarchy(verts, N: int, kind: str, pre: int, post: int, orders=None,
                  lmax=None, lanczos_seed: int = 7, schwarz: str | None = None) -> Hierarchy:
    """p-multigrid hierarchy with rediscretised SEM levels on the same vertices.

    lmax: optional list of lambda_max(S_j A_j) per smoothed level; otherwise
    each is estimated (dense eigensolve for small levels, Lanczos otherwise).
    schwarz: None for Jacobi smoothing, "asm" or "ras" for the Schwarz smoothers of
    Sec. 4.1 (eq. asm) inside the same Chebyshev algorithms; their lambda_max is
    estimated densely (small problems only) unless given.
    """
    from .schwarz import SchwarzLevel
    orders = default_orders(N) if orders is None else list(orders)
    boxes = [SemBox(verts, o) for o in orders]
    levels = []
    for j, bx in enumerate(boxes):
        smoothed = j < len(boxes) - 1
        S = SchwarzLevel(bx, schwarz) if (schwarz and smoothed) else 1.0 / bx.diag()
        lev = Level(A=bx.apply, Sinv=S, n=bx.n)
        if smoothed:
            if lmax is not None:
                lev.lmax = float(lmax[j])
            elif schwarz:
                lev.lmax = lambda_max_nonsym(bx.apply, S, bx.n)
            else:
                lev.lmax = lambda_max_SA(bx.apply, lev.Sinv, bx.n, seed=lanczos_seed)
        levels.append(lev)
    tr = [SemTransfer(boxes[j], boxes[j + 1]) for j in range(len(boxes) - 1)]
    coarse = exact_coarse(boxes[-1].assemble())
    return Hierarchy(levels=levels, prolong=[t.prolong for t in tr],
                     restrict=[t.restrict for t in tr], coarse_solve=coarse,
                     kind=kind, pre=pre, post=post, extra={"boxes": boxes, "orders": orders})
