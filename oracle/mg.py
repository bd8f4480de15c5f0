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
    # (pre, post) orders of individual levels, where they differ from (pre, post)
    level_orders: dict = field(default_factory=dict)

    def vcycle(self, b: np.ndarray, j: int = 0) -> np.ndarray:
        if j == len(self.levels) - 1:
            return self.coarse_solve(b)
        lev = self.levels[j]
        pre, post = self.level_orders.get(j, (self.pre, self.post))
        if pre > 0:
            x = cheb.smooth(self.kind, pre, lev.apply, lev.Sinv, lev.lmax, b, None)
            r = b - lev.apply(x)
        else:
            x = np.zeros_like(b)
            r = b.copy()
        x = x + self.prolong[j](self.vcycle(self.restrict[j](r), j + 1))
        if post > 0:
            x = cheb.smooth(self.kind, post, lev.apply, lev.Sinv, lev.lmax, b, x)
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


def trilinear_1d(m: int) -> sp.csr_matrix:
    """1D linear interpolation from the interior vertices of m/2 uniform intervals to those
    of m intervals: fine vertex 2I takes coarse vertex I, an odd fine vertex the mean of its
    two coarse neighbours (a boundary neighbour is a Dirichlet zero). Tensor products of it
    interpolate trilinearly."""
    mc = m // 2
    rows, cols, vals = [], [], []
    for I in range(1, mc):
        for d, wgt in ((-1, 0.5), (0, 1.0), (1, 0.5)):
            rows.append(2 * I + d - 1)
            cols.append(I - 1)
            vals.append(wgt)
    return sp.csr_matrix((vals, (rows, cols)), shape=(m - 1, mc - 1))


def q1_lattice_levels(box1: SemBox, dense_max: int):
    """Geometric multigrid on the order-1 (Q1) vertex lattice below the p-levels.

    The paper solves its order-1 level with one algebraic multigrid V-cycle (Sec. 4.1); on
    a structured box the vertex lattice coarsens geometrically: lattices of m, m/2, m/4, ...
    elements per direction, trilinear interpolation P_j (the Kronecker product of the 1D
    interpolations, x fastest) and Galerkin operators A_{j+1} = P_j^T A_j P_j (eq.
    galerkin-coarse-grid), until a level has at most dense_max unknowns or a direction can
    no longer be halved. Returns (As, Ps): As[0] is the assembled order-1 operator, Ps[j]
    interpolates level j+1 to level j."""
    As, Ps = [box1.assemble()], []
    m = [box1.mx, box1.my, box1.mz]
    while As[-1].shape[0] > dense_max and all(v % 2 == 0 and v >= 4 for v in m):
        Px, Py, Pz = (trilinear_1d(v) for v in m)
        P = sp.kron(Pz, sp.kron(Py, Px)).tocsr()
        Ps.append(P)
        As.append((P.T @ As[-1] @ P).tocsr())
        m = [v // 2 for v in m]
    return As, Ps


def sem_hierarchy(verts, N: int, kind: str, pre: int, post: int, orders=None,
                  lmax=None, lanczos_seed: int = 7, schwarz: str | None = None,
                  coarse: str = "exact", dense_max: int = 4096) -> Hierarchy:
    """p-multigrid hierarchy with rediscretised SEM levels on the same vertices.

    verts: box vertices (mz+1, my+1, mx+1, 3), or an unstructured conforming hexahedral
    mesh as a tuple (vertex_xyz, elem_vertices[, vertex_dirichlet]) (oracle.mesh).

    lmax: optional list of lambda_max(S_j A_j) per smoothed level; otherwise
    each is estimated (dense eigensolve for small levels, Lanczos otherwise).
    schwarz: None for Jacobi smoothing, "asm" or "ras" for the Schwarz smoothers of
    Sec. 4.1 (eq. asm) inside the same Chebyshev algorithms; their lambda_max is
    estimated densely (small problems only) unless given.
    coarse: "exact" solves the order-1 level exactly (M_l^{-1} = A_l^{-1}, Sec. 2);
    "lattice" continues the V-cycle below order 1 on the Q1 vertex lattice
    (q1_lattice_levels) with the same Jacobi-Chebyshev kind, smoothed symmetrically with
    (m, m), m = max(pre, post), on every lattice level (the order-1 level included), and
    solves only the last lattice level (at most dense_max unknowns) exactly. It equals
    "exact" when the order-1 level already has at most dense_max unknowns.
    """
    from .schwarz import SchwarzLevel
    orders = default_orders(N) if orders is None else list(orders)
    if isinstance(verts, tuple):   # unstructured mesh: (vertex_xyz, elem_vertices, vertex_dirichlet)
        from .mesh import SemMesh
        if coarse != "exact" or schwarz:
            raise ValueError("unstructured meshes use Jacobi smoothing and the exact order-1 solve")
        boxes = [SemMesh(verts[0], verts[1], o, verts[2] if len(verts) > 2 else None) for o in orders]
    else:
        boxes = [SemBox(verts, o) for o in orders]
    hAs, hPs = q1_lattice_levels(boxes[-1], dense_max) if coarse == "lattice" else ([None], [])
    nh = len(hPs)  # smoothed lattice levels (the order-1 level among them when nh > 0)
    nsm = len(boxes) - 1 + nh
    levels = []

    def add_level(Aop, S, n):
        lev = Level(A=Aop, Sinv=S, n=n)
        j = len(levels)
        if j < nsm:
            if lmax is not None:
                lev.lmax = float(lmax[j])
            elif isinstance(S, np.ndarray):   # Jacobi: S A is similar to a symmetric matrix
                lev.lmax = lambda_max_SA(Aop, S, n, seed=lanczos_seed)
            else:                             # a Schwarz smoother
                lev.lmax = lambda_max_nonsym(Aop, S, n)
        levels.append(lev)

    for j, bx in enumerate(boxes[:-1]):
        add_level(bx.apply, SchwarzLevel(bx, schwarz) if schwarz else 1.0 / bx.diag(), bx.n)
    prolong = [SemTransfer(boxes[j], boxes[j + 1]) for j in range(len(boxes) - 1)]
    restrict = [t.restrict for t in prolong]
    prolong = [t.prolong for t in prolong]
    if nh == 0:
        add_level(boxes[-1].apply, 1.0 / boxes[-1].diag(), boxes[-1].n)
        coarse_solve = exact_coarse(boxes[-1].assemble())
    else:
        for A in hAs[:-1]:
            add_level(lambda x, A=A: A @ x, 1.0 / A.diagonal(), A.shape[0])
        Ac = hAs[-1]
        add_level(lambda x, A=Ac: A @ x, 1.0 / Ac.diagonal(), Ac.shape[0])
        prolong += [(lambda x, P=P: P @ x) for P in hPs]
        restrict += [(lambda x, P=P: P.T @ x) for P in hPs]
        coarse_solve = exact_coarse(Ac)
    m = max(pre, post)
    lattice_orders = {j: (m, m) for j in range(len(boxes) - 1, nsm)} if nh else {}
    return Hierarchy(levels=levels, prolong=prolong, restrict=restrict, coarse_solve=coarse_solve,
                     kind=kind, pre=pre, post=post, level_orders=lattice_orders,
                     extra={"boxes": boxes, "orders": orders, "lattice_As": hAs if nh else [],
                            "lattice_Ps": hPs})
