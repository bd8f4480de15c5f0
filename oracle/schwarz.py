"""Schwarz smoothers with fast-diagonalisation local solves (paper, Sec. 4.1, eq. asm).
Test infrastructure: a plain FP64 definition, not the product path.

Each element e owns an overlapping subdomain: its (N+1) GLL nodes per axis extended by one
node into each neighbour (the neighbour's first node past the shared face), N+3 unknowns per
axis, with homogeneous Dirichlet conditions beyond. The local operator is the tensor-product
Poisson operator of a box that approximates the element,
    Abar = Bz x By x Ax + Bz x Ay x Bx + Az x By x Bx,
where (A_*, B_*) are the 1D GLL stiffness and (diagonal) mass matrices of the three-element
1D mesh (left neighbour, element, right neighbour), restricted to the N+3 subdomain nodes.
Element lengths are the mean of the four element edges along each axis (the box
approximation of a deformed element). The fast diagonalisation method solves it:
    A_* S_* = B_* S_* Lambda_*  (generalised eigenproblems, S_*^T B_* S_* = I),
    Abar^{-1} = (Sz x Sy x Sx) D^{-1} (Sz^T x Sy^T x Sx^T),  D = 1 x 1 x Lx + 1 x Ly x 1 + Lz x 1 x 1.
On a side without neighbour (the Dirichlet boundary of the box) the missing unknowns (the
element's face node and the node beyond) are decoupled identity rows in A_* and B_*.

  ASM  (eq. asm):   S r = sum_e W_e R_e^T Abar_e^{-1} R_e r, W = 1 / (number of subdomains
                    containing the node), applied after the sum (post-multiplication).
  RAS:              overlap values are dropped after the local solve: every element keeps the
                    values at its own (N+1)^3 nodes, and shared element nodes are averaged
                    (1 / number of element copies), as in the direct-stiffness weighting.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .gll import derivative_matrix, gll_nodes_weights
from .sem import SemBox


def reference_1d(N: int):
    """GLL stiffness D^T W D and mass W on [-1, 1]."""
    _, w = gll_nodes_weights(N)
    D = derivative_matrix(N)
    return D.T @ (w[:, None] * D), w


def element_lengths(box: SemBox) -> np.ndarray:
    """(E, 3) mean edge length of every element along x, y, z."""
    C = box.corners  # [e, ck, cj, ci, d]
    lx = np.linalg.norm(C[:, :, :, 1, :] - C[:, :, :, 0, :], axis=-1).mean(axis=(1, 2))
    ly = np.linalg.norm(C[:, :, 1, :, :] - C[:, :, 0, :, :], axis=-1).mean(axis=(1, 2))
    lz = np.linalg.norm(C[:, 1, :, :, :] - C[:, 0, :, :, :], axis=-1).mean(axis=(1, 2))
    return np.stack([lx, ly, lz], axis=1)


def extended_1d(N: int, h_left: float, h: float, h_right: float, has_left: bool, has_right: bool):
    """1D (A, B) on the N+3 subdomain nodes [left N-1, 0..N, right 1] of the three-element mesh."""
    Ar, w = reference_1d(N)
    n = 3 * N + 1
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    for q, hq in enumerate((h_left, h, h_right)):
        sl = slice(q * N, q * N + N + 1)
        K[sl, sl] += (2.0 / hq) * Ar
        M[sl, sl] += np.diag((hq / 2.0) * w)
    ext = np.arange(N - 1, 2 * N + 2)
    A = K[np.ix_(ext, ext)].copy()
    B = M[np.ix_(ext, ext)].copy()
    absent = []
    if not has_left:
        absent += [0, 1]
    if not has_right:
        absent += [N + 1, N + 2]
    for i in absent:
        A[i, :] = 0.0
        A[:, i] = 0.0
        B[i, :] = 0.0
        B[:, i] = 0.0
        A[i, i] = 1.0
        B[i, i] = 1.0
    return A, B


def fdm_1d(A: np.ndarray, B: np.ndarray):
    """Generalised eigenpairs A s = lambda B s with S^T B S = I."""
    lam, S = sla.eigh(A, B)
    return lam, S


class SchwarzLevel:
    """ASM / RAS smoother of one SEM level (callable: r -> S r)."""

    def __init__(self, box: SemBox, kind: str = "asm"):
        if kind not in ("asm", "ras"):
            raise ValueError("kind must be 'asm' or 'ras'")
        self.box, self.kind = box, kind
        N = box.N
        self.N, self.nb = N, N + 3
        mx, my, mz = box.mx, box.my, box.mz
        L = element_lengths(box)
        Lg = L.reshape(mz, my, mx, 3)
        self.S = np.empty((box.E, 3, self.nb, self.nb))
        self.lam = np.empty((box.E, 3, self.nb))
        for e in range(box.E):
            ex, ey, ez = e % mx, (e // mx) % my, e // (mx * my)
            idx = (ex, ey, ez)
            cnt = (mx, my, mz)
            for a in range(3):
                def length(off):
                    c = list(idx)
                    c[a] += off
                    return float(Lg[c[2], c[1], c[0], a])
                has_l, has_r = idx[a] > 0, idx[a] < cnt[a] - 1
                A1, B1 = extended_1d(N, length(-1) if has_l else length(0), length(0),
                                     length(1) if has_r else length(0), has_l, has_r)
                self.lam[e, a], self.S[e, a] = fdm_1d(A1, B1)
        # D[e, k, j, i] = lx[i] + ly[j] + lz[k]
        self.D = (self.lam[:, 0][:, None, None, :] + self.lam[:, 1][:, None, :, None]
                  + self.lam[:, 2][:, :, None, None])
        # subdomain-local -> global map (-1: not an unknown)
        r = np.arange(self.nb) - 1  # local index -1 .. N+1 relative to the element's node 0
        ex = np.arange(box.E) % mx
        ey = (np.arange(box.E) // mx) % my
        ez = np.arange(box.E) // (mx * my)
        I = ex[:, None, None, None] * N + r[None, None, None, :]
        J = ey[:, None, None, None] * N + r[None, None, :, None]
        K = ez[:, None, None, None] * N + r[None, :, None, None]
        I, J, K = np.broadcast_arrays(I, J, K)
        inside = (I >= 1) & (I <= box.nx) & (J >= 1) & (J <= box.ny) & (K >= 1) & (K <= box.nz)
        g = (I - 1) + box.nx * ((J - 1) + box.ny * (K - 1))
        self.ext_l2g = np.where(inside, g, -1).astype(np.int64)
        own = np.zeros((self.nb,) * 3, dtype=bool)
        own[1:N + 2, 1:N + 2, 1:N + 2] = True
        self.own = own
        mask = self.ext_l2g >= 0
        self.count = np.bincount(self.ext_l2g[mask], minlength=box.n).astype(np.float64)
        self.mult = box.mult

    def local_solve(self, re: np.ndarray) -> np.ndarray:
        """Abar_e^{-1} re for every element, re of shape (E, nb, nb, nb) [e, k, j, i]."""
        Sx, Sy, Sz = self.S[:, 0], self.S[:, 1], self.S[:, 2]
        t = np.einsum("eia,ekji->ekja", Sx, re)      # S_x^T along i
        t = np.einsum("ejb,ekja->ekba", Sy, t)       # S_y^T along j
        t = np.einsum("ekc,ekba->ecba", Sz, t)       # S_z^T along k
        t = t / self.D
        t = np.einsum("ekc,ecba->ekba", Sz, t)       # S_z along k
        t = np.einsum("ejb,ekba->ekja", Sy, t)       # S_y along j
        return np.einsum("eia,ekja->ekji", Sx, t)    # S_x along i

    def restrict(self, r: np.ndarray) -> np.ndarray:
        out = np.zeros(self.ext_l2g.shape)
        mask = self.ext_l2g >= 0
        out[mask] = r[self.ext_l2g[mask]]
        return out

    def __call__(self, r: np.ndarray) -> np.ndarray:
        y = self.local_solve(self.restrict(r))
        mask = self.ext_l2g >= 0
        if self.kind == "asm":
            z = np.bincount(self.ext_l2g[mask], weights=y[mask], minlength=self.box.n)
            return z / self.count
        own = mask & self.own[None]
        z = np.bincount(self.ext_l2g[own], weights=y[own], minlength=self.box.n)
        return z / self.mult
