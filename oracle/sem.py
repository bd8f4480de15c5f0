"""Spectral-element Poisson operator on a structured (possibly deformed) hexahedral box.

Discrete problem (paper, Sec. 1, eq. poisson and the definition a_ij =
integral of grad phi_i . grad phi_j): A u = b with A SPD. The standard SEM
realisation used here:

* every element is the trilinear image of the reference cube [-1,1]^3 under its
  8 corner vertices; nodes are the tensor GLL points of order N;
* J = dx/dr is obtained by differentiating the nodal coordinates with D (exact
  for a trilinear map); G_ab = w_i w_j w_k |J| sum_d (dr_a/dx_d)(dr_b/dx_d),
  six unique entries (rr, rs, rt, ss, st, tt); B = w_i w_j w_k |J|;
* local operator w_e = sum_{a,b} D_a^T (G_ab o D_b u_e) with D_r = I x I x D,
  D_s = I x D x I, D_t = D x I x I;
* assembly A = R Q^T A_L Q R^T: Q copies global values to element-local nodes,
  Q^T sums the local copies back, R removes the Dirichlet (boundary) nodes.

Array conventions: element e = ex + mx*(ey + my*ez); a local array has shape
(E, N+1, N+1, N+1) indexed [e, k, j, i] (i along r / x fastest). Global
unknowns are the interior lattice nodes (I, J, K), 1 <= I <= mx*N-1 etc.,
numbered g = (I-1) + nx*((J-1) + ny*(K-1)) with nx = mx*N-1, ny = my*N-1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .gll import gll_nodes_weights, derivative_matrix, interpolation_matrix

# order of the six stored geometric-factor components
COMPONENTS = ("rr", "rs", "rt", "ss", "st", "tt")
_PAIR = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}


def _comp(a: int, b: int) -> int:
    return _PAIR[(min(a, b), max(a, b))]


def grad_local(D: np.ndarray, u: np.ndarray):
    """(D_r u, D_s u, D_t u) for a local array u[e, k, j, i]."""
    ur = np.einsum("il,ekjl->ekji", D, u)
    us = np.einsum("jl,ekli->ekji", D, u)
    ut = np.einsum("kl,elji->ekji", D, u)
    return ur, us, ut


def grad_transpose_local(D: np.ndarray, wr, ws, wt):
    """D_r^T wr + D_s^T ws + D_t^T wt."""
    return (np.einsum("li,ekjl->ekji", D, wr)
            + np.einsum("lj,ekli->ekji", D, ws)
            + np.einsum("lk,elji->ekji", D, wt))


class SemDiscretisation:
    """Order-N SEM discretisation of -Laplace(u) = f on hexahedral elements, each the
    trilinear image of the reference cube under its 8 corners. Subclasses give the
    corners and the local-to-global map; the operator and its relatives only use D, G,
    B_local and l2g."""

    def _set_geometry(self, C: np.ndarray, N: int):
        """C[e, ck, cj, ci, d]: corner coordinates, reference corner (ci, cj, ck) in {0,1}^3."""
        self.N = N
        self.E = C.shape[0]
        n1 = N + 1
        self.xi, self.w = gll_nodes_weights(N)
        self.D = derivative_matrix(N)
        self.corners = C
        # trilinear map evaluated at the GLL points
        h = np.stack([(1.0 - self.xi) / 2.0, (1.0 + self.xi) / 2.0], axis=0)  # h[c, i]
        self.X = np.einsum("ck,bj,ai,ecbad->ekjid", h, h, h, C)  # X[e,k,j,i,d]

        # Jacobian dx_d / dr_a by differentiating the nodal coordinates
        Jm = np.empty((self.E, n1, n1, n1, 3, 3))
        for d in range(3):
            ur, us, ut = grad_local(self.D, self.X[..., d])
            Jm[..., d, 0], Jm[..., d, 1], Jm[..., d, 2] = ur, us, ut
        self.detJ = np.linalg.det(Jm)
        if np.any(self.detJ <= 0.0):
            raise ValueError("mesh has an element with non-positive Jacobian")
        Jinv = np.linalg.inv(Jm)  # Jinv[..., a, d] = dr_a / dx_d
        W = np.einsum("k,j,i->kji", self.w, self.w, self.w)
        self.B_local = W[None] * self.detJ
        self.G = np.empty((self.E, 6, n1, n1, n1))
        for a in range(3):
            for b in range(a, 3):
                self.G[:, _comp(a, b)] = self.B_local * np.einsum(
                    "...d,...d->...", Jinv[..., a, :], Jinv[..., b, :])


class SemBox(SemDiscretisation):
    """Order-N SEM discretisation of -Laplace(u) = f on a structured hexahedral box.

    verts: (mz+1, my+1, mx+1, 3) vertex coordinates (x fastest). Dirichlet
    conditions hold on the whole boundary of the box.
    """

    def __init__(self, verts: np.ndarray, N: int):
        verts = np.asarray(verts, dtype=np.float64)
        self.verts = verts
        self.mz, self.my, self.mx = (s - 1 for s in verts.shape[:3])
        E = self.mx * self.my * self.mz
        n1 = N + 1

        # element corner coordinates C[e, ck, cj, ci, d]
        C = np.empty((E, 2, 2, 2, 3))
        e = 0
        for ez in range(self.mz):
            for ey in range(self.my):
                for ex in range(self.mx):
                    C[e] = verts[ez:ez + 2, ey:ey + 2, ex:ex + 2, :]
                    e += 1
        self._set_geometry(C, N)

        # local-to-global map of interior unknowns (-1 on the Dirichlet boundary)
        self.nx, self.ny, self.nz = self.mx * N - 1, self.my * N - 1, self.mz * N - 1
        self.n = self.nx * self.ny * self.nz
        ex = np.arange(self.E) % self.mx
        ey = (np.arange(self.E) // self.mx) % self.my
        ez = np.arange(self.E) // (self.mx * self.my)
        r = np.arange(n1)
        I = ex[:, None, None, None] * N + r[None, None, None, :]
        J = ey[:, None, None, None] * N + r[None, None, :, None]
        K = ez[:, None, None, None] * N + r[None, :, None, None]
        I, J, K = np.broadcast_arrays(I, J, K)
        inside = ((I >= 1) & (I <= self.mx * N - 1) & (J >= 1) & (J <= self.my * N - 1)
                  & (K >= 1) & (K <= self.mz * N - 1))
        g = (I - 1) + self.nx * ((J - 1) + self.ny * (K - 1))
        self.l2g = np.where(inside, g, -1).astype(np.int64)
        self.mult = self.gather(np.ones_like(self.B_local))  # copies per unknown

    # ---- Q and Q^T (with the Dirichlet restriction R) -------------------------
    # (these and the methods below need only D, G, B_local, X and l2g; SemMesh shares them)
    def scatter(self, u: np.ndarray) -> np.ndarray:
        """Q R^T u: global unknowns -> element-local copies (zero on the boundary)."""
        out = np.zeros(self.l2g.shape)
        mask = self.l2g >= 0
        out[mask] = u[self.l2g[mask]]
        return out

    def gather(self, uL: np.ndarray) -> np.ndarray:
        """R Q^T uL: sum of the element-local copies of every interior unknown."""
        mask = self.l2g >= 0
        return np.bincount(self.l2g[mask], weights=uL[mask], minlength=self.n)

    # ---- operator ---------------------------------------------------------------
    def apply_local(self, uL: np.ndarray, G: np.ndarray | None = None) -> np.ndarray:
        """A_L uL = sum_{a,b} D_a^T (G_ab o D_b uL)."""
        G = self.G if G is None else G
        g = [grad for grad in grad_local(self.D, uL)]
        wv = []
        for a in range(3):
            acc = np.zeros_like(uL)
            for b in range(3):
                acc = acc + G[:, _comp(a, b)] * g[b]
            wv.append(acc)
        return grad_transpose_local(self.D, *wv)

    def apply(self, u: np.ndarray, G: np.ndarray | None = None) -> np.ndarray:
        """A u for a global vector u of interior unknowns."""
        return self.gather(self.apply_local(self.scatter(u), G))

    def diag(self) -> np.ndarray:
        """diag(A): local diagonal of A_L assembled with R Q^T."""
        D, G = self.D, self.G
        D2 = D ** 2
        dd = np.diag(D)
        # explicit formula: sum_l D_li^2 Grr(l,j,k) + sum_l D_lj^2 Gss(i,l,k) + sum_l D_lk^2 Gtt(i,j,l)
        dl = (np.einsum("li,ekjl->ekji", D2, G[:, 0])
              + np.einsum("lj,ekli->ekji", D2, G[:, 3])
              + np.einsum("lk,elji->ekji", D2, G[:, 5]))
        di = dd[None, None, None, :]
        dj = dd[None, None, :, None]
        dk = dd[None, :, None, None]
        dl = dl + 2.0 * (di * dj * G[:, 1] + di * dk * G[:, 2] + dj * dk * G[:, 4])
        return self.gather(dl)

    def mass(self) -> np.ndarray:
        """Assembled diagonal mass R Q^T B_L Q R^T (as a vector)."""
        return self.gather(self.B_local)

    def coords(self) -> np.ndarray:
        """Coordinates of the interior unknowns, shape (n, 3)."""
        out = np.zeros((self.n, 3))
        mask = self.l2g >= 0
        for d in range(3):
            out[self.l2g[mask], d] = self.X[..., d][mask]
        return out

    def element_matrices(self, G: np.ndarray | None = None) -> np.ndarray:
        """Dense local matrices A_e = sum_ab D_a^T diag(G_ab) D_b, shape (E, n1^3, n1^3)."""
        G = self.G if G is None else G
        n1 = self.N + 1
        I1 = np.eye(n1)
        Dr = np.kron(I1, np.kron(I1, self.D))
        Ds = np.kron(I1, np.kron(self.D, I1))
        Dt = np.kron(self.D, np.kron(I1, I1))
        Ds_ = (Dr, Ds, Dt)
        Gf = G.reshape(self.E, 6, -1)
        out = np.zeros((self.E, n1 ** 3, n1 ** 3))
        for a in range(3):
            for b in range(3):
                # D_a^T diag(G_ab) D_b for every element (batched matrix product)
                out += np.matmul(Ds_[a].T[None, :, :] * Gf[:, _comp(a, b)][:, None, :], Ds_[b][None])
        return out

    def assemble(self) -> sp.csr_matrix:
        """Sparse assembled A = R Q^T (block-diag A_e) Q R^T (for small N or small E)."""
        Ae = self.element_matrices()
        l2g = self.l2g.reshape(self.E, -1)
        rows, cols, vals = [], [], []
        for e in range(self.E):
            idx = l2g[e]
            keep = np.nonzero(idx >= 0)[0]
            gi = idx[keep]
            sub = Ae[e][np.ix_(keep, keep)]
            rows.append(np.repeat(gi, len(gi)))
            cols.append(np.tile(gi, len(gi)))
            vals.append(sub.ravel())
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.n, self.n))
        return A.tocsr()


class SemTransfer:
    """Order transfer between two SEM levels on the same vertices (p-multigrid).

    P = R_f W_f Q_f^T (J x J x J)_L Q_c R_c^T with J[i, j] = l_j^{(Nc)}(x_i^{(Nf)})
    and W_f the inverse multiplicity of the fine unknowns; P^T is its exact
    transpose (paper, Sec. 2, eq. recursive-v-cycle-err-prop uses P and P^T).
    """

    def __init__(self, fine: SemBox, coarse: SemBox):
        self.f, self.c = fine, coarse
        self.J = interpolation_matrix(coarse.N, fine.N)
        self.winv = 1.0 / fine.mult

    def _interp_local(self, uc):
        J = self.J
        return np.einsum("ia,jb,kc,ecba->ekji", J, J, J, uc)

    def _interp_local_T(self, uf):
        J = self.J
        return np.einsum("ia,jb,kc,ekji->ecba", J, J, J, uf)

    def prolong(self, xc: np.ndarray) -> np.ndarray:
        """P xc."""
        return self.winv * self.f.gather(self._interp_local(self.c.scatter(xc)))

    def restrict(self, rf: np.ndarray) -> np.ndarray:
        """P^T rf."""
        return self.c.gather(self._interp_local_T(self.f.scatter(self.winv * rf)))
