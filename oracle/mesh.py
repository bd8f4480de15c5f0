"""SEM discretisation on a conforming unstructured hexahedral mesh (test infrastructure).

The mesh is given as vertex coordinates and, per element, its 8 corner vertices in
lexicographic reference order (corner ci + 2 cj + 4 ck sits at reference point
(2ci-1, 2cj-1, 2ck-1)). Every element is the trilinear image of the reference cube; the
operator is the same as on the box (paper, Sec. 1, eq. poisson, with the standard SEM
realisation of oracle.sem), and the paper stresses that p-multigrid coarsens such meshes
as robustly as structured ones (Sec. 4.1).

Conventions (shared with the library by definition, not by code):
* global node identity: element-local nodes that sit at the same point of space are one
  node (conforming mesh). Here they are matched by position (a k-d tree query within a
  tiny radius), which needs no knowledge of element orientation;
* Dirichlet nodes: the nodes of boundary faces (faces that belong to one element) whose 4
  corner vertices are all flagged; with no flags, every boundary face is Dirichlet;
* numbering of the unknowns: first appearance when the element-local nodes are visited
  in the order (e, k, j, i), i fastest, Dirichlet nodes skipped.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

from .sem import SemBox

# the 6 faces of the reference cube as (axis, side): the local index along `axis` is 0 or N
FACES = [(a, s) for a in range(3) for s in (0, 1)]


def _corner_ids(axis: int, side: int):
    """Corner numbers ci + 2 cj + 4 ck on face (axis, side)."""
    out = []
    for c in range(8):
        bits = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
        if bits[axis] == side:
            out.append(c)
    return out


class SemMesh(SemBox):
    """Order-N SEM discretisation on an unstructured conforming hexahedral mesh.

    vertex_xyz: (num_vertices, 3); elem_vertices: (E, 8) vertex indices per element in
    lexicographic corner order; vertex_dirichlet: (num_vertices,) flags or None (whole
    boundary Dirichlet). Shares the operator, mass, diagonal, assembly and transfers of
    SemBox, which only use the element geometry and the local-to-global map."""

    def __init__(self, vertex_xyz, elem_vertices, N: int, vertex_dirichlet=None):
        V = np.asarray(vertex_xyz, dtype=np.float64)
        EV = np.asarray(elem_vertices, dtype=np.int64)
        self.vertex_xyz, self.elem_vertices = V, EV
        E = EV.shape[0]
        C = V[EV].reshape(E, 2, 2, 2, 3)             # [e, ck, cj, ci, d]
        self._set_geometry(C, N)
        n1 = N + 1
        P = self.X.reshape(-1, 3)

        # node identity by position
        span = float(np.max(np.ptp(P, axis=0)))
        pairs = np.array(list(cKDTree(P).query_pairs(r=1e-9 * span)), dtype=np.int64).reshape(-1, 2)
        graph = sp.coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(len(P), len(P)))
        _, comp = connected_components(graph, directed=False)

        # Dirichlet faces: boundary faces (one element) with all corners flagged
        flags = np.ones(len(V), dtype=bool) if vertex_dirichlet is None else np.asarray(vertex_dirichlet, bool)
        count = {}
        for e in range(E):
            for (a, s) in FACES:
                key = tuple(sorted(EV[e, _corner_ids(a, s)]))
                count[key] = count.get(key, 0) + 1
        dirichlet = np.zeros(comp.max() + 1, dtype=bool)
        idx = np.arange(n1)
        for e in range(E):
            for (a, s) in FACES:
                corners = EV[e, _corner_ids(a, s)]
                if count[tuple(sorted(corners))] != 1 or not np.all(flags[corners]):
                    continue
                sel = [slice(None)] * 3                  # local array order [k, j, i]
                sel[2 - a] = idx[-1] if s else idx[0]
                loc = np.arange(n1 ** 3).reshape(n1, n1, n1)[tuple(sel)].ravel()
                dirichlet[comp[e * n1 ** 3 + loc]] = True
        if np.all(dirichlet[comp]):
            raise ValueError("every node is a Dirichlet node")
        if not np.any(dirichlet):
            raise ValueError("no Dirichlet face: the operator would be singular")

        # numbering by first appearance in (e, k, j, i) order
        first = np.full(comp.max() + 1, -1, dtype=np.int64)
        uniq, pos = np.unique(comp, return_index=True)
        first[uniq] = pos
        order = np.argsort(first[uniq])
        gid = np.full(comp.max() + 1, -1, dtype=np.int64)
        nxt = 0
        for c in uniq[order]:
            if not dirichlet[c]:
                gid[c] = nxt
                nxt += 1
        self.n = nxt
        self.l2g = gid[comp].reshape(E, n1, n1, n1)
        self.mult = self.gather(np.ones_like(self.B_local))
