"""Seeded generators for the synthetic workloads.

Workload recipes (the paper's Kershaw and pebble meshes are not available, so
these stand in for them with the same shape: hexahedral boxes, order 7, a sine
load and a 1e-8 relative-residual stop, see the Kershaw case in the paper's
section on high-order cases):

* deformed box: [0,1]^3 split into mx*my*mz hexahedra; every vertex is moved by
  the same scalar a*sin(pi x)sin(pi y)sin(pi z) in each coordinate (boundary
  vertices stay put because the sine vanishes there).
* batched boxes: per system an independent amplitude per coordinate drawn from
  U[0.025, 0.05] and integer wavenumbers drawn from {1, 2}.
* load: f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z), whose exact solution on the
  unit cube with homogeneous Dirichlet data is sin(pi x) sin(pi y) sin(pi z).
* noise: i.i.d. U[-1, 1] (PCG64, explicit seed).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def box_vertices(mx: int, my: int, mz: int) -> np.ndarray:
    """Undeformed lattice vertices of [0,1]^3, shape (mz+1, my+1, mx+1, 3).

    Vertex (i, j, k) sits at (i/mx, j/my, k/mz); flattened index is
    i + (mx+1)*(j + (my+1)*k) (x fastest).
    """
    x = np.arange(mx + 1, dtype=np.float64) / mx
    y = np.arange(my + 1, dtype=np.float64) / my
    z = np.arange(mz + 1, dtype=np.float64) / mz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def deformed_box(m: int | tuple, amplitude: float = 0.05) -> np.ndarray:
    """Box vertices displaced by amplitude*sin(pi x)sin(pi y)sin(pi z) in x, y and z."""
    mx, my, mz = (m, m, m) if np.isscalar(m) else m
    V = box_vertices(mx, my, mz)
    s = (np.sin(np.pi * V[..., 0]) * np.sin(np.pi * V[..., 1])
         * np.sin(np.pi * V[..., 2]))
    return V + amplitude * s[..., None]


def batched_box(m: int, seed: int) -> np.ndarray:
    """Box with a per-coordinate random sine displacement.

    Coordinate d moves by a_d * sin(k_d0 pi x) sin(k_d1 pi y) sin(k_d2 pi z),
    with a_d ~ U[0.025, 0.05] and k_d* drawn from {1, 2}.
    """
    g = _rng(seed)
    a = g.uniform(0.025, 0.05, size=3)
    k = g.integers(1, 3, size=(3, 3))
    V = box_vertices(m, m, m)
    out = V.copy()
    for d in range(3):
        s = (np.sin(k[d, 0] * np.pi * V[..., 0]) * np.sin(k[d, 1] * np.pi * V[..., 1])
             * np.sin(k[d, 2] * np.pi * V[..., 2]))
        out[..., d] += a[d] * s
    return out


def manufactured_load(xyz: np.ndarray) -> np.ndarray:
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) evaluated at points xyz[..., 3]."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    return 3.0 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def manufactured_solution(xyz: np.ndarray) -> np.ndarray:
    """u* = sin(pi x) sin(pi y) sin(pi z), the exact solution for manufactured_load."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def uniform_noise(n: int, seed: int = 0) -> np.ndarray:
    """n i.i.d. draws from U[-1, 1]."""
    return _rng(seed).uniform(-1.0, 1.0, size=n)


def fd_rhs(n_interior: int, seed: int = 0) -> np.ndarray:
    """Finite-difference right-hand side on an n_interior^2 grid, i.i.d. U[-1,1], x fastest."""
    return _rng(seed).uniform(-1.0, 1.0, size=n_interior * n_interior)


@dataclass(frozen=True)
class BoxSpec:
    m: int          # elements per direction (E = m^3)
    N: int          # polynomial order
    mesh_seed: int  # seed of the per-system deformation
    rhs_seed: int   # seed of the per-system rhs noise


def batched_specs(nsys: int = 64, base_seed: int = 1000) -> list[BoxSpec]:
    """Per-system sizes: m ~ U{4..16}, N ~ U{5,7,9}, drawn with seed base_seed+s."""
    out = []
    for s in range(nsys):
        g = _rng(base_seed + s)
        m = int(g.integers(4, 17))
        N = int(g.choice([5, 7, 9]))
        out.append(BoxSpec(m=m, N=N, mesh_seed=base_seed + s, rhs_seed=base_seed + 100 + s))
    return out


def target_coeffs(seed: int = 0, terms: int = 4):
    """Coefficients c_q ~ N(0,1) and wavenumbers in {1,2,3} for target_field."""
    g = _rng(seed)
    c = g.standard_normal(terms)
    k = g.integers(1, 4, size=(terms, 3))
    return c, k


def target_field(xyz: np.ndarray, seed: int = 0, terms: int = 4) -> np.ndarray:
    """Smooth seeded target u_t = sum_q c_q sin(a_q pi x) sin(b_q pi y) sin(c_q pi z)."""
    c, k = target_coeffs(seed, terms)
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    out = np.zeros(np.shape(x))
    for q in range(terms):
        out = out + c[q] * (np.sin(k[q, 0] * np.pi * x) * np.sin(k[q, 1] * np.pi * y)
                            * np.sin(k[q, 2] * np.pi * z))
    return out


def gaussian_directions(count: int, sizes: tuple, seed: int = 1):
    """count random directions over a product space of the given sizes, unit 2-norm overall."""
    g = _rng(seed)
    out = []
    for _ in range(count):
        parts = [g.standard_normal(s) for s in sizes]
        nrm = np.sqrt(sum(float(np.dot(p, p)) for p in parts))
        out.append([p / nrm for p in parts])
    return out


# ---- unstructured (element list) form of a box mesh
def _rotations():
    """The 24 proper rotations of the cube as signed 3x3 permutation matrices."""
    out = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        for signs in np.ndindex(2, 2, 2):
            R = np.zeros((3, 3), dtype=int)
            for r in range(3):
                R[r, perm[r]] = 1 - 2 * signs[r]
            if round(np.linalg.det(R)) == 1:
                out.append(R)
    return out


def box_as_mesh(V: np.ndarray):
    """(vertex_xyz (nv, 3), elem_vertices (E, 8)) of a box given as (mz+1, my+1, mx+1, 3)
    vertices: vertex (i, j, k) -> i + (mx+1)(j + (my+1) k); elements x fastest; corner
    ci + 2 cj + 4 ck of element (ex, ey, ez) is vertex (ex+ci, ey+cj, ez+ck)."""
    mz, my, mx = (s - 1 for s in V.shape[:3])
    xyz = V.reshape(-1, 3).copy()
    ev = []
    for ez in range(mz):
        for ey in range(my):
            for ex in range(mx):
                ev.append([(ex + ci) + (mx + 1) * ((ey + cj) + (my + 1) * (ez + ck))
                           for ck in (0, 1) for cj in (0, 1) for ci in (0, 1)])
    return xyz, np.array(ev, dtype=np.int64)


def shuffled_mesh(xyz: np.ndarray, ev: np.ndarray, seed: int):
    """The same mesh with its elements in random order, every element's reference frame
    turned by a random proper rotation of the cube (its corner list reordered to match)
    and its vertices renumbered at random. Returns (xyz, ev, vertex_perm) with
    vertex_perm[old] = new index."""
    g = _rng(seed)
    rots = _rotations()
    nv = len(xyz)
    vperm = g.permutation(nv)
    new_xyz = np.empty_like(xyz)
    new_xyz[vperm] = xyz
    out = np.empty_like(ev)
    for q, e in enumerate(g.permutation(len(ev))):
        R = rots[int(g.integers(len(rots)))]
        for c in range(8):
            ref = np.array([2 * (c & 1) - 1, 2 * ((c >> 1) & 1) - 1, 2 * ((c >> 2) & 1) - 1])
            rc = R @ ref                                   # the corner's new reference position
            cn = ((rc[0] + 1) // 2) + 2 * ((rc[1] + 1) // 2) + 4 * ((rc[2] + 1) // 2)
            out[q, cn] = vperm[ev[e, c]]
    return new_xyz, out, vperm


def face_flags(xyz: np.ndarray, faces) -> np.ndarray:
    """Vertex flags of the unit-box faces named in `faces` ("x0", "x1", "y0", ...)."""
    out = np.zeros(len(xyz), dtype=np.uint8)
    for f in faces:
        d, side = "xyz".index(f[0]), float(f[1])
        out |= np.isclose(xyz[:, d], side, atol=1e-12).astype(np.uint8)
    return out
