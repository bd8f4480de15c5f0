"""Pins of the unstructured-mesh oracle (oracle/mesh.py).

* a box given as an element list reproduces the structured oracle (itself pinned by a
  brute-force assembly) up to the numbering of the unknowns: operator, diagonal, mass;
* the same after shuffling the elements, turning every element's reference frame by a
  random rotation of the cube and renumbering the vertices;
* partial Dirichlet flags: the assembled operator equals a brute-force assembly over all
  lattice nodes with the rows and columns of the flagged faces' nodes removed;
* mixed boundary conditions: u = sin(pi x / 2) with Dirichlet data on x = 0 only
  (natural conditions elsewhere) is reproduced with an error decaying spectrally in N;
* the p-multigrid cycle commutes with the renumbering.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import workload as wl
from oracle import chebyshev as cheb, mg
from oracle.mesh import SemMesh
from oracle.sem import SemBox
from test_oracle_sem import _lagrange_polys
from oracle.gll import gll_nodes_weights


def _match(coords_a, coords_b):
    """idx with coords_b[i] == coords_a[idx[i]]."""
    d, idx = cKDTree(coords_a).query(coords_b)
    assert d.max() < 1e-12
    return idx


@pytest.mark.parametrize("shuffle", [False, True])
@pytest.mark.parametrize("m,N", [((3, 2, 2), 3), ((2, 2, 3), 5)])
def test_mesh_reproduces_box(m, N, shuffle):
    V = wl.deformed_box(m, 0.07)
    box = SemBox(V, N)
    xyz, ev = wl.box_as_mesh(V)
    if shuffle:
        xyz, ev, _ = wl.shuffled_mesh(xyz, ev, 5)
    mesh = SemMesh(xyz, ev, N)
    assert mesh.n == box.n
    idx = _match(box.coords(), mesh.coords())
    A, Am = box.assemble().toarray(), mesh.assemble().toarray()
    assert np.max(np.abs(Am - A[np.ix_(idx, idx)])) < 1e-13 * np.max(np.abs(A))
    u = wl.uniform_noise(box.n, 3)
    assert np.max(np.abs(mesh.apply(u[idx]) - box.apply(u)[idx])) < 1e-13 * np.max(np.abs(A))
    assert np.max(np.abs(mesh.diag() - box.diag()[idx])) < 1e-13 * np.max(box.diag())
    assert np.max(np.abs(mesh.mass() - box.mass()[idx])) < 1e-15


def _full_lattice_matrix(V, N):
    """Brute-force a_pq over all lattice nodes of the box (boundary included), from
    explicit Lagrange basis gradients and the analytic trilinear Jacobian."""
    mz, my, mx = (s - 1 for s in V.shape[:3])
    x, w = gll_nodes_weights(N)
    L = _lagrange_polys(x)
    Lv = np.array([[l(t) for l in L] for t in x])
    dLv = np.array([[l.deriv()(t) for l in L] for t in x])
    n1 = N + 1
    NX, NY, NZ = mx * N + 1, my * N + 1, mz * N + 1
    A = np.zeros((NX * NY * NZ,) * 2)
    for ez in range(mz):
        for ey in range(my):
            for ex in range(mx):
                C = V[ez:ez + 2, ey:ey + 2, ex:ex + 2, :]
                Ae = np.zeros((n1 ** 3, n1 ** 3))
                for c in range(n1):
                    for b in range(n1):
                        for a in range(n1):
                            r, s, t = x[a], x[b], x[c]
                            Jm = np.zeros((3, 3))
                            for ck in range(2):
                                for cj in range(2):
                                    for ci in range(2):
                                        hr = (1 + (2 * ci - 1) * r) / 2
                                        hs = (1 + (2 * cj - 1) * s) / 2
                                        ht = (1 + (2 * ck - 1) * t) / 2
                                        g = np.array([(2 * ci - 1) / 2 * hs * ht, hr * (2 * cj - 1) / 2 * ht,
                                                      hr * hs * (2 * ck - 1) / 2])
                                        Jm += np.outer(C[ck, cj, ci], g)
                            JinvT = np.linalg.inv(Jm).T
                            grads = np.zeros((n1 ** 3, 3))
                            for kk in range(n1):
                                for jj in range(n1):
                                    for ii in range(n1):
                                        gr = np.array([dLv[a, ii] * Lv[b, jj] * Lv[c, kk],
                                                       Lv[a, ii] * dLv[b, jj] * Lv[c, kk],
                                                       Lv[a, ii] * Lv[b, jj] * dLv[c, kk]])
                                        grads[ii + n1 * (jj + n1 * kk)] = JinvT @ gr
                            Ae += w[a] * w[b] * w[c] * np.linalg.det(Jm) * grads @ grads.T
                idx = [(ex * N + ii) + NX * ((ey * N + jj) + NY * (ez * N + kk))
                       for kk in range(n1) for jj in range(n1) for ii in range(n1)]
                A[np.ix_(idx, idx)] += Ae
    I, J, K = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    lattice = np.stack([I.T.ravel(), J.T.ravel(), K.T.ravel()], axis=1)   # x fastest
    return A, lattice, (NX, NY, NZ)


@pytest.mark.parametrize("faces", [("x0",), ("x0", "y1"), ("z0", "z1", "x1")])
def test_partial_dirichlet_equals_bruteforce(faces):
    V = wl.deformed_box((2, 2, 2), 0.06)
    N = 2
    A, lat, (NX, NY, NZ) = _full_lattice_matrix(V, N)
    on = np.zeros(len(lat), dtype=bool)
    for f in faces:      # the flagged faces' lattice nodes, by lattice position
        d, side = "xyz".index(f[0]), int(f[1])
        on |= lat[:, d] == (0 if side == 0 else (NX, NY, NZ)[d] - 1)
    keep = np.nonzero(~on)[0]
    Aref = A[np.ix_(keep, keep)]
    xyz, ev = wl.box_as_mesh(V)
    xyz, ev, _ = wl.shuffled_mesh(xyz, ev, 11)
    mesh = SemMesh(xyz, ev, N, wl.face_flags(xyz, faces))
    assert mesh.n == len(keep)
    # positions of the lattice nodes, from the box oracle's element nodes (2 x 2 x 2 elements)
    box = SemBox(V, N)
    Xall = box.X.reshape(-1, 3)
    ex = np.repeat(np.arange(box.E), (N + 1) ** 3)
    r = np.arange((N + 1) ** 3)
    ii, jj, kk = r % (N + 1), (r // (N + 1)) % (N + 1), r // (N + 1) ** 2
    gx = (ex % 2) * N + np.tile(ii, box.E)
    gy = ((ex // 2) % 2) * N + np.tile(jj, box.E)
    gz = (ex // 4) * N + np.tile(kk, box.E)
    pos = np.zeros((NX * NY * NZ, 3))
    pos[gx + NX * (gy + NY * gz)] = Xall
    idx = _match(pos[keep], mesh.coords())
    Am = mesh.assemble().toarray()
    assert np.max(np.abs(Am - Aref[np.ix_(idx, idx)])) < 1e-12 * np.max(np.abs(Aref))


def test_mixed_conditions_manufactured_solution():
    """-Laplace u = (pi/2)^2 sin(pi x / 2): u = sin(pi x / 2) satisfies u = 0 on x = 0 and
    du/dn = 0 on the other faces, which the weak form imposes naturally."""
    V = wl.deformed_box(2, 0.05)
    errs = []
    for N in (2, 4, 6, 8):
        xyz, ev = wl.box_as_mesh(V)
        mesh = SemMesh(xyz, ev, N, wl.face_flags(xyz, ("x0",)))
        X = mesh.coords()
        f = (np.pi / 2) ** 2 * np.sin(np.pi * X[:, 0] / 2)
        import scipy.sparse.linalg as spla
        u = spla.spsolve(mesh.assemble().tocsc(), mesh.mass() * f)
        errs.append(np.max(np.abs(u - np.sin(np.pi * X[:, 0] / 2))))
    assert errs[-1] < 1e-6
    assert all(errs[i + 1] < 0.1 * errs[i] for i in range(len(errs) - 1)), errs


def test_no_dirichlet_face_is_refused():
    xyz, ev = wl.box_as_mesh(wl.deformed_box(2, 0.05))
    with pytest.raises(ValueError):
        SemMesh(xyz, ev, 2, np.zeros(len(xyz), np.uint8))


def test_cycle_commutes_with_renumbering():
    V = wl.deformed_box((3, 2, 2), 0.05)
    N = 4
    hb = mg.sem_hierarchy(V, N, cheb.CHEB4_OPT, 4, 0)
    lmax = [lev.lmax for lev in hb.levels[:-1]]
    xyz, ev = wl.box_as_mesh(V)
    xyz, ev, _ = wl.shuffled_mesh(xyz, ev, 2)
    hm = mg.sem_hierarchy((xyz, ev, None), N, cheb.CHEB4_OPT, 4, 0, lmax=lmax)
    idx = _match(hb.extra["boxes"][0].coords(), hm.extra["boxes"][0].coords())
    r = wl.uniform_noise(hb.levels[0].n, 4)
    zb, zm = hb.vcycle(r), hm.vcycle(r[idx])
    assert np.max(np.abs(zm - zb[idx])) < 1e-12 * np.max(np.abs(zb))
