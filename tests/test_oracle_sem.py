"""Pins of the SEM operator oracle.

* matrix-free A equals an independently assembled matrix built from explicit
  basis-function gradients (numpy polynomials, analytic trilinear Jacobian);
* undeformed box: A equals the Kronecker sum of 1D SEM stiffness/mass matrices;
* A_L annihilates constants, A is symmetric positive definite, diag matches;
* the GLL mass integrates the domain volume exactly;
* manufactured solution: nodal error decays exponentially with N.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
from numpy.polynomial import Polynomial

import workload as wl
from oracle.gll import gll_nodes_weights, derivative_matrix
from oracle.sem import SemBox


def _lagrange_polys(nodes):
    out = []
    for j, xj in enumerate(nodes):
        others = np.delete(nodes, j)
        p = Polynomial.fromroots(others)
        out.append(p / p(xj))
    return out


def _bruteforce_matrix(verts, N):
    """a_pq = sum_quad W |J| grad phi_p . grad phi_q, assembled by lattice position."""
    mz, my, mx = (s - 1 for s in verts.shape[:3])
    x, w = gll_nodes_weights(N)
    L = _lagrange_polys(x)
    Lv = np.array([[l(t) for l in L] for t in x])            # [quad, basis]
    dLv = np.array([[l.deriv()(t) for l in L] for t in x])
    n1 = N + 1
    nx, ny, nz = mx * N - 1, my * N - 1, mz * N - 1
    n = nx * ny * nz
    A = np.zeros((n, n))
    for ez in range(mz):
        for ey in range(my):
            for ex in range(mx):
                C = verts[ez:ez + 2, ey:ey + 2, ex:ex + 2, :]  # [ck, cj, ci, d]
                Ae = np.zeros((n1 ** 3, n1 ** 3))
                for c in range(n1):
                    for b in range(n1):
                        for a in range(n1):
                            r, s, t = x[a], x[b], x[c]
                            # analytic derivative of the trilinear map
                            Jm = np.zeros((3, 3))
                            for ck in range(2):
                                for cj in range(2):
                                    for ci in range(2):
                                        hr = (1 + (2 * ci - 1) * r) / 2
                                        hs = (1 + (2 * cj - 1) * s) / 2
                                        ht = (1 + (2 * ck - 1) * t) / 2
                                        g = np.array([(2 * ci - 1) / 2 * hs * ht,
                                                      hr * (2 * cj - 1) / 2 * ht,
                                                      hr * hs * (2 * ck - 1) / 2])
                                        Jm += np.outer(C[ck, cj, ci], g)
                            det = np.linalg.det(Jm)
                            JinvT = np.linalg.inv(Jm).T
                            grads = np.zeros((n1 ** 3, 3))
                            for kk in range(n1):
                                for jj in range(n1):
                                    for ii in range(n1):
                                        p = ii + n1 * (jj + n1 * kk)
                                        gr = np.array([dLv[a, ii] * Lv[b, jj] * Lv[c, kk],
                                                       Lv[a, ii] * dLv[b, jj] * Lv[c, kk],
                                                       Lv[a, ii] * Lv[b, jj] * dLv[c, kk]])
                                        grads[p] = JinvT @ gr
                            Ae += w[a] * w[b] * w[c] * det * grads @ grads.T
                idx = []
                for kk in range(n1):
                    for jj in range(n1):
                        for ii in range(n1):
                            I, J, K = ex * N + ii, ey * N + jj, ez * N + kk
                            ok = 0 < I < mx * N and 0 < J < my * N and 0 < K < mz * N
                            idx.append((I - 1) + nx * ((J - 1) + ny * (K - 1)) if ok else -1)
                idx = np.array(idx)
                keep = np.nonzero(idx >= 0)[0]
                A[np.ix_(idx[keep], idx[keep])] += Ae[np.ix_(keep, keep)]
    return A


@pytest.mark.parametrize("m,N,amp", [((2, 2, 2), 2, 0.05), ((2, 2, 2), 3, 0.08), ((3, 2, 2), 2, 0.1)])
def test_apply_equals_bruteforce_assembly(m, N, amp):
    V = wl.deformed_box(m, amp)
    box = SemBox(V, N)
    A = _bruteforce_matrix(V, N)
    Amf = np.column_stack([box.apply(e) for e in np.eye(box.n)])
    assert np.max(np.abs(A - Amf)) < 1e-12 * np.max(np.abs(A))
    assert np.max(np.abs(box.assemble().toarray() - A)) < 1e-12 * np.max(np.abs(A))


@pytest.mark.parametrize("m,N", [(2, 3), (3, 2), (2, 5)])
def test_undeformed_kronecker_sum(m, N):
    box = SemBox(wl.box_vertices(m, m, m), N)
    _, w = gll_nodes_weights(N)
    D = derivative_matrix(N)
    h = 1.0 / m
    nn = m * N + 1
    K = np.zeros((nn, nn))
    M = np.zeros((nn, nn))
    for e in range(m):
        sl = slice(e * N, e * N + N + 1)
        K[sl, sl] += (2.0 / h) * D.T @ np.diag(w) @ D
        M[sl, sl] += (h / 2.0) * np.diag(w)
    K, M = K[1:-1, 1:-1], M[1:-1, 1:-1]
    A = np.kron(M, np.kron(M, K)) + np.kron(M, np.kron(K, M)) + np.kron(K, np.kron(M, M))
    Amf = np.column_stack([box.apply(e) for e in np.eye(box.n)])
    assert np.max(np.abs(A - Amf)) < 1e-12 * np.max(np.abs(A))


def test_constants_symmetry_spd_diag():
    V = wl.deformed_box(3, 0.05)
    box = SemBox(V, 3)
    one = np.ones(box.l2g.shape)
    assert np.max(np.abs(box.apply_local(one))) < 1e-12
    A = box.assemble().toarray()
    assert np.max(np.abs(A - A.T)) < 1e-14 * np.max(np.abs(A))
    assert np.linalg.eigvalsh(A)[0] > 0
    assert np.max(np.abs(np.diag(A) - box.diag())) < 1e-13 * np.max(np.abs(A))
    col = np.column_stack([box.apply(e) for e in np.eye(box.n)[:50]])
    assert np.max(np.abs(col - A[:, :50])) < 1e-12 * np.max(np.abs(A))


@pytest.mark.parametrize("N", [2, 3, 7])
def test_mass_integrates_volume(N):
    # boundary vertices are not moved, so the deformed box still fills [0,1]^3;
    # |J| of a trilinear map has degree 2 per direction, which GLL(N>=2) integrates exactly
    box = SemBox(wl.deformed_box(3, 0.05), N)
    assert abs(box.B_local.sum() - 1.0) < 1e-13


def test_vertex_coordinates():
    V = wl.deformed_box(3, 0.05)
    box = SemBox(V, 4)
    # element (1,1,1) node (0,0,0) is vertex (1,1,1)
    e = 1 + 3 * (1 + 3 * 1)
    assert np.allclose(box.X[e, 0, 0, 0], V[1, 1, 1], atol=1e-15)
    assert np.allclose(box.X[e, 4, 4, 4], V[2, 2, 2], atol=1e-15)


def test_manufactured_solution_spectral_convergence():
    V = wl.deformed_box(2, 0.05)
    errs = []
    for N in range(2, 10):
        box = SemBox(V, N)
        xyz = box.coords()
        b = box.mass() * wl.manufactured_load(xyz)
        u = spla.spsolve(box.assemble().tocsc(), b)
        errs.append(np.max(np.abs(u - wl.manufactured_solution(xyz))))
    errs = np.array(errs)
    assert errs[-1] < 1e-6
    # exponential decay: log error drops at least ~linearly in N
    assert np.all(errs[2:] < errs[:-2])
    slope = np.polyfit(np.arange(2, 10), np.log(errs), 1)[0]
    assert slope < -1.5
