"""Pins of the oracle's Schwarz smoothers (paper, Sec. 4.1, eq. asm; FDM local solves).

- FDM: the fast-diagonalisation solve equals the dense inverse of the Kronecker-sum operator
  Bz x By x Ax + Bz x Ay x Bx + Az x By x Bx, for interior and boundary elements.
- On an undeformed box the box approximation is exact: the local operator equals the
  Galerkin restriction R_e A R_e^T of the assembled SEM matrix, so ASM and RAS equal their
  brute-force definitions with dense subdomain solves.
- Chebyshev-Schwarz smoothing reduces the iteration count against Chebyshev-Jacobi of the
  same order (the premise of Sec. 4.1).
"""
import numpy as np
import pytest

import workload as wl
from oracle import chebyshev as cheb
from oracle import krylov, mg
from oracle.schwarz import SchwarzLevel, element_lengths, extended_1d
from oracle.sem import SemBox


def _kron_operator(sw, e):
    mats = []
    for a in range(3):
        # rebuild the 1D pair from the stored eigen-decomposition: S^T A S = Lam, S^T B S = I
        S = sw.S[e, a]
        Si = np.linalg.inv(S)
        mats.append((Si.T @ np.diag(sw.lam[e, a]) @ Si, Si.T @ Si))
    (Ax, Bx), (Ay, By), (Az, Bz) = mats
    return np.kron(Bz, np.kron(By, Ax)) + np.kron(Bz, np.kron(Ay, Bx)) + np.kron(Az, np.kron(By, Bx))


@pytest.mark.parametrize("N", [2, 3, 5])
def test_fdm_equals_dense_inverse(N):
    box = SemBox(wl.deformed_box((3, 3, 2), 0.05), N)
    sw = SchwarzLevel(box, "asm")
    g = np.random.default_rng(N)
    re = g.standard_normal((box.E,) + (sw.nb,) * 3)
    y = sw.local_solve(re)
    for e in (0, 4, box.E - 1):  # boundary elements and the interior one of a 3x3x2 box
        Abar = _kron_operator(sw, e)
        ref = np.linalg.solve(Abar, re[e].ravel())
        assert np.allclose(y[e].ravel(), ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_extended_1d_stiffness_is_restricted_assembly():
    N = 4
    A, B = extended_1d(N, 0.3, 0.5, 0.2, True, True)
    # constants: the assembled 1D stiffness annihilates them, so rows whose whole stencil lies
    # inside the subdomain (the element's interior nodes 1..N-1, subdomain rows 2..N) sum to 0
    assert np.allclose(A[2:N + 1].sum(axis=1), 0.0, atol=1e-12)
    assert not np.allclose(A[1].sum(), 0.0)
    assert np.allclose(np.diag(B).sum(), B.sum())  # diagonal mass
    A, B = extended_1d(N, 0.3, 0.5, 0.2, False, True)
    assert np.allclose(A[:2, :2], np.eye(2)) and np.allclose(A[:2, 2:], 0)


def _brute(sw, box, r, A):
    n = box.n
    z = np.zeros(n)
    for e in range(box.E):
        l2g = sw.ext_l2g[e].ravel()
        valid = l2g >= 0
        idx = l2g[valid]
        Ae = A[np.ix_(idx, idx)]
        ye = np.linalg.solve(Ae, r[idx])
        if sw.kind == "asm":
            z[idx] += ye
        else:
            own = sw.own.ravel()[valid]
            z[idx[own]] += ye[own]
    return z / (sw.count if sw.kind == "asm" else box.mult)


@pytest.mark.parametrize("kind", ["asm", "ras"])
def test_undeformed_box_matches_galerkin_subdomains(kind):
    box = SemBox(wl.box_vertices(3, 2, 3), 3)
    assert np.allclose(element_lengths(box), [[1 / 3, 1 / 2, 1 / 3]] * box.E)
    A = box.assemble().toarray()
    sw = SchwarzLevel(box, kind)
    # local operator = R_e A R_e^T on the subdomain's unknowns
    for e in (0, 7, box.E - 1):
        l2g = sw.ext_l2g[e].ravel()
        valid = l2g >= 0
        Abar = _kron_operator(sw, e)
        assert np.allclose(Abar[np.ix_(valid, valid)], A[np.ix_(l2g[valid], l2g[valid])], atol=1e-11)
    r = wl.uniform_noise(box.n, 3)
    assert np.allclose(sw(r), _brute(sw, box, r, A), atol=1e-11 * np.abs(r).max())


@pytest.mark.parametrize("kind", ["asm", "ras"])
def test_schwarz_smoothing_beats_jacobi(kind):
    V = wl.deformed_box(3, 0.05)
    N = 5
    hj = mg.sem_hierarchy(V, N, cheb.CHEB4, 2, 2)
    hs = mg.sem_hierarchy(V, N, cheb.CHEB4, 2, 2, schwarz=kind)
    box = hj.extra["boxes"][0]
    b = box.mass() * wl.manufactured_load(box.coords()) + 1e-2 * wl.uniform_noise(box.n, 2)
    rj = krylov.fgmres(box.apply, b, hj.vcycle, 1e-8, 30, 200)
    rs = krylov.fgmres(box.apply, b, hs.vcycle, 1e-8, 30, 200)
    assert rj.converged and rs.converged
    assert rs.iterations < rj.iterations
    assert np.linalg.norm(b - box.apply(rs.x)) <= 1.01e-8 * np.linalg.norm(b)
