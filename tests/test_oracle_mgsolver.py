"""Pins of the oracle's multigrid-as-the-solver iteration (paper, Sec. 3; eq.
avg-convergence-rate; Lemma multilevel-poly-bound).

- An exact inverse as M converges in one iteration.
- Brute force: the error after i iterations is E^i e_0 with E = I - M A assembled column by
  column from the V-cycle (a sign or a missing residual update fails it).
- The per-iteration residual ratio tends to the spectral radius of E (library eigenvalues).
- The symmetric (k,k) cycle's spectral radius obeys the multilevel bound
  rho(E_V) = ||E_down||_A^2 <= max_j C_j / (C_j + gamma^{-1}(k)).
"""
import numpy as np
import pytest

import workload as wl
from oracle import analysis as an
from oracle import chebyshev as cheb
from oracle import fd2d, krylov


def _fd(n, kind, pre, post, Lx=1.0):
    h = fd2d.fd_hierarchy(n, 2, kind, pre, post, Lx=Lx, Ly=1.0, coarsest_n=2)
    return h, h.extra["As"][0].toarray()


def test_exact_inverse_one_iteration():
    A = fd2d.laplacian_5pt(8).toarray()
    b = wl.fd_rhs(7, 1)
    res = krylov.mg_solver(lambda x: A @ x, b, lambda r: np.linalg.solve(A, r), 1e-12, 5)
    assert res.converged and res.iterations == 1
    assert np.linalg.norm(b - A @ res.x) <= 1e-12 * np.linalg.norm(b)
    z = krylov.mg_solver(lambda x: A @ x, np.zeros_like(b), lambda r: r, 1e-12, 5)
    assert z.converged and z.iterations == 0


@pytest.mark.parametrize("kind,pre,post", [(cheb.CHEB4, 2, 2), (cheb.CHEB1_OPT, 3, 0), (cheb.CHEB4_OPT, 1, 2)])
def test_error_propagation_brute_force(kind, pre, post):
    h, A = _fd(8, kind, pre, post, Lx=2.0)
    E = an.error_propagator(h.vcycle, A)
    b = wl.fd_rhs(7, 2)
    xs = np.linalg.solve(A, b)
    e = xs.copy()                                   # e_0 = x* - 0
    for i in range(1, 7):
        res = krylov.mg_solver(lambda x: A @ x, b, h.vcycle, 0.0, i)
        e = E @ e
        assert res.iterations == i and not res.converged
        assert np.linalg.norm((xs - res.x) - e) <= 1e-12 * np.linalg.norm(xs), i
        assert abs(res.history[-1] - np.linalg.norm(A @ e)) <= 1e-12 * np.linalg.norm(b), i


@pytest.mark.parametrize("kind,Lx", [(cheb.CHEB1, 1.0), (cheb.CHEB4, 8.0)])
def test_residual_ratio_tends_to_spectral_radius(kind, Lx):
    h, A = _fd(16, kind, 1, 1, Lx=Lx)
    rho = float(np.max(np.abs(np.linalg.eigvals(an.error_propagator(h.vcycle, A)))))
    b = wl.fd_rhs(15, 3)
    res = krylov.mg_solver(lambda x: A @ x, b, h.vcycle, 1e-12, 400)
    hs = np.array(res.history)
    assert abs(hs[-1] / hs[-2] - rho) <= 2e-3 * rho
    # eq. avg-convergence-rate: the geometric mean of the ratios
    assert abs(res.avg_rate() - np.exp(np.mean(np.log(hs[1:] / hs[:-1])))) < 1e-14


@pytest.mark.parametrize("kind,k", [(cheb.CHEB4, 1), (cheb.CHEB4, 2), (cheb.CHEB4_OPT, 2), (cheb.CHEB1_OPT, 3)])
def test_symmetric_cycle_spectral_radius_within_bound(kind, k):
    h, A = _fd(16, kind, k, k, Lx=4.0)
    As, Ps = h.extra["As"], h.extra["Ps"]
    rho = float(np.max(np.abs(np.linalg.eigvals(an.error_propagator(h.vcycle, A)))))
    Cs = [an.approximation_constant(As[j].toarray(), Ps[j].toarray(), As[j + 1].toarray())
          for j in range(len(Ps))]
    g = an.gamma_inv(kind, k)
    assert rho <= max(C / (C + g) for C in Cs) + 1e-12
