"""Pins of the oracle's restarted flexible GMRES (paper, Sec. 6.1 and Sec. 3).

- Minimal residual: without restart, iterate k minimises ||b - A x|| over x in the
  preconditioned Krylov space M K_k(A M, b); checked by brute-force least squares.
- The rotated recurrence |g_{k+1}| equals the true residual of the k-th iterate.
- Finite termination in at most n steps; restarts still converge.
- Against CG on an SPD system (identity preconditioner), the GMRES residual is never larger.
- Table fastest_solver_fd (Sec. 3): GMRES(20) preconditioned by the FD V-cycles reaches 1e-6 in
  the printed number of iterations on the 4th-kind rows and within two iterations below it on
  the optimised 4th-kind rows (orders 14..20).
"""
import numpy as np
import pytest

import workload as wl
from oracle import chebyshev as cheb
from oracle import fd2d, krylov
from oracle.lanczos import lambda_max_SA


def _system(n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    A = 4.0 * np.eye(n) + 0.6 * g.standard_normal((n, n))      # non-symmetric, well conditioned
    M = np.eye(n) + 0.2 * g.standard_normal((n, n)) / np.sqrt(n)  # fixed non-symmetric preconditioner
    b = g.standard_normal(n)
    return A, M, b


def test_minimal_residual_property():
    A, M, b = _system(30, 1)
    AM = A @ M
    for k in range(1, 9):
        res = krylov.fgmres(lambda x: A @ x, b, lambda v: M @ v, 1e-14, restart=30, maxit=k)
        assert res.iterations == k
        K = np.column_stack([np.linalg.matrix_power(AM, i) @ b for i in range(k)])
        Q, _ = np.linalg.qr(K)
        c, *_ = np.linalg.lstsq(AM @ Q, b, rcond=None)
        best = np.linalg.norm(b - AM @ Q @ c)
        true = np.linalg.norm(b - A @ res.x)
        assert abs(true - best) <= 1e-10 * np.linalg.norm(b), k
        assert abs(res.history[-1] - true) <= 1e-10 * np.linalg.norm(b), k


def test_finite_termination_and_restart():
    A, M, b = _system(12, 2)
    res = krylov.fgmres(lambda x: A @ x, b, lambda v: M @ v, 1e-12, restart=12, maxit=12)
    assert res.converged and res.iterations <= 12
    assert np.linalg.norm(b - A @ res.x) <= 1e-11 * np.linalg.norm(b)
    res = krylov.fgmres(lambda x: A @ x, b, lambda v: M @ v, 1e-12, restart=4, maxit=200)
    assert res.converged and res.iterations > 4
    assert np.linalg.norm(b - A @ res.x) <= 1.01e-12 * np.linalg.norm(b)
    # the identity as operator: one iteration
    res = krylov.fgmres(lambda x: x, b, lambda v: v, 1e-12, restart=5, maxit=5)
    assert res.iterations == 1 and np.allclose(res.x, b)


def test_gmres_residual_never_above_cg():
    A = fd2d.laplacian_5pt(16).toarray()
    b = wl.fd_rhs(15, 3)
    ident = lambda v: v  # noqa: E731
    cg = krylov.pcg(lambda x: A @ x, b, ident, 1e-10, 200)
    gm = krylov.fgmres(lambda x: A @ x, b, ident, 1e-10, restart=300, maxit=300)
    k = min(len(cg.history), len(gm.history))
    assert np.all(np.array(gm.history[:k]) <= np.array(cg.history[:k]) * (1 + 1e-10))
    assert gm.iterations <= cg.iterations


def _fd_table_case(Lx, f, kind, pre, post, seed):
    """Sec. 3 set-up: n = 128, [0,Lx] x [0,1], u = sin(3 pi x / Lx) sin(4 pi y) + g, b = A u,
    levels down to one unknown, GMRES(20) to 1e-6 from x0 = 0. The fine-level lambda_max of the
    Jacobi-scaled 5-point operator is 1 + cos(pi / n) for any aspect ratio (pinned in
    test_oracle_mg); coarser levels use Lanczos."""
    n = 128
    As, _, _ = fd2d.hierarchy_matrices(n, f, Lx, 1.0, 2)
    lmax = [1.0 + np.cos(np.pi / n)] + [lambda_max_SA(lambda x, A=A: A @ x, 1.0 / A.diagonal(), A.shape[0])
                                         for A in As[1:-1]]
    h = fd2d.fd_hierarchy(n, f, kind, pre, post, Lx=Lx, Ly=1.0, coarsest_n=2, lmax=lmax)
    A = h.extra["As"][0]
    X, Y = np.meshgrid(np.arange(1, n) / n * Lx, np.arange(1, n) / n)  # x fastest
    u = (np.sin(3 * np.pi * X / Lx) * np.sin(4 * np.pi * Y)).ravel() + wl.uniform_noise((n - 1) ** 2, seed)
    b = A @ u
    return krylov.fgmres(lambda x: A @ x, b, h.vcycle, 1e-6, restart=20, maxit=200)


def _golden():
    return np.loadtxt(__file__.replace("test_oracle_gmres.py", "golden/fastest_solver_fd.txt"),
                      dtype=int, comments="#")


FD_ROWS = [(1, 2, cheb.CHEB4, 2, 2), (8, 2, cheb.CHEB4, 14, 0), (64, 2, cheb.CHEB4_OPT, 20, 0),
           (128, 2, cheb.CHEB4_OPT, 20, 0), (1, 8, cheb.CHEB4, 7, 7), (8, 8, cheb.CHEB4_OPT, 14, 0),
           (64, 8, cheb.CHEB4_OPT, 18, 0), (128, 8, cheb.CHEB4_OPT, 20, 0)]


@pytest.mark.parametrize("Lx,f,kind,pre,post", FD_ROWS)
def test_fastest_solver_fd_iterations(Lx, f, kind, pre, post):
    """Every row of Table fastest_solver_fd. The 4th-kind rows reproduce the printed
    iteration and mat-vec counts exactly. The optimised 4th-kind rows (orders 14 to 20,
    beta beyond the printed table computed by minimising eq. gamma-defn) converge one or two
    iterations sooner than printed, for every seed of the random part g tried: the paper
    states neither g nor how lambda_max was estimated, and a lambda_max taken 5-20 % high
    moves these rows towards the printed counts while the 4th-kind rows stay put."""
    row = [r for r in _golden() if r[0] == Lx and r[1] == f][0]
    assert (row[2], row[3]) == (pre, post)
    assert row[4] == row[5] * (pre + post + 1)              # printed mat-vecs = iterations (m+n+1)
    res = _fd_table_case(Lx, f, kind, pre, post, seed=0)
    assert res.converged
    if kind == cheb.CHEB4:
        assert res.iterations == row[5]                     # printed iteration count
    else:
        assert row[5] - 2 <= res.iterations <= row[5]
