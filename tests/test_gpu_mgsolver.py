"""Multigrid as the solver on the GPU against the oracle's stationary iteration (paper,
Sec. 3; eq. avg-convergence-rate).

Same lambda_max on both sides: identical iteration counts, true-residual histories to
1e-11 ||b||, solutions to 1e-10. Also: changing the smoothing of a context after setup
gives the cycle of a context set up with that smoothing, and a single-precision cycle
as iterative refinement reaches the FP64 tolerance.
"""
import numpy as np
import pytest
import torch

import workload as wl
from oracle import chebyshev as cheb
from oracle import fd2d, krylov, mg
from oracle.lanczos import lambda_max_SA
from oracle.sem import SemBox
from paper_2210_03179_amd.solver import FdSolver, SemSolver

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _compare(info, u, res, bnorm):
    assert info.iterations == res.iterations and info.converged == res.converged
    assert np.max(np.abs(info.history - np.array(res.history))) <= 1e-11 * bnorm
    assert np.linalg.norm(u.cpu().numpy() - res.x) <= 1e-10 * np.linalg.norm(res.x)


def _fd_lmax(n, f, Lx):
    As, _, _ = fd2d.hierarchy_matrices(n, f, Lx, 1.0, 2)
    return [1.0 + np.cos(np.pi / n)] + [lambda_max_SA(lambda x, A=A: A @ x, 1.0 / A.diagonal(), A.shape[0])
                                         for A in As[1:-1]]


@pytest.mark.parametrize("n,f,Lx,kind,pre,post", [
    (32, 2, 1.0, cheb.CHEB4, 2, 2), (32, 2, 8.0, cheb.CHEB4_OPT, 4, 0), (64, 8, 4.0, cheb.CHEB1, 3, 3),
    (64, 2, 16.0, cheb.CHEB1_OPT, 6, 0), (128, 8, 8.0, cheb.CHEB4, 5, 5)])
def test_fd_mg_solver_parity(n, f, Lx, kind, pre, post):
    print(f"fd mg n={n} f={f} Lx={Lx} {kind} ({pre},{post})", flush=True)
    lmax = _fd_lmax(n, f, Lx)
    h = fd2d.fd_hierarchy(n, f, kind, pre, post, Lx=Lx, Ly=1.0, coarsest_n=2, lmax=lmax)
    A = h.extra["As"][0]
    b = wl.fd_rhs(n - 1, 7)
    res = krylov.mg_solver(lambda x: A @ x, b, h.vcycle, 1e-6, 150)
    s = FdSolver(n=n, Lx=Lx, Ly=1.0, factor=f, coarsest_n=2, smoother=kind, pre=pre, post=post,
                 krylov="mg", lambda_max=lmax)
    s.reset_counts()
    u, info = s.solve(dev(b), rtol=1e-6, maxit=150)
    _compare(info, u, res, np.linalg.norm(b))
    assert s.apply_counts()[0] == info.iterations * (pre + post + 1)
    assert abs(info.avg_rate() - res.avg_rate()) < 1e-9


@pytest.mark.parametrize("kind,pre,post,schwarz", [(cheb.CHEB4_OPT, 4, 0, None), (cheb.CHEB4, 2, 2, None),
                                                   (cheb.CHEB1, 2, 0, "ras")])
def test_sem_mg_solver_parity(kind, pre, post, schwarz):
    print(f"sem mg {kind} ({pre},{post}) {schwarz}", flush=True)
    V = wl.deformed_box((2, 2, 3), 0.05)
    orders = [5, 3, 1]
    ref = mg.sem_hierarchy(V, 5, kind, pre, post, orders=orders, schwarz=schwarz)
    lmax = [lev.lmax for lev in ref.levels[:-1]]
    box = ref.extra["boxes"][0]
    b = box.mass() * wl.manufactured_load(box.coords()) + 1e-2 * wl.uniform_noise(box.n, 8)
    res = krylov.mg_solver(box.apply, b, ref.vcycle, 1e-9, 100)
    s = SemSolver(V, N=5, orders=orders, smoother=kind, pre=pre, post=post, krylov="mg", lambda_max=lmax,
                  schwarz=schwarz)
    u, info = s.solve(dev(b), rtol=1e-9, maxit=100)
    assert info.converged
    _compare(info, u, res, np.linalg.norm(b))


def test_set_smoothing_matches_fresh_context(monkeypatch):
    # both contexts use the same operator variant (the autotuner may pick different ones, whose
    # rounding differs)
    monkeypatch.setenv("SEMCHEB_AX_VARIANT", "0")
    V = wl.deformed_box(3, 0.05)
    s = SemSolver(V, N=6, smoother="cheb4opt", pre=4, post=0)
    lmax = s.lambda_max()
    r = dev(wl.uniform_noise(s.n, 9))
    z0 = s.vcycle(r)                       # captures the (4,0) cycle
    for kind, pre, post in [("cheb1", 2, 3), ("cheb4", 3, 3), ("cheb1opt", 6, 0)]:
        s.set_smoothing(kind, pre, post)
        fresh = SemSolver(V, N=6, smoother=kind, pre=pre, post=post, lambda_max=lmax)
        z, zf = s.vcycle(r), fresh.vcycle(r)
        assert torch.equal(z, zf), kind
        assert not torch.equal(z, z0)
        fresh.close()


def test_mixed_mg_solver_iterative_refinement():
    V = wl.deformed_box(4, 0.05)
    box = SemBox(V, 7)
    b = box.mass() * wl.manufactured_load(box.coords()) + 1e-3 * wl.uniform_noise(box.n, 0)
    s = SemSolver(V, N=7, smoother="cheb4opt", pre=4, post=0, precision="mixed", krylov="mg")
    u, info = s.solve(dev(b), rtol=1e-9, maxit=200)
    assert info.converged
    true = np.linalg.norm(b - box.apply(u.cpu().numpy())) / np.linalg.norm(b)
    assert true <= 1e-9 and abs(true - info.relres) <= 1e-12
    s64 = SemSolver(V, N=7, smoother="cheb4opt", pre=4, post=0, krylov="mg")
    _, info64 = s64.solve(dev(b), rtol=1e-9, maxit=200)
    assert abs(info.iterations - info64.iterations) <= 1


def test_mg_solver_limits():
    s = FdSolver(n=32, factor=2, coarsest_n=2, smoother="cheb4", pre=1, post=1, krylov="mg")
    u, info = s.solve(torch.zeros(s.n, dtype=torch.float64, device="cuda"))
    assert info.converged and info.iterations == 0
    b = dev(wl.fd_rhs(31, 4))
    u, info = s.solve(b, rtol=1e-15, maxit=4)
    assert not info.converged and info.iterations == 4 and len(info.history) == 5
