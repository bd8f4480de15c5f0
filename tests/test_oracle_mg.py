"""Pins of transfers, V-cycles, coarse solves, Krylov and the FD hierarchy."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workload as wl
from oracle import analysis as an
from oracle import chebyshev as cheb
from oracle import fd2d, krylov, mg
from oracle.sem import SemBox, SemTransfer


def _poly_field(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return x * (1 - x) * (1 + x) * y * (1 - y) * z * (1 - z) * (2 - z)


@pytest.mark.parametrize("Nf,Nc", [(7, 3), (3, 1), (5, 2)])
def test_prolongation_reproduces_coarse_functions(Nf, Nc):
    # On an undeformed 2x2x2 box, P applied to the coarse nodal values of a function in
    # the coarse space must return that function at the fine nodes.
    V = wl.box_vertices(2, 2, 2)
    f, c = SemBox(V, Nf), SemBox(V, Nc)
    tr = SemTransfer(f, c)
    if Nc >= 3:
        fun = _poly_field
    elif Nc == 2:
        fun = lambda p: p[:, 0] * (1 - p[:, 0]) * p[:, 1] * (1 - p[:, 1]) * p[:, 2] * (1 - p[:, 2])
    else:  # the single interior Q1 node: trilinear hat centred at (1/2, 1/2, 1/2)
        fun = lambda p: np.prod(1 - np.abs(p - 0.5) / 0.5, axis=1)
    assert np.max(np.abs(tr.prolong(fun(c.coords())) - fun(f.coords()))) < 1e-14


@pytest.mark.parametrize("Nf,Nc", [(4, 2), (3, 1)])
def test_restriction_is_exact_transpose(Nf, Nc):
    V = wl.deformed_box(2, 0.05)
    tr = SemTransfer(SemBox(V, Nf), SemBox(V, Nc))
    P = np.column_stack([tr.prolong(e) for e in np.eye(tr.c.n)])
    R = np.column_stack([tr.restrict(e) for e in np.eye(tr.f.n)])
    assert np.max(np.abs(P.T - R)) < 1e-15


def test_fd_grid_complexity_and_levels():
    # Sec. 3 and eq. mg-cycle-complexity: 1.568 with 7 levels (n_c = n/2),
    # 1.023 with 3 levels (n_c = n/8), n = 128, Galerkin coarse operators
    As, _, ns = fd2d.hierarchy_matrices(128, 2, coarsest_n=2)
    assert len(As) == 7 and As[-1].shape == (1, 1)
    assert round(fd2d.grid_complexity(As), 3) == 1.568
    As, _, ns = fd2d.hierarchy_matrices(128, 8, coarsest_n=2)
    assert len(As) == 3 and As[-1].shape == (1, 1)
    assert round(fd2d.grid_complexity(As), 3) == 1.023


def test_fd_lambda_max_exact():
    # isotropic 5-point Laplacian with Jacobi: lambda_max(S A) = 1 + cos(pi h)
    A = fd2d.laplacian_5pt(64)
    from oracle.lanczos import lambda_max_SA
    lm = lambda_max_SA(lambda x: A @ x, 1 / A.diagonal(), A.shape[0], dense_limit=0)
    assert abs(lm - (1 + np.cos(np.pi / 64))) < 1e-10


def test_fd_approximation_constant_unit_aspect():
    # Sec. 3: C ~ 4 for L_x = 1 with n_c = n/2 (first level of the n = 64 grid)
    As, Ps, _ = fd2d.hierarchy_matrices(64, 2)
    C = an.approximation_constant(As[0].toarray(), Ps[0].toarray(), As[1].toarray())
    assert 3.9 < C < 4.1


@pytest.mark.parametrize("kind", [cheb.CHEB4, cheb.CHEB4_OPT, cheb.CHEB1_OPT])
def test_multilevel_bound_holds(kind):
    # Lemma multilevel-poly-bound: ||E_fine-to-coarse||_A^2 <= max_j C_j / (C_j + 1/gamma)
    n, k = 16, 2
    h = fd2d.fd_hierarchy(n, 2, kind, 2 * k, 0, coarsest_n=2)
    As, Ps = h.extra["As"], h.extra["Ps"]
    A = As[0].toarray()
    E = an.error_propagator(h.vcycle, A)
    lhs = an.a_norm(E, A) ** 2
    Cs = [an.approximation_constant(As[j].toarray(), Ps[j].toarray(), As[j + 1].toarray())
          for j in range(len(Ps))]
    g = an.gamma_inv(kind, 2 * k)
    bound = max(C / (C + g) for C in Cs)
    assert lhs <= bound + 1e-12


def test_symmetric_cycle_is_symmetric_one_sided_is_not():
    n = 16
    hs = fd2d.fd_hierarchy(n, 2, cheb.CHEB4, 2, 2, coarsest_n=2)
    M = np.column_stack([hs.vcycle(e) for e in np.eye(hs.levels[0].n)])
    assert np.max(np.abs(M - M.T)) < 1e-12 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(0.5 * (M + M.T))[0] > 0
    h1 = fd2d.fd_hierarchy(n, 2, cheb.CHEB4, 4, 0, coarsest_n=2)
    M1 = np.column_stack([h1.vcycle(e) for e in np.eye(h1.levels[0].n)])
    assert np.max(np.abs(M1 - M1.T)) > 1e-6 * np.max(np.abs(M1))


def test_coarse_solve_exact():
    box = SemBox(wl.deformed_box(4, 0.05), 1)
    solve = mg.exact_coarse(box.assemble())
    b = wl.uniform_noise(box.n, 3)
    x = solve(b)
    assert np.linalg.norm(box.apply(x) - b) <= 1e-13 * np.linalg.norm(b)


def test_pcg_identity_preconditioner_finite_termination():
    # CG on a matrix with 6 distinct eigenvalues terminates in 6 iterations
    d = np.repeat([1.0, 2.0, 3.5, 7.0, 11.0, 20.0], 5)
    b = wl.uniform_noise(d.size, 4)
    res = krylov.pcg(lambda x: d * x, b, lambda r: r.copy(), tol=1e-13, maxit=50)
    assert res.converged and res.iterations == 6
    assert np.max(np.abs(res.x - b / d)) < 1e-12


def test_pcg_exact_preconditioner_one_iteration_and_dense_solution():
    A = fd2d.laplacian_5pt(10).toarray()
    b = wl.uniform_noise(A.shape[0], 5)
    Ainv = np.linalg.inv(A)
    res = krylov.pcg(lambda x: A @ x, b, lambda r: Ainv @ r, tol=1e-10, maxit=5)
    assert res.iterations == 1
    res = krylov.pcg(lambda x: A @ x, b, lambda r: r / np.diag(A), tol=1e-12, maxit=500)
    assert np.max(np.abs(res.x - np.linalg.solve(A, b))) < 1e-9 * np.max(np.abs(res.x))


def test_flexible_equals_standard_for_symmetric_preconditioner():
    h = fd2d.fd_hierarchy(32, 2, cheb.CHEB4, 2, 2, coarsest_n=4)
    A = h.extra["As"][0]
    b = wl.fd_rhs(31, 0)
    r1 = krylov.pcg(lambda x: A @ x, b, h.vcycle, 1e-8, 50, flexible=False)
    r2 = krylov.pcg(lambda x: A @ x, b, h.vcycle, 1e-8, 50, flexible=True)
    assert r1.iterations == r2.iterations
    assert np.max(np.abs(np.array(r1.history) - np.array(r2.history))) < 1e-9 * r1.history[0]


def test_matvec_accounting_m_plus_n_plus_1():
    # Table fastest_solver_fd: fine mat-vecs = iterations x (m + n + 1)
    table = np.loadtxt(__file__.replace("test_oracle_mg.py", "golden/fastest_solver_fd.txt"),
                       dtype=int, comments="#")
    for m, n, matvec, iters in table[:, 2:6]:
        assert matvec == iters * (m + n + 1)
    for (pre, post) in [(4, 0), (2, 2), (3, 1)]:
        h = fd2d.fd_hierarchy(64, 2, cheb.CHEB4, pre, post, coarsest_n=8)
        A = h.extra["As"][0]
        calls = cheb.ApplyCounter(lambda x: A @ x)
        h.reset_counters()
        res = krylov.pcg(calls, wl.fd_rhs(63, 0), h.vcycle, 1e-8, 100, flexible=True)
        # one V-cycle per iteration (the first before the loop, none after convergence)
        assert h.levels[0].applies + calls.count == res.iterations * (pre + post + 1)


def test_sem_pmg_solve_small():
    V = wl.deformed_box(3, 0.05)
    for kind, pre, post in [(cheb.CHEB4_OPT, 4, 0), (cheb.CHEB1, 2, 2), (cheb.CHEB4, 2, 2),
                            (cheb.CHEB1_OPT, 4, 0)]:
        h = mg.sem_hierarchy(V, 5, kind, pre, post)
        box = h.extra["boxes"][0]
        b = box.mass() * wl.manufactured_load(box.coords())
        res = krylov.pcg(box.apply, b, h.vcycle, 1e-10, 60, flexible=True)
        assert res.converged and res.iterations < 25
        x = spla.spsolve(box.assemble().tocsc(), b)
        assert np.max(np.abs(res.x - x)) < 1e-8 * np.max(np.abs(x))


def test_lanczos_matches_dense_eigensolver():
    from oracle.lanczos import lambda_max_SA, lambda_max_dense
    box = SemBox(wl.deformed_box(2, 0.05), 5)   # 729 unknowns
    A = box.assemble().toarray()
    Sinv = 1.0 / box.diag()
    dense = lambda_max_dense(A, Sinv)
    lz = lambda_max_SA(box.apply, Sinv, box.n, dense_limit=0)
    assert abs(lz - dense) < 1e-10 * dense


# ---- geometric multigrid on the order-1 vertex lattice below the p-levels
def test_lattice_interpolation_is_the_trilinear_hat():
    """P e_c (one coarse vertex) is the coarse trilinear hat sampled on the fine lattice:
    the product over x, y, z of max(0, 1 - |fine index - 2 * coarse index| / 2)."""
    m = (8, 6, 4)
    Px, Py, Pz = (mg.trilinear_1d(v) for v in m)
    import scipy.sparse as sp
    P = sp.kron(Pz, sp.kron(Py, Px)).tocsr()
    nf = [v - 1 for v in m]
    nc = [v // 2 - 1 for v in m]
    assert P.shape == (np.prod(nf), np.prod(nc))
    for (ci, cj, ck) in [(1, 1, 1), (3, 2, 1), (2, 1, 1)]:
        e = np.zeros(np.prod(nc))
        e[(ci - 1) + nc[0] * ((cj - 1) + nc[1] * (ck - 1))] = 1.0
        I, J, K = np.meshgrid(np.arange(1, nf[0] + 1), np.arange(1, nf[1] + 1), np.arange(1, nf[2] + 1),
                              indexing="ij")
        hat = (np.maximum(0, 1 - np.abs(I - 2 * ci) / 2) * np.maximum(0, 1 - np.abs(J - 2 * cj) / 2)
               * np.maximum(0, 1 - np.abs(K - 2 * ck) / 2))
        expect = hat.transpose(2, 1, 0).ravel()   # x fastest
        assert np.max(np.abs(P @ e - expect)) == 0.0


def test_lattice_galerkin_operator_closed_form_on_undeformed_box():
    """On an undeformed box the order-1 GLL operator is sum over axes of K (x) M (x) M with
    the 1D stiffness K = tridiag(-1, 2, -1)/h and the lumped mass M = h I. Linear
    interpolation keeps the stiffness (P^T K_h P = K_H, H = 2h) and turns the lumped mass
    into H tridiag(1/8, 3/4, 1/8), so the Galerkin lattice operator is that Kronecker sum."""
    import scipy.sparse as sp
    m = (8, 4, 6)
    V = wl.box_vertices(*m)
    h = mg.sem_hierarchy(V, 3, cheb.CHEB4, 2, 2, lmax=[2.0, 2.0, 2.0], coarse="lattice", dense_max=8)
    As = h.extra["lattice_As"]
    assert len(As) == 2 and As[1].shape[0] == 3 * 1 * 2

    def K(nint, H):
        k = nint - 1
        return sp.diags([-np.ones(k - 1), 2 * np.ones(k), -np.ones(k - 1)], [-1, 0, 1]) / H

    def Mg(nint, H):
        k = nint - 1
        return H * sp.diags([np.full(k - 1, 1 / 8), np.full(k, 3 / 4), np.full(k - 1, 1 / 8)], [-1, 0, 1])

    mc = [v // 2 for v in m]
    Hs = [2.0 / v for v in m]   # coarse spacing 2h with h = 1/m
    Kx, Ky, Kz = (K(n, H) for n, H in zip(mc, Hs))
    Mx, My, Mz = (Mg(n, H) for n, H in zip(mc, Hs))
    expect = sp.kron(Mz, sp.kron(My, Kx)) + sp.kron(Mz, sp.kron(Ky, Mx)) + sp.kron(Kz, sp.kron(My, Mx))
    assert abs(As[1] - expect).max() < 1e-13 * abs(expect).max()


def test_lattice_multigrid_cycle_is_symmetric_and_reduces_to_exact():
    """With symmetric smoothing the whole cycle (p-levels, then the lattice levels, exact
    solve on the last) is a symmetric positive definite operator; with dense_max above
    the order-1 size it is the cycle with the exact order-1 solve."""
    V = wl.deformed_box(4, 0.05)
    h = mg.sem_hierarchy(V, 3, cheb.CHEB4, 2, 2, coarse="lattice", dense_max=8)
    assert [lev.n for lev in h.levels] == [11 ** 3, 3 ** 3, 1]
    r1, r2 = wl.uniform_noise(h.levels[0].n, 1), wl.uniform_noise(h.levels[0].n, 2)
    a, b = r2 @ h.vcycle(r1), r1 @ h.vcycle(r2)
    assert abs(a - b) <= 1e-12 * abs(a)
    assert r1 @ h.vcycle(r1) > 0
    lm = [lev.lmax for lev in h.levels[:2]]
    he = mg.sem_hierarchy(V, 3, cheb.CHEB4, 2, 2, lmax=lm[:1])
    hx = mg.sem_hierarchy(V, 3, cheb.CHEB4, 2, 2, lmax=lm[:1], coarse="lattice", dense_max=27)
    assert np.array_equal(he.vcycle(r1), hx.vcycle(r1))
    # an inexact lattice cycle still gives a convergent preconditioned solve
    box = h.extra["boxes"][0]
    res = krylov.pcg(box.apply, r1, h.vcycle, 1e-10, 60, flexible=True)
    assert res.converged
