"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (FP64): operator 1e-14 (N+1)^2 relative in the max norm (its rounding
grows with the size of the GLL derivative entries, ~N^2/4), V-cycle
1e-12 relative (2-norm), PCG/FCG solves: identical iteration counts, every
residual norm within 1e-12 ||b||, solution within 1e-12 relative. lambda_max
is estimated by the oracle and handed to both sides, so the solve comparison
does not depend on the two eigenvalue estimators, which are compared on their
own.
"""
import numpy as np
import pytest
import torch

import rounding
import workload as wl
from oracle import adjoint, chebyshev as cheb, fd2d, krylov, mg
from oracle.sem import SemBox
from paper_2210_03179_amd import _lib as L
from paper_2210_03179_amd.solver import SemSolver, FdSolver

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ------------------------------------------------------------------ operator
@pytest.mark.parametrize("m,N", [((2, 3, 2), N) for N in range(1, 13)] + [((8, 8, 8), 7), ((3, 2, 4), 5)])
def test_apply_A_parity(m, N):
    print(f"apply_A parity m={m} N={N}", flush=True)
    V = wl.deformed_box(m, 0.05)
    box = SemBox(V, N)
    # order 1 alone is a one-level hierarchy (its cycle is the coarse solve)
    s = SemSolver(V, N=N, lambda_max=[1.0] * 8, orders=[N, 1] if N > 1 else [1])
    u = wl.uniform_noise(box.n, 11)
    w = host(s.apply_A(dev(u)))
    assert relmax(w, box.apply(u)) < 1e-14 * (N + 1) ** 2


@pytest.mark.parametrize("variant", range(7))
@pytest.mark.parametrize("N", [2, 3, 4, 5, 7, 9])
def test_operator_variants_parity(N, variant, monkeypatch):
    # every operator kernel variant the autotuner may pick, FP64 and FP32/BF16, against the oracle
    print(f"operator variant {variant} N={N}", flush=True)
    monkeypatch.setenv("SEMCHEB_AX_VARIANT", str(variant))
    V = wl.deformed_box((3, 2, 3), 0.05)
    box = SemBox(V, N)
    s = SemSolver(V, N=N, lambda_max=[1.0] * 8, orders=[N, 1], precision="mixed")
    u = wl.uniform_noise(box.n, 12)
    w = host(s.apply_A(dev(u)))
    assert relmax(w, box.apply(u)) < 1e-14 * (N + 1) ** 2
    # element-local outputs: FP64 path exact to rounding; FP32 arithmetic with BF16 factors
    # within the factors' 2^-8 relative rounding
    wl64 = host(s.apply_local(dev(u)))
    wl32 = s.apply_local(dev(u).float()).double().cpu().numpy()
    ref = box.apply_local(box.scatter(u)).ravel()
    assert relmax(wl64, ref) < 1e-14 * (N + 1) ** 2
    assert relmax(wl32, ref) < 1e-2  # BF16 rounding of the factors alone gives up to 2.4e-3 here


def test_apply_A_order1_and_deterministic():
    V = wl.deformed_box((3, 3, 2), 0.05)
    s = SemSolver(V, N=2, orders=[2, 1], lambda_max=[1.0])
    box = SemBox(V, 2)
    u = dev(wl.uniform_noise(box.n, 5))
    a, b = host(s.apply_A(u)), host(s.apply_A(u))
    assert np.array_equal(a, b)


# ------------------------------------------------------------------ V-cycle
@pytest.fixture(scope="module")
def small_case():
    V = wl.deformed_box((3, 3, 4), 0.05)
    N = 5
    ref = mg.sem_hierarchy(V, N, cheb.CHEB4, 2, 2)
    lmax = [lev.lmax for lev in ref.levels[:-1]]
    return V, N, lmax


@pytest.mark.parametrize("kind", ["cheb1", "cheb1opt", "cheb4", "cheb4opt"])
@pytest.mark.parametrize("pre,post", [(4, 0), (2, 2), (3, 1), (1, 0), (0, 3)])
def test_vcycle_parity(small_case, kind, pre, post):
    print(f"vcycle parity {kind} ({pre},{post})", flush=True)
    V, N, lmax = small_case
    ref = mg.sem_hierarchy(V, N, kind, pre, post, lmax=lmax)
    s = SemSolver(V, N=N, smoother=kind, pre=pre, post=post, lambda_max=lmax)
    r = wl.uniform_noise(ref.levels[0].n, 3)
    z = host(s.vcycle(dev(r)))
    zo = ref.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)
    # fine-level operator applications per cycle: (pre - 1) + 1 + post from a zero guess
    cnt = s.apply_counts()
    expect0 = (pre - 1 + 1 if pre > 0 else 0) + post
    assert cnt[0] == expect0
    assert cnt[-1] == 0


def test_lanczos_matches_oracle(small_case):
    V, N, lmax = small_case
    s = SemSolver(V, N=N)
    got = s.lambda_max()
    assert len(got) == len(lmax)
    for a, b in zip(got, lmax):
        assert abs(a - b) <= 1e-8 * b


# ------------------------------------------------------------------ solves
@pytest.fixture(scope="module")
def cfg2():
    """8x8x8 deformed box (amplitude 0.05), N=7, schedule (7,3,1), opt. 4th kind (4,0),
    manufactured load plus 1e-3 relative U[-1,1] noise (seed 0)."""
    V = wl.deformed_box(8, 0.05)
    ref = mg.sem_hierarchy(V, 7, cheb.CHEB4_OPT, 4, 0)
    box = ref.extra["boxes"][0]
    b0 = box.mass() * wl.manufactured_load(box.coords())
    b = b0 + 1e-3 * np.max(np.abs(b0)) * wl.uniform_noise(box.n, 0)
    lmax = [lev.lmax for lev in ref.levels[:-1]]
    return V, ref, box, b, lmax


def _solve_parity(s, ref, Aop, b, flexible, tol=1e-8, maxit=200):
    res = krylov.pcg(Aop, b, ref.vcycle, tol, maxit, flexible=flexible)
    u, info = s.solve(dev(b), rtol=tol, maxit=maxit)
    u = host(u)
    assert info.converged and res.converged
    assert info.iterations == res.iterations
    h_o = np.array(res.history)
    assert np.max(np.abs(info.history - h_o)) <= 1e-12 * h_o[0]
    assert np.linalg.norm(u - res.x) <= 1e-12 * np.linalg.norm(res.x)
    margin = (tol * h_o[0] - h_o[-1]) / (tol * h_o[0])
    print(f"iterations {info.iterations}, last-iteration margin to tol {margin:.3e}", flush=True)
    return u, info, res


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pcg_one_sided_history_parity(small_case, precision):
    # plain CG with a one-sided cycle (a non-symmetric preconditioner) stagnates, here and in
    # the oracle; its first iterations still agree, which covers the single z.r reduction the
    # cycle's last prolongation computes for CG (flexible CG takes two)
    V, N, lmax = small_case
    print(f"pcg one-sided history {precision}", flush=True)
    ref = mg.sem_hierarchy(V, N, "cheb4opt", 4, 0, lmax=lmax)
    box = ref.extra["boxes"][0]
    b = box.mass() * wl.manufactured_load(box.coords()) + 1e-2 * wl.uniform_noise(box.n, 1)
    s = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, krylov="pcg", lambda_max=lmax,
                  precision=precision)
    its = 12
    res = krylov.pcg(box.apply, b, ref.vcycle, 1e-8, its, flexible=False)
    u, info = s.solve(dev(b), rtol=1e-8, maxit=its)
    assert not res.converged and not info.converged
    assert info.iterations == res.iterations == its
    h_o = np.array(res.history)
    if precision == "fp64":
        assert np.max(np.abs(info.history - h_o)) <= 1e-10 * h_o[0]
        assert np.linalg.norm(host(u) - res.x) <= 1e-10 * np.linalg.norm(res.x)
    else:  # single-precision cycle: the same descent, within the BF16 factors' rounding
        assert np.max(np.abs(info.history - h_o) / h_o) <= 0.2


def test_cfg2_rhs_parity(cfg2):
    V, ref, box, b, lmax = cfg2
    s = SemSolver(V, N=7, lambda_max=lmax)
    f = wl.manufactured_load(host(s.coords()))
    bg = host(s.mass_apply(dev(f)))
    err = relmax(bg, box.mass() * wl.manufactured_load(box.coords()))
    # 1e-13 lies below the first-order bound on two FP64 evaluations of the mass (1.7e-11 here,
    # tests/rounding.py); the coordinates' rounding, amplified by differentiation, sets it
    print(f"cfg2 rhs: {err:.2e} (tolerance 1e-13, bound {rounding.mass_bound(box):.1e})", flush=True)
    assert 1e-13 <= rounding.mass_bound(box)
    assert err < 1e-13


def test_cfg2_solve_parity(cfg2):
    V, ref, box, b, lmax = cfg2
    s = SemSolver(V, N=7, smoother="cheb4opt", pre=4, post=0, krylov="fcg", lambda_max=lmax)
    s.reset_counts()
    u, info, res = _solve_parity(s, ref, box.apply, b, flexible=True)
    # fine-grid mat-vecs = iterations x (m + n + 1)
    assert s.apply_counts()[0] == info.iterations * (4 + 0 + 1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_matches_direct_launches(cfg2, precision, monkeypatch):
    # V-cycles replayed from captured graphs (default) against the same kernels launched one by
    # one: every replay of a solve, and repeated solves with host work in between, are bitwise equal
    V, ref, box, b, lmax = cfg2
    print(f"graph replay {precision}", flush=True)
    # both contexts use the same operator variant (the autotuner may pick different ones, whose
    # rounding differs)
    monkeypatch.setenv("SEMCHEB_AX_VARIANT", "0")
    monkeypatch.setenv("SEMCHEB_GRAPHS", "0")
    direct = SemSolver(V, N=7, precision=precision, lambda_max=lmax)
    monkeypatch.delenv("SEMCHEB_GRAPHS")
    graph = SemSolver(V, N=7, precision=precision, lambda_max=lmax)
    ud, infod = direct.solve(dev(b))
    direct.reset_counts()
    direct.solve(dev(b))
    counts_direct = direct.apply_counts()
    for rep in range(3):
        graph.reset_counts()
        ug, infog = graph.solve(dev(b))
        assert infog.iterations == infod.iterations
        assert np.array_equal(infog.history, infod.history), rep
        assert torch.equal(ug, ud), rep
        assert graph.apply_counts() == counts_direct
        zg = graph.vcycle(dev(b))  # eager cycle between replays
        assert torch.isfinite(zg).all()


@pytest.mark.parametrize("kind,pre,post,kry", [("cheb4", 2, 2, "pcg"), ("cheb1", 3, 3, "pcg"),
                                               ("cheb1opt", 4, 0, "fcg"), ("cheb4opt", 2, 2, "fcg")])
def test_small_solve_parity(small_case, kind, pre, post, kry):
    V, N, lmax = small_case
    ref = mg.sem_hierarchy(V, N, kind, pre, post, lmax=lmax)
    box = ref.extra["boxes"][0]
    b = box.mass() * wl.manufactured_load(box.coords()) + 1e-2 * wl.uniform_noise(box.n, 1)
    s = SemSolver(V, N=N, smoother=kind, pre=pre, post=post, krylov=kry, lambda_max=lmax)
    _solve_parity(s, ref, box.apply, b, flexible=(kry == "fcg"))


def test_solve_nonzero_initial_guess(small_case):
    V, N, lmax = small_case
    s = SemSolver(V, N=N, lambda_max=lmax)
    box = SemBox(V, N)
    b = dev(wl.uniform_noise(box.n, 2))
    x0 = dev(wl.uniform_noise(box.n, 3))
    u, info = s.solve(b, x0=x0, rtol=1e-10)
    assert info.converged
    r0 = host(b) - box.apply(host(x0))
    assert abs(info.history[0] - np.linalg.norm(r0)) <= 1e-12 * np.linalg.norm(r0)
    assert np.linalg.norm(box.apply(host(u)) - host(b)) <= 2e-10 * np.linalg.norm(host(b))


def test_solve_edge_cases(small_case):
    V, N, lmax = small_case
    s = SemSolver(V, N=N, lambda_max=lmax)
    n = s.n
    u, info = s.solve(torch.zeros(n, dtype=torch.float64, device="cuda"))
    assert info.converged and info.iterations == 0 and float(u.abs().max()) == 0.0
    b = dev(wl.uniform_noise(n, 4))
    u, info = s.solve(b, rtol=1e-14, maxit=3)
    assert info.status == L.SEM_ENOTCONV and info.iterations == 3
    bad = b.clone()
    bad[7] = float("nan")
    with pytest.raises(L.SemError) as e:
        s.solve(bad)
    assert e.value.status == L.SEM_ENAN
    # deterministic: two solves are bitwise identical, also into a preallocated output
    u1, _ = s.solve(b)
    u2, _ = s.solve(b)
    assert torch.equal(u1, u2)
    out = torch.full_like(b, 7.0)
    u3, _ = s.solve(b, out=out)
    assert u3.data_ptr() == out.data_ptr() and torch.equal(u3, u1)


# ------------------------------------------------------------------ finite differences (config 1)
@pytest.mark.parametrize("pre,post,kry", [(4, 0, "fcg"), (2, 2, "pcg"), (2, 2, "fcg")])
def test_fd_cfg1_parity(pre, post, kry):
    """2D FD, 63x63 interior, levels 63/31/15/7 Galerkin, 4th-kind Chebyshev, rhs U[-1,1] seed 0."""
    ref = fd2d.fd_hierarchy(64, 2, cheb.CHEB4, pre, post, coarsest_n=8)
    lmax = [lev.lmax for lev in ref.levels[:-1]]
    s = FdSolver(n=64, factor=2, coarsest_n=8, smoother="cheb4", pre=pre, post=post, krylov=kry,
                 lambda_max=lmax)
    b = wl.fd_rhs(63, 0)
    A = ref.extra["As"][0]
    s.reset_counts()
    u, info, res = _solve_parity(s, ref, lambda x: A @ x, b, flexible=(kry == "fcg"))
    assert s.apply_counts()[0] == info.iterations * (pre + post + 1)


def test_fd_lanczos_exact():
    s = FdSolver(n=64, factor=2, coarsest_n=8)
    assert abs(s.lambda_max()[0] - (1 + np.cos(np.pi / 64))) < 1e-9


# ------------------------------------------------------------------ mixed precision
def test_mixed_precision_reaches_fp64_residual(cfg2):
    V, ref, box, b, lmax = cfg2
    s = SemSolver(V, N=7, precision="mixed", krylov="fcg", lambda_max=lmax)
    u, info = s.solve(dev(b), rtol=1e-8)
    assert info.converged
    uh = host(u)
    true_rel = np.linalg.norm(b - box.apply(uh)) / np.linalg.norm(b)
    assert true_rel <= 1.01e-8
    s64 = SemSolver(V, N=7, lambda_max=lmax)
    u64, info64 = s64.solve(dev(b), rtol=1e-8)
    err = np.linalg.norm(uh - host(u64)) / np.linalg.norm(host(u64))
    print(f"mixed: {info.iterations} its (fp64 {info64.iterations}), true rel res {true_rel:.2e}, "
          f"||u-u64||/||u64|| {err:.2e}", flush=True)
    assert err < 1e-7


# ------------------------------------------------------------------ adjoint contraction
def test_adjoint_contract_parity():
    V = wl.deformed_box((3, 4, 3), 0.05)
    N = 5
    box = SemBox(V, N)
    s = SemSolver(V, N=N, lambda_max=[2.0, 2.0])
    lam = wl.uniform_noise(box.n, 8)
    u = wl.uniform_noise(box.n, 9)
    dG, df = s.adjoint_contract(dev(lam), dev(u))
    ref = adjoint.contract(box, lam, u)
    e_dG = relmax(host(dG), ref)
    e_df = relmax(host(df), box.mass() * lam)
    e_G = relmax(host(s.factors()), box.G)
    # df = B lambda carries the mass's rounding (bound 18 u kappa), G the factors' (30 u kappa);
    # the fixed tolerances lie below both bounds (tests/rounding.py). dG multiplies gradients of
    # lambda and u: neither the coordinates nor the factors enter it
    print(f"adjoint: dG {e_dG:.2e}, df {e_df:.2e} (bound {rounding.mass_bound(box):.1e}), "
          f"G {e_G:.2e} (bound {rounding.factor_bound(box):.1e})", flush=True)
    assert 1e-14 <= rounding.mass_bound(box) and 1e-13 <= rounding.factor_bound(box)
    assert e_dG < 1e-13
    assert e_df < 1e-14
    assert e_G < 1e-13


@pytest.mark.parametrize("planes", [1, 2])
def test_blocked_coarse_solve_parity(small_case, planes):
    # the coarse order-1 solve split into blocks of z-planes (block-tridiagonal elimination)
    V, N, lmax = small_case
    ref = mg.sem_hierarchy(V, N, cheb.CHEB4, 2, 2, lmax=lmax)
    s = SemSolver(V, N=N, smoother="cheb4", pre=2, post=2, lambda_max=lmax, coarse_planes=planes)
    r = wl.uniform_noise(ref.levels[0].n, 6)
    z = host(s.vcycle(dev(r)))
    zo = ref.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)


def test_mixed_cycle_single_precision_coarse_factors(small_case, monkeypatch):
    # with coarse_storage="mixed" the mixed cycle reads single-precision copies of the coarse
    # factor blocks: the dense inverse
    # (planes = 0 on this small mesh) and the two-ended block elimination (1 or 2 planes per block)
    # are different factorizations of one matrix, so their cycles differ only by the rounding of
    # the stored factors; all three stay within the mixed cycle's BF16 accuracy of the FP64 oracle
    monkeypatch.setenv("SEMCHEB_AX_VARIANT", "0")  # the same operator kernel in all three
    V, N, lmax = small_case
    ref = mg.sem_hierarchy(V, N, cheb.CHEB4, 2, 2, lmax=lmax)
    r = wl.uniform_noise(ref.levels[0].n, 6)
    zo = ref.vcycle(r)
    zs = []
    for planes in (0, 1, 2):
        s = SemSolver(V, N=N, smoother="cheb4", pre=2, post=2, lambda_max=lmax, coarse_planes=planes,
                      precision="mixed", coarse_storage="mixed")
        zs.append(host(s.vcycle(dev(r))))
        assert np.linalg.norm(zs[-1] - zo) <= 1e-2 * np.linalg.norm(zo), planes
    for z in zs[1:]:
        assert np.linalg.norm(z - zs[0]) <= 1e-5 * np.linalg.norm(zs[0])


@pytest.mark.parametrize("nz,planes", [(9, 1), (8, 1), (9, 3), (6, 2)])
def test_blocked_coarse_solve_block_counts(nz, planes):
    # two-ended block elimination with an even (8) and odd (7, 3) number of blocks and a
    # ragged last block (8 planes in blocks of 3)
    print(f"blocked coarse nz={nz} planes={planes}", flush=True)
    V = wl.deformed_box((3, 2, nz), 0.05)
    N = 3
    ref = mg.sem_hierarchy(V, N, cheb.CHEB4, 2, 0)
    lmax = [lev.lmax for lev in ref.levels[:-1]]
    s = SemSolver(V, N=N, smoother="cheb4", pre=2, post=0, lambda_max=lmax, coarse_planes=planes)
    r = wl.uniform_noise(ref.levels[0].n, 16)
    z = host(s.vcycle(dev(r)))
    zo = ref.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)


def test_breakdown_on_indefinite_preconditioner():
    """A lambda_max override far below the true lambda_max(S A) makes the Chebyshev
    smoother amplify the upper spectrum with alternating signs, so the V-cycle is no
    longer positive definite. The oracle shows r.z < 0 for the first residual of this
    input; the library must then stop with SEM_EBREAKDOWN (r.z <= 0) instead of
    iterating on a meaningless alpha."""
    from oracle import fd2d
    from oracle.lanczos import lambda_max_SA
    from paper_2210_03179_amd.solver import FdSolver
    As, _, _ = fd2d.hierarchy_matrices(16, 2, 1.0, 1.0, coarsest_n=2)
    true = [lambda_max_SA(lambda x, A=A: A @ x, 1.0 / A.diagonal(), A.shape[0]) for A in As[:-1]]
    bad = [0.3 * t for t in true]
    b = wl.uniform_noise(As[0].shape[0], 0)
    ref = fd2d.fd_hierarchy(16, 2, "cheb4", 2, 2, coarsest_n=2, lmax=bad)
    assert float(b @ ref.vcycle(b)) < -float(b @ b)   # indefinite, by a wide margin
    for krylov in ("pcg", "fcg"):
        s = FdSolver(n=16, factor=2, coarsest_n=2, smoother="cheb4", pre=2, post=2, krylov=krylov,
                     lambda_max=bad)
        with pytest.raises(L.SemError) as ex:   # the binding raises for every status but OK / ENOTCONV
            s.solve(dev(b), rtol=1e-8, maxit=50)
        assert ex.value.status == L.SEM_EBREAKDOWN and "breakdown" in str(ex.value)
        s.close()
    # the same hierarchy with the true lambda_max converges
    s = FdSolver(n=16, factor=2, coarsest_n=2, smoother="cheb4", pre=2, post=2, krylov="pcg", lambda_max=true)
    u, info = s.solve(dev(b), rtol=1e-8, maxit=50)
    assert info.converged


def test_mixed_cycle_elementwise(cfg2):
    """The mixed-precision cycle (FP32 arithmetic, BF16 factors) node by node against the
    oracle, in the max norm relative to the largest entry:
    - against the FP64 oracle within one BF16 unit roundoff, 2^-9 (the factors' storage
      rounding alone moves this cycle by about 6e-4);
    - against the oracle run with the same BF16-rounded factors (FP64 arithmetic) within
      1e-5: what is left is the FP32 arithmetic (unit roundoff 6e-8, measured 1.9e-7 over
      the cycle's operator applications and transfers), so a wrong node shows up here far
      above the rounding level."""
    V, ref, box, b, lmax = cfg2
    r = wl.uniform_noise(box.n, 5)
    zo = ref.vcycle(r)
    hb = mg.sem_hierarchy(V, 7, cheb.CHEB4_OPT, 4, 0, lmax=lmax)
    for bx in hb.extra["boxes"][:-1]:   # the smoothed levels store BF16 factors on the GPU
        bx.G[:] = rounding.bf16_round(bx.G)
    zb = hb.vcycle(r)
    s = SemSolver(V, N=7, precision="mixed", lambda_max=lmax)
    z = host(s.vcycle(dev(r)))
    e64, ebf = relmax(z, zo), relmax(z, zb)
    e2 = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    print(f"mixed cycle 8^3: vs FP64 oracle max-norm {e64:.2e} (2-norm {e2:.2e}), "
          f"vs BF16-factor oracle {ebf:.2e}; BF16 storage alone {relmax(zb, zo):.2e}", flush=True)
    assert e64 <= 2.0 ** -9
    assert ebf <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_krylov_apply_matches_separate_pass(cfg2, precision, monkeypatch):
    """The Krylov operator that reduces p . Ap as sum over nodes of (D u) . G (D u) and leaves
    A p as element copies for the residual update, against the separate summation pass with
    p . Ap from the summed vector: the same iterations, histories within 1e-13 ||b|| in FP64.
    A mixed cycle gets the FP32 copy of the residual: a last-bit change of the FP64 residual
    can move that copy by one FP32 unit (6e-8 relative), which the single-precision cycle
    carries into z, so there the histories agree to 1e-10 ||b|| (measured 1.3e-12)."""
    V, ref, box, b, lmax = cfg2
    monkeypatch.setenv("SEMCHEB_AX_VARIANT", "0")
    s1 = SemSolver(V, N=7, precision=precision, lambda_max=lmax)
    u1, i1 = s1.solve(dev(b))
    monkeypatch.setenv("SEMCHEB_FUSED_KRYLOV", "0")
    u2, i2 = s1.solve(dev(b))
    tol = 1e-13 if precision == "fp64" else 1e-10
    assert i1.iterations == i2.iterations
    assert np.max(np.abs(i1.history - i2.history)) <= tol * np.linalg.norm(b)
    assert np.linalg.norm(host(u1) - host(u2)) <= 10 * tol * np.linalg.norm(host(u2))


def test_matrix_core_operator_matches_vector_variant(monkeypatch):
    """The BF16 operator with its contractions on the matrix cores (variant 6, N = 7) against
    the vector-ALU variant with the same BF16 factors in LDS (variant 5): the
    same FP32 products summed in another order, so element by element within a few FP32
    rounding units of the largest entry; 5 x 4 x 3 elements, all boundary cases."""
    V = wl.deformed_box((5, 4, 3), 0.07)
    u = dev(wl.uniform_noise(SemBox(V, 7).n, 21)).float()
    out = {}
    for v in (5, 6):
        monkeypatch.setenv("SEMCHEB_AX_VARIANT", str(v))
        s = SemSolver(V, N=7, lambda_max=[1.0] * 3, precision="mixed")
        out[v] = s.apply_local(u).double().cpu().numpy()
        s.close()
    d = relmax(out[6], out[5])
    print(f"matrix-core vs vector BF16 operator: max rel {d:.2e}", flush=True)
    assert d < 2e-6


def test_krylov_operator_timing(small_case, monkeypatch):
    """SEMCHEB_TIME_KRYLOV_OP=1 makes sem_solve time each Krylov operator launch with an event
    pair on its stream: one positive duration per iteration in "krylov_operator_us", the same
    solve bitwise, and an empty array once a solve runs without the switch."""
    V, N, lmax = small_case
    s = SemSolver(V, N=N, lambda_max=lmax, krylov="fcg")
    b = dev(wl.uniform_noise(s.n, 41))
    u0, info0 = s.solve(b)
    assert s.host_array("krylov_operator_us").size == 0
    monkeypatch.setenv("SEMCHEB_TIME_KRYLOV_OP", "1")
    u1, info1 = s.solve(b)
    t = s.host_array("krylov_operator_us")
    print(f"Krylov operator: {t.size} launches timed, mean {t.mean():.1f} us", flush=True)
    assert t.size == info1.iterations and np.all(t > 0)
    assert torch.equal(u0, u1) and np.array_equal(info0.history, info1.history)
    monkeypatch.delenv("SEMCHEB_TIME_KRYLOV_OP")
    s.solve(b)
    assert s.host_array("krylov_operator_us").size == 0
    s.close()
