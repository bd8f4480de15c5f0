"""Operator with geometric factors formed inside the kernel from the trilinear element
geometry (G = w |J| J^{-1} J^{-T} of the SEM quadrature, eq. poisson) against the oracle,
whose factors come from spectral differentiation of the mapped GLL coordinates: the two
agree up to rounding for trilinear elements.
"""
import numpy as np
import pytest
import torch

import workload as wl
from oracle import chebyshev as cheb
from oracle import krylov, mg
from oracle.sem import SemBox
from paper_2210_03179_amd import _lib as L
from paper_2210_03179_amd.solver import SemSolver

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("N", list(range(1, 13)))
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_trilinear_operator_parity(N, variant, monkeypatch):
    print(f"trilinear operator N={N} variant {variant}", flush=True)
    monkeypatch.setenv("SEMCHEB_AX_VARIANT", str(variant))
    V = wl.deformed_box((3, 2, 3), 0.08)
    box = SemBox(V, N)
    s = SemSolver(V, N=N, orders=[N, 1] if N > 1 else [1], lambda_max=[1.0] * 8, precision="mixed",
                  geometry="trilinear")
    u = wl.uniform_noise(box.n, 3)
    w = s.apply_A(dev(u)).cpu().numpy()
    ref = box.apply(u)
    assert np.max(np.abs(w - ref)) <= 1e-13 * (N + 1) ** 2 * np.max(np.abs(ref))
    # element-local FP32 result with the factors formed in single precision
    w64 = s.apply_local(dev(u))
    w32 = s.apply_local(dev(u).float())
    assert torch.max(torch.abs(w32.double() - w64)) <= 2e-5 * (N + 1) ** 2 * torch.max(torch.abs(w64))


def test_trilinear_solve_matches_oracle():
    V = wl.deformed_box((3, 3, 4), 0.05)
    N = 5
    ref = mg.sem_hierarchy(V, N, cheb.CHEB4_OPT, 4, 0)
    lmax = [lev.lmax for lev in ref.levels[:-1]]
    box = ref.extra["boxes"][0]
    b = box.mass() * wl.manufactured_load(box.coords()) + 1e-2 * wl.uniform_noise(box.n, 4)
    res = krylov.pcg(box.apply, b, ref.vcycle, 1e-10, 200, flexible=True)
    s = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, lambda_max=lmax, geometry="trilinear")
    u, info = s.solve(dev(b), rtol=1e-10, maxit=200)
    assert info.converged and info.iterations == res.iterations
    assert np.max(np.abs(info.history - np.array(res.history))) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(u.cpu().numpy() - res.x) <= 1e-11 * np.linalg.norm(res.x)


def test_trilinear_mixed_reaches_fp64_residual():
    V = wl.deformed_box(4, 0.05)
    box = SemBox(V, 7)
    b = box.mass() * wl.manufactured_load(box.coords()) + 1e-3 * wl.uniform_noise(box.n, 0)
    s = SemSolver(V, N=7, precision="mixed", geometry="trilinear")
    u, info = s.solve(dev(b), rtol=1e-8, maxit=100)
    assert info.converged
    true = np.linalg.norm(b - box.apply(u.cpu().numpy())) / np.linalg.norm(b)
    assert true <= 1.01e-8
    s64 = SemSolver(V, N=7, precision="fp64")
    _, info64 = s64.solve(dev(b), rtol=1e-8, maxit=100)
    assert abs(info.iterations - info64.iterations) <= 1


def test_trilinear_has_no_stored_factors():
    V = wl.deformed_box(3, 0.05)
    s = SemSolver(V, N=4, geometry="trilinear")
    with pytest.raises(L.SemError) as ex:
        s.factors()
    assert ex.value.status == L.SEM_EINVAL
    tune = s.host_array("ax_tuning")
    nvar = (len(tune) // s.num_levels - 2) // 2
    per = 2 * (1 + nvar)
    for j in range(s.num_levels - 1):   # three variants timed, the others marked -1
        t64 = tune[j * per + 1: j * per + 1 + nvar]
        assert np.all(t64[:3] > 0) and np.all(t64[3:] == -1)
