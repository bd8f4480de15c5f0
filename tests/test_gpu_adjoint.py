"""Adjoint gradients through torch.autograd on the GPU.

* small mesh: dL/df and dL/dG equal the oracle's gradient (its own solves);
* 16^3 elements, N = 7 (the adjoint workload): central finite differences with
  h = 1e-6 on 32 seeded random unit directions in (f, G) space. Forward and
  adjoint solves run to 1e-13 so that solver error stays far below the
  finite-difference resolution; a direction passes when
  |FD - <grad, v>| <= 1e-6 max(|FD|, 1e-3 ||grad|| ||v||).
Loss: L = ||u - u_t||^2 with u_t a seeded smooth field at the unknowns.
"""
import numpy as np
import pytest
import torch

import workload as wl
from oracle import adjoint, chebyshev as cheb, krylov, mg
from paper_2210_03179_amd.autograd import sem_solve
from paper_2210_03179_amd.solver import SemSolver

pytestmark = pytest.mark.gpu


def test_gradient_matches_oracle():
    V = wl.deformed_box(4, 0.05)
    N = 5
    ref = mg.sem_hierarchy(V, N, cheb.CHEB4_OPT, 4, 4)
    box = ref.extra["boxes"][0]
    lmax = [lev.lmax for lev in ref.levels[:-1]]

    def osolve(rhs, G=None):
        return krylov.pcg(box.apply, rhs, ref.vcycle, 1e-13, 400).x

    xyz = box.coords()
    f = wl.manufactured_load(xyz)
    u_t = wl.target_field(xyz, seed=0)
    L0, u0, dfo, dGo = adjoint.loss_and_grad(box, osolve, f, u_t)

    s = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=4, krylov="pcg", lambda_max=lmax)
    G = s.factors().requires_grad_(True)
    ft = torch.from_numpy(f).cuda().requires_grad_(True)
    ut = torch.from_numpy(u_t).cuda()
    u = sem_solve(ft, G, s, rtol=1e-13)
    loss = ((u - ut) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - L0) <= 1e-11 * L0
    dG = G.grad.cpu().numpy()
    df = ft.grad.cpu().numpy()
    assert np.max(np.abs(df - dfo)) <= 1e-9 * np.max(np.abs(dfo))
    assert np.max(np.abs(dG - dGo)) <= 1e-9 * np.max(np.abs(dGo))


def test_cfg5_finite_differences():
    """16^3 deformed box, N = 7, FP64, opt. 4th-kind (4,4) symmetric V-cycle, PCG."""
    V = wl.deformed_box(16, 0.05)
    s = SemSolver(V, N=7, smoother="cheb4opt", pre=4, post=4, krylov="pcg")
    xyz = s.coords().cpu().numpy()
    f = torch.from_numpy(wl.manufactured_load(xyz)).cuda()
    ut = torch.from_numpy(wl.target_field(xyz, seed=0)).cuda()
    G0 = s.factors()

    def loss_of(ff, GG):
        with torch.no_grad():
            u = sem_solve(ff, GG, s, rtol=1e-13)
            return float(((u - ut) ** 2).sum())

    G = G0.clone().requires_grad_(True)
    fr = f.clone().requires_grad_(True)
    u = sem_solve(fr, G, s, rtol=1e-13)
    loss = ((u - ut) ** 2).sum()
    loss.backward()
    gf, gG = fr.grad.detach(), G.grad.detach()
    gnorm = float(torch.sqrt((gf ** 2).sum() + (gG ** 2).sum()))
    h = 1e-6
    dirs = wl.gaussian_directions(32, (f.numel(), G0.numel()), seed=1)
    worst = 0.0
    for k, (vf, vG) in enumerate(dirs):
        vf_t = torch.from_numpy(vf).cuda()
        vG_t = torch.from_numpy(vG).cuda().reshape(G0.shape)
        lp = loss_of(f + h * vf_t, G0 + h * vG_t)
        lm = loss_of(f - h * vf_t, G0 - h * vG_t)
        fd = (lp - lm) / (2 * h)
        an = float((gf * vf_t).sum() + (gG * vG_t).sum())
        tol = 1e-6 * max(abs(fd), 1e-3 * gnorm)
        worst = max(worst, abs(fd - an) / max(abs(fd), 1e-300))
        assert abs(fd - an) <= tol, (k, fd, an)
    print(f"cfg5 FD check: 32 directions, worst relative difference {worst:.2e}", flush=True)
    s.set_factors(G0)
