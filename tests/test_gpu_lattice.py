"""Lattice multigrid below the order-1 level (coarse="lattice") on the GPU against the
oracle's construction of the same cycle: vertex-lattice levels with trilinear interpolation
and Galerkin operators, Jacobi-Chebyshev smoothing, exact solve of the last level.

FP64: V-cycles to 1e-12 (2-norm and max-norm); FCG/PCG solves with identical iteration
counts, residual histories within 1e-12 ||b|| and solutions within 1e-12. Mixed precision
(the lattice levels stay FP64): the cycle node by node within one BF16 unit roundoff of
the FP64 oracle, and the solve to a true 1e-8 with the oracle's operator. lambda_max of
every smoothed level (p-levels and lattice levels) comes from the oracle."""
import numpy as np
import pytest
import torch

import workload as wl
from oracle import chebyshev as cheb, krylov, mg
from paper_2210_03179_amd.solver import SemSolver

pytestmark = pytest.mark.gpu

DENSE_MAX = 8   # 8^3 elements: order-1 lattice 343 -> 27 -> 1 (dense)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def mesh():
    return wl.deformed_box(8, 0.05)


@pytest.fixture(scope="module")
def lmax(mesh):
    h = mg.sem_hierarchy(mesh, 5, cheb.CHEB4_OPT, 4, 0, coarse="lattice", dense_max=DENSE_MAX)
    assert [lev.n for lev in h.levels] == [39 ** 3, 15 ** 3, 7 ** 3, 3 ** 3, 1]
    return [lev.lmax for lev in h.levels[:-1]]


@pytest.mark.parametrize("kind,pre,post", [("cheb4opt", 4, 0), ("cheb4", 2, 2), ("cheb1", 3, 3), ("cheb1opt", 2, 0)])
def test_lattice_vcycle_parity(mesh, lmax, kind, pre, post):
    print(f"lattice cycle {kind} ({pre},{post})", flush=True)
    ref = mg.sem_hierarchy(mesh, 5, kind, pre, post, lmax=lmax, coarse="lattice", dense_max=DENSE_MAX)
    s = SemSolver(mesh, N=5, smoother=kind, pre=pre, post=post, lambda_max=lmax, coarse="lattice",
                  dense_max=DENSE_MAX)
    assert s.num_levels == 5
    r = wl.uniform_noise(ref.levels[0].n, 31)
    z = s.vcycle(dev(r)).cpu().numpy()
    zo = ref.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)
    assert relmax(z, zo) <= 1e-12
    # every level is applied as often as in the oracle's cycle
    ref.reset_counters()
    s.reset_counts()
    ref.vcycle(r)
    s.vcycle(dev(r))
    torch.cuda.synchronize()
    assert s.apply_counts() == [lev.applies for lev in ref.levels]


@pytest.mark.parametrize("kry", ["fcg", "pcg"])
def test_lattice_solve_parity(mesh, lmax, kry):
    kind, pre, post = ("cheb4opt", 4, 0) if kry == "fcg" else ("cheb4", 2, 2)
    ref = mg.sem_hierarchy(mesh, 5, kind, pre, post, lmax=lmax, coarse="lattice", dense_max=DENSE_MAX)
    box = ref.extra["boxes"][0]
    b0 = box.mass() * wl.manufactured_load(box.coords())
    b = b0 + 1e-3 * np.max(np.abs(b0)) * wl.uniform_noise(box.n, 0)
    res = krylov.pcg(box.apply, b, ref.vcycle, 1e-8, 100, flexible=(kry == "fcg"))
    s = SemSolver(mesh, N=5, smoother=kind, pre=pre, post=post, krylov=kry, lambda_max=lmax, coarse="lattice",
                  dense_max=DENSE_MAX)
    u, info = s.solve(dev(b), rtol=1e-8, maxit=100)
    print(f"lattice {kry}: {info.iterations} iterations (oracle {res.iterations})", flush=True)
    assert info.converged and res.converged and info.iterations == res.iterations
    assert np.max(np.abs(info.history - np.array(res.history))) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(u.cpu().numpy() - res.x) <= 1e-12 * np.linalg.norm(res.x)


def test_lattice_mixed_cycle_and_solve(mesh, lmax):
    ref = mg.sem_hierarchy(mesh, 5, cheb.CHEB4_OPT, 4, 0, lmax=lmax, coarse="lattice", dense_max=DENSE_MAX)
    box = ref.extra["boxes"][0]
    s = SemSolver(mesh, N=5, precision="mixed", lambda_max=lmax, coarse="lattice", dense_max=DENSE_MAX)
    r = wl.uniform_noise(ref.levels[0].n, 32)
    z = s.vcycle(dev(r)).cpu().numpy()
    e = relmax(z, ref.vcycle(r))
    print(f"lattice mixed cycle: max-norm {e:.2e}", flush=True)
    assert e <= 2.0 ** -9
    b0 = box.mass() * wl.manufactured_load(box.coords())
    b = b0 + 1e-3 * np.max(np.abs(b0)) * wl.uniform_noise(box.n, 0)
    u, info = s.solve(dev(b), rtol=1e-8, maxit=100)
    assert info.converged
    assert np.linalg.norm(b - box.apply(u.cpu().numpy())) <= 1.01e-8 * np.linalg.norm(b)
