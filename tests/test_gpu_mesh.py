"""Unstructured conforming hexahedral meshes (sem_setup) on the GPU against the oracle's
unstructured discretisation (oracle/mesh.py), through the C ABI.

Meshes: boxes given as element lists with the elements shuffled, every element's reference
frame turned by a random rotation of the cube and the vertices renumbered; Dirichlet data
on the whole boundary or on flagged faces only. Tolerances as for the box path: operator
1e-14 (N+1)^2 relative (max norm), FP64 cycles 1e-12, solves with identical iteration counts,
residual histories within 1e-12 ||b|| and solutions within 1e-12; the mixed cycle within one
BF16 unit roundoff (2^-9) node by node, its solve to a true 1e-8."""
import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

import rounding
import workload as wl
from oracle import chebyshev as cheb, krylov, mg
from oracle.mesh import SemMesh
from paper_2210_03179_amd.solver import MeshSolver, SemSolver

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _mesh(m, seed, faces=None, amp=0.06):
    xyz, ev = wl.box_as_mesh(wl.deformed_box(m, amp))
    xyz, ev, _ = wl.shuffled_mesh(xyz, ev, seed)
    return xyz, ev, (None if faces is None else wl.face_flags(xyz, faces))


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 9, 12])
@pytest.mark.parametrize("faces", [None, ("x0", "z1")])
def test_mesh_apply_A_parity(N, faces):
    print(f"mesh apply_A N={N} faces={faces}", flush=True)
    xyz, ev, flags = _mesh((3, 2, 2), 3, faces)
    ref = SemMesh(xyz, ev, N, flags)
    s = MeshSolver(xyz, ev, N=N, vertex_dirichlet=flags, lambda_max=[1.0] * 8, orders=[N, 1] if N > 1 else [1])
    assert s.n == ref.n
    u = wl.uniform_noise(ref.n, 11)
    assert relmax(host(s.apply_A(dev(u))), ref.apply(u)) < 1e-14 * (N + 1) ** 2
    f = wl.uniform_noise(ref.n, 12)
    # the two sides' masses differ by the rounding of the differentiated coordinates: the
    # tolerance is 1e-13 or their first-order bound where that is smaller (tests/rounding.py)
    assert relmax(host(s.mass_apply(dev(f))), ref.mass() * f) < min(1e-13, rounding.mass_bound(ref))
    assert np.max(np.abs(host(s.coords()) - ref.coords())) < 1e-15


@pytest.fixture(scope="module")
def mesh_case():
    xyz, ev, flags = _mesh((4, 3, 3), 5, ("x0", "y0", "y1", "z1"))
    h = mg.sem_hierarchy((xyz, ev, flags), 5, cheb.CHEB4_OPT, 4, 0)
    return xyz, ev, flags, [lev.lmax for lev in h.levels[:-1]]


@pytest.mark.parametrize("kind,pre,post", [("cheb4opt", 4, 0), ("cheb4", 2, 2), ("cheb1", 3, 3), ("cheb1opt", 2, 0)])
def test_mesh_vcycle_parity(mesh_case, kind, pre, post):
    xyz, ev, flags, lmax = mesh_case
    ref = mg.sem_hierarchy((xyz, ev, flags), 5, kind, pre, post, lmax=lmax)
    s = MeshSolver(xyz, ev, N=5, vertex_dirichlet=flags, smoother=kind, pre=pre, post=post, lambda_max=lmax)
    r = wl.uniform_noise(ref.levels[0].n, 21)
    ref.reset_counters()
    zo = ref.vcycle(r)
    s.reset_counts()
    z = host(s.vcycle(dev(r)))
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)
    assert relmax(z, zo) <= 1e-12
    assert s.apply_counts() == [lev.applies for lev in ref.levels]


@pytest.mark.parametrize("kry,kind,pre,post", [("fcg", "cheb4opt", 4, 0), ("pcg", "cheb4", 2, 2)])
def test_mesh_solve_parity(mesh_case, kry, kind, pre, post):
    xyz, ev, flags, lmax = mesh_case
    ref = mg.sem_hierarchy((xyz, ev, flags), 5, kind, pre, post, lmax=lmax)
    box = ref.extra["boxes"][0]
    b = box.mass() * wl.manufactured_load(box.coords()) + 1e-2 * wl.uniform_noise(box.n, 1)
    res = krylov.pcg(box.apply, b, ref.vcycle, 1e-8, 200, flexible=(kry == "fcg"))
    s = MeshSolver(xyz, ev, N=5, vertex_dirichlet=flags, smoother=kind, pre=pre, post=post, krylov=kry,
                   lambda_max=lmax)
    u, info = s.solve(dev(b), rtol=1e-8, maxit=200)
    print(f"mesh {kry}: {info.iterations} iterations (oracle {res.iterations})", flush=True)
    assert info.converged and res.converged and info.iterations == res.iterations
    assert np.max(np.abs(info.history - np.array(res.history))) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(host(u) - res.x) <= 1e-12 * np.linalg.norm(res.x)


def test_mesh_mixed_precision(mesh_case):
    xyz, ev, flags, lmax = mesh_case
    ref = mg.sem_hierarchy((xyz, ev, flags), 5, cheb.CHEB4_OPT, 4, 0, lmax=lmax)
    box = ref.extra["boxes"][0]
    s = MeshSolver(xyz, ev, N=5, vertex_dirichlet=flags, precision="mixed", lambda_max=lmax)
    r = wl.uniform_noise(ref.levels[0].n, 22)
    e = relmax(host(s.vcycle(dev(r))), ref.vcycle(r))
    print(f"mesh mixed cycle: max-norm {e:.2e}", flush=True)
    assert e <= 2.0 ** -9
    b = box.mass() * wl.manufactured_load(box.coords()) + 1e-2 * wl.uniform_noise(box.n, 1)
    u, info = s.solve(dev(b), rtol=1e-8, maxit=200)
    assert info.converged
    assert np.linalg.norm(b - box.apply(host(u))) <= 1.01e-8 * np.linalg.norm(b)


def test_mesh_and_box_paths_agree():
    """The same deformed box through sem_setup_box and through sem_setup (as a shuffled
    element list): after matching unknowns by position, equal solutions and iterations."""
    V = wl.deformed_box((4, 4, 3), 0.05)
    sb = SemSolver(V, N=5, lambda_max=[2.3, 2.1])
    xyz, ev = wl.box_as_mesh(V)
    xyz, ev, _ = wl.shuffled_mesh(xyz, ev, 9)
    sm = MeshSolver(xyz, ev, N=5, lambda_max=[2.3, 2.1])
    cb, cm = host(sb.coords()), host(sm.coords())
    d, idx = cKDTree(cb).query(cm)
    assert d.max() < 1e-12
    b = wl.uniform_noise(sb.n, 4)
    ub, ib = sb.solve(dev(b), rtol=1e-10)
    um, im = sm.solve(dev(b[idx]), rtol=1e-10)
    assert ib.iterations == im.iterations
    assert np.max(np.abs(host(um) - host(ub)[idx])) <= 1e-11 * np.max(np.abs(host(ub)))
