"""CPU checks of the native library: exported symbols, and the host-side setup
(GLL data, geometric factors, diagonals, transfers, coarse operators, FD
hierarchy, error codes) compared with the oracle. No GPU calls."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workload as wl
from oracle import fd2d
from oracle.gll import gll_nodes_weights, derivative_matrix, interpolation_matrix
from oracle.sem import SemBox
from paper_2210_03179_amd import _lib as L
from paper_2210_03179_amd.solver import SemSolver, FdSolver, beta_table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    header = open(os.path.join(ROOT, "include", "semcheb.h")).read()
    declared = set(re.findall(r"\b(sem_[A-Za-z0-9_]+)\s*\(", header))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(L.EXPORTS)


def test_beta_table_matches_golden():
    rows = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "beta_coef.txt")):
        if line.strip() and not line.startswith("#"):
            k, i, v = line.split()
            rows.setdefault(int(k), []).append(float(v))
    for k, vals in rows.items():
        assert beta_table(k) == vals
    lib = L.load()
    assert lib.sem_beta_table(33, (C.c_double * 33)()) == L.SEM_EINVAL
    assert lib.sem_beta_table(0, (C.c_double * 1)()) == L.SEM_EINVAL


def test_computed_beta_rows_match_the_oracle():
    """Orders 17..32: the library's own minimax solver (maxima located by bisection, Newton
    on the extreme values) and the oracle's (maxima as unknowns of one Newton system) agree."""
    from oracle import chebyshev as cheb
    ref = cheb.minimax_betas(32)
    for k in range(17, 33):
        assert np.max(np.abs(np.array(beta_table(k)) - np.array(ref[k]))) < 1e-12, k


@pytest.fixture(scope="module")
def host_ctx():
    V = wl.deformed_box((3, 2, 2), 0.05)
    s = SemSolver(V, N=5, device=-1, lambda_max=[2.0, 2.0])
    return V, s


def test_host_levels_and_gll(host_ctx):
    V, s = host_ctx
    assert s.num_levels == 3
    assert [s.level_info(j)[0] for j in range(3)] == [5, 2, 1]
    for j, N in enumerate([5, 2, 1]):
        x, w = gll_nodes_weights(N)
        assert np.max(np.abs(s.host_array("gll_nodes", j) - x)) < 1e-15
        assert np.max(np.abs(s.host_array("gll_weights", j) - w)) < 1e-15
        assert np.max(np.abs(s.host_array("deriv", j) - derivative_matrix(N).ravel())) < 1e-13
    assert np.max(np.abs(s.host_array("interp", 0) - interpolation_matrix(2, 5).ravel())) < 1e-15
    assert np.max(np.abs(s.host_array("interp", 1) - interpolation_matrix(1, 2).ravel())) < 1e-15


def test_host_geometry_matches_oracle(host_ctx):
    V, s = host_ctx
    for j, N in enumerate([5, 2, 1]):
        box = SemBox(V, N)
        G = s.host_array("factors", j).reshape(box.G.shape)
        assert np.max(np.abs(G - box.G)) < 1e-14 * np.max(np.abs(box.G))
        assert np.max(np.abs(s.host_array("diag", j) - box.diag())) < 1e-13 * np.max(box.diag())
        assert np.max(np.abs(s.host_array("mass", j) - box.mass())) < 1e-15
        assert np.max(np.abs(s.host_array("coords", j).reshape(-1, 3) - box.coords())) < 1e-15


def test_host_coarse_matrix_matches_oracle(host_ctx):
    V, s = host_ctx
    box = SemBox(V, 1)
    A = box.assemble().toarray()
    Ah = s.host_array("coarse_matrix").reshape(box.n, box.n)
    assert np.max(np.abs(Ah - A)) < 1e-14 * np.max(np.abs(A))


def test_host_lambda_passthrough(host_ctx):
    _, s = host_ctx
    assert s.lambda_max() == [2.0, 2.0]


def test_fd_host_hierarchy_matches_oracle():
    s = FdSolver(n=32, Lx=2.0, factor=2, coarsest_n=4, device=-1, lambda_max=[1, 1, 1])
    As, Ps, ns = fd2d.hierarchy_matrices(32, 2, 2.0, 1.0, coarsest_n=4)
    assert s.num_levels == len(As)
    for j, A in enumerate(As):
        M = s.host_array("matrix", j).reshape(A.shape)
        assert np.max(np.abs(M - A.toarray())) < 1e-12 * abs(A).max()
    assert np.max(np.abs(s.host_array("coarse_matrix").reshape(As[-1].shape) - As[-1].toarray())) < 1e-10


def test_error_codes():
    V = wl.deformed_box(3, 0.05)
    with pytest.raises(L.SemError) as e:
        SemSolver(V, N=5, smoother="cheb4opt", pre=33, device=-1)
    assert e.value.status == L.SEM_EINVAL
    with pytest.raises(L.SemError) as e:
        SemSolver(V, N=13, device=-1)
    assert e.value.status == L.SEM_EINVAL
    with pytest.raises(L.SemError) as e:
        SemSolver(V, N=5, orders=[5, 3], device=-1)
    assert e.value.status == L.SEM_EINVAL
    with pytest.raises(L.SemError) as e:
        SemSolver(wl.deformed_box((1, 2, 2), 0.05), N=3, device=-1)
    assert e.value.status == L.SEM_EINVAL
    with pytest.raises(L.SemError) as e:
        SemSolver(V, N=5, pre=0, post=0, device=-1)
    assert e.value.status == L.SEM_EINVAL
    # an inverted element: swap two vertices of the lattice
    bad = V.copy()
    bad[1, 1, 1], bad[1, 1, 2] = V[1, 1, 2].copy(), V[1, 1, 1].copy()
    with pytest.raises(L.SemError) as e:
        SemSolver(bad, N=3, device=-1)
    assert e.value.status == L.SEM_EMESH
    with pytest.raises(L.SemError) as e:
        FdSolver(n=64, factor=3, device=-1)
    assert e.value.status == L.SEM_EINVAL


def test_device_calls_on_host_context_fail_loudly(host_ctx):
    _, s = host_ctx
    lib = L.load()
    st = lib.sem_apply_A(s._ctx, C.c_void_p(8), C.c_void_p(8), None)
    assert st == L.SEM_ENODEV


def test_schwarz_option_validation():
    import workload as wl
    from paper_2210_03179_amd import _lib as L
    from paper_2210_03179_amd.solver import SemSolver
    V = wl.deformed_box(2, 0.05)
    with pytest.raises(L.SemError) as ex:  # order 2 on a smoothed level
        SemSolver(V, N=5, orders=[5, 2, 1], schwarz="asm", device=-1, lambda_max=[1.0, 1.0])
    assert ex.value.status == L.SEM_EINVAL
    with pytest.raises(L.SemError) as ex:  # default schedule 4 -> 2 -> 1
        SemSolver(V, N=4, schwarz="ras", device=-1, lambda_max=[1.0, 1.0])
    assert ex.value.status == L.SEM_EINVAL
    with pytest.raises(L.SemError) as ex:  # unknown smoother code
        SemSolver(V, N=5, schwarz=7, device=-1, lambda_max=[1.0, 1.0])
    assert ex.value.status == L.SEM_EINVAL


def test_fd_sparse_host_arrays_match_oracle():
    s = FdSolver(n=32, Lx=4.0, factor=2, coarsest_n=2, device=-1, lambda_max=[1, 1, 1, 1])
    As, Ps, _ = fd2d.hierarchy_matrices(32, 2, 4.0, 1.0, coarsest_n=2)
    for j, A in enumerate(As):
        rp, col, val = s.sparse("csr", j)
        D = np.zeros(A.shape)
        for r in range(A.shape[0]):
            D[r, col[rp[r]:rp[r + 1]]] = val[rp[r]:rp[r + 1]]
        assert np.max(np.abs(D - A.toarray())) < 1e-12 * abs(A).max()
    for j, P in enumerate(Ps):
        rp, col, val = s.sparse("interp", j)
        D = np.zeros(P.shape)
        for r in range(P.shape[0]):
            D[r, col[rp[r]:rp[r + 1]]] = val[rp[r]:rp[r + 1]]
        assert np.max(np.abs(D - P.toarray())) < 1e-15
    with pytest.raises(L.SemError):
        s.host_array("interp_val", len(As) - 1)   # no interpolation below the coarsest level


def test_set_smoothing_validation_and_mg_option():
    s = FdSolver(n=16, factor=2, coarsest_n=2, device=-1, lambda_max=[1, 1, 1], krylov="mg")
    s.set_smoothing("cheb1opt", 3, 3)
    s.set_smoothing("cheb4opt", 20, 0)   # beyond the printed table: computed coefficients
    for args in (("cheb4opt", 33, 0), ("cheb4", 0, 0), (9, 1, 1)):
        with pytest.raises(L.SemError) as ex:
            s.set_smoothing(*args)
        assert ex.value.status == L.SEM_EINVAL
    with pytest.raises(L.SemError):
        FdSolver(n=16, factor=2, coarsest_n=2, device=-1, lambda_max=[1, 1, 1], krylov=7)


def test_geometry_option_validation():
    V = wl.deformed_box(2, 0.05)
    s = SemSolver(V, N=4, geometry="trilinear", device=-1, lambda_max=[1.0, 1.0])
    assert s.num_levels == 3
    with pytest.raises(L.SemError) as ex:
        SemSolver(V, N=4, geometry=5, device=-1, lambda_max=[1.0, 1.0])
    assert ex.value.status == L.SEM_EINVAL
    o = L.make_options(device=-1)
    assert o.geometry == 0 and o.coarse_storage == 0  # stored factors, FP64 coarse factors by default
    with pytest.raises(L.SemError) as ex:   # FP32 coarse factors belong to a mixed cycle
        SemSolver(V, N=4, coarse_storage="mixed", device=-1, lambda_max=[1.0, 1.0])
    assert ex.value.status == L.SEM_EINVAL
    SemSolver(V, N=4, precision="mixed", coarse_storage="mixed", device=-1, lambda_max=[1.0, 1.0])


def test_batched_setup_rejects_orders_beyond_the_coefficient_table():
    """The batched descriptors hold 16 Chebyshev steps per smoothing: longer smoothings
    are refused at setup (before any device work), for the pre- and the post-smoother."""
    lib = L.load()
    V = np.ascontiguousarray(wl.deformed_box(2, 0.05))
    meshes = (L.SemBoxMesh * 1)(L.SemBoxMesh(2, 2, 2, V.ctypes.data_as(C.POINTER(C.c_double))))
    orders = (C.c_int32 * 1)(5)
    for pre, post in ((20, 0), (17, 0), (4, 17)):
        opt = L.make_options(5, "cheb4", pre, post, "mixed", "fcg", device=-1)
        ctx = C.c_void_p()
        assert lib.sem_setup_batched(1, meshes, orders, C.byref(opt), None, C.byref(ctx)) == L.SEM_EINVAL
        assert b"16" in lib.sem_global_error()
    opt = L.make_options(5, "cheb4", 16, 0, "mixed", "fcg", device=-1)
    ctx = C.c_void_p()
    assert lib.sem_setup_batched(1, meshes, orders, C.byref(opt), None, C.byref(ctx)) == L.SEM_ENODEV


def test_lattice_multigrid_host_hierarchy_matches_oracle():
    """coarse="lattice": the levels below order 1 (vertex lattice halved per direction) and
    the Galerkin operator of the last one, built in C++, against the oracle's construction."""
    from oracle import chebyshev as cheb, mg
    V = wl.deformed_box((8, 4, 6), 0.05)
    ref = mg.sem_hierarchy(V, 3, cheb.CHEB4, 2, 2, lmax=[2.0] * 3, coarse="lattice", dense_max=8)
    s = SemSolver(V, N=3, smoother="cheb4", pre=2, post=2, device=-1, lambda_max=[2.0] * 3,
                  coarse="lattice", dense_max=8)
    assert s.num_levels == len(ref.levels) == 3
    assert [s.level_info(j)[1] for j in range(3)] == [lev.n for lev in ref.levels]
    assert [s.level_info(j)[0] for j in range(3)] == [3, 1, 1]
    Ac = ref.extra["lattice_As"][-1].toarray()
    Ah = s.host_array("coarse_matrix").reshape(Ac.shape)
    assert np.max(np.abs(Ah - Ac)) < 1e-14 * np.max(np.abs(Ac))
    # a level that fits dense_max keeps the exact order-1 solve; an odd element count stops
    # the halving
    s2 = SemSolver(V, N=3, device=-1, lambda_max=[2.0], coarse="lattice")
    assert s2.num_levels == 2
    s3 = SemSolver(wl.deformed_box((8, 5, 6), 0.05), N=3, device=-1, lambda_max=[2.0], coarse="lattice",
                   dense_max=8)
    assert s3.num_levels == 2
    with pytest.raises(L.SemError) as ex:
        SemSolver(V, N=3, device=-1, lambda_max=[2.0] * 3, coarse="lattice", schwarz="ras")
    assert ex.value.status == L.SEM_EINVAL


@pytest.mark.parametrize("faces", [None, ("x0",), ("x0", "y1", "z0")])
def test_mesh_host_setup_matches_oracle(faces):
    """sem_setup on an unstructured mesh (a box with shuffled, rotated elements and renumbered
    vertices): the library numbers nodes by the vertices of their edge or face, the oracle by
    position; both number the unknowns by first appearance, so the host arrays must agree
    entry by entry: coordinates, diagonal, mass, factors and the order-1 matrix."""
    from oracle.mesh import SemMesh as OracleMesh
    from paper_2210_03179_amd.solver import MeshSolver
    V = wl.deformed_box((3, 2, 2), 0.06)
    xyz, ev = wl.box_as_mesh(V)
    xyz, ev, _ = wl.shuffled_mesh(xyz, ev, 7)
    flags = None if faces is None else wl.face_flags(xyz, faces)
    s = MeshSolver(xyz, ev, N=4, vertex_dirichlet=flags, device=-1, lambda_max=[2.0, 2.0])
    assert s.num_levels == 3
    for j, N in enumerate([4, 2, 1]):
        ref = OracleMesh(xyz, ev, N, flags)
        assert s.level_info(j)[1] == ref.n
        assert np.max(np.abs(s.host_array("coords", j).reshape(-1, 3) - ref.coords())) < 1e-15
        assert np.max(np.abs(s.host_array("diag", j) - ref.diag())) < 1e-13 * np.max(ref.diag())
        assert np.max(np.abs(s.host_array("mass", j) - ref.mass())) < 1e-15
        G = s.host_array("factors", j).reshape(ref.G.shape)
        assert np.max(np.abs(G - ref.G)) < 1e-14 * np.max(np.abs(ref.G))
    A1 = OracleMesh(xyz, ev, 1, flags).assemble().toarray()
    Ah = s.host_array("coarse_matrix").reshape(A1.shape)
    assert np.max(np.abs(Ah - A1)) < 1e-14 * np.max(np.abs(A1))


def test_mesh_setup_validation():
    from paper_2210_03179_amd.solver import MeshSolver
    xyz, ev = wl.box_as_mesh(wl.deformed_box(2, 0.05))
    for bad_ev, flags in ((np.where(ev == 5, 999, ev), None),             # vertex index out of range
                          (ev, np.zeros(len(xyz), np.uint8))):           # no Dirichlet face
        with pytest.raises(L.SemError) as ex:
            MeshSolver(xyz, bad_ev, N=2, vertex_dirichlet=flags, device=-1, lambda_max=[2.0])
        assert ex.value.status == L.SEM_EINVAL
    inverted = ev.copy()
    inverted[0, [0, 1]] = inverted[0, [1, 0]]                           # mirrored element
    with pytest.raises(L.SemError) as ex:
        MeshSolver(xyz, inverted, N=2, device=-1, lambda_max=[2.0])
    assert ex.value.status == L.SEM_EMESH
