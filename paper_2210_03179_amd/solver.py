"""Python front end of libsemcheb: solver objects over torch device tensors.

The classes only marshal arguments (device pointers, the current torch stream)
to the C ABI; all arithmetic runs in the library's HIP kernels. Vectors are
contiguous float64 CUDA/HIP tensors of the documented lengths.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, numel=None, what="tensor") -> C.c_void_p:
    """Device pointer of a contiguous float64 tensor; with `numel`, the tensor must hold
    exactly that many elements (the library reads and writes the context's sizes)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{what}: expected a contiguous float64 device tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


@dataclass
class SolveInfo:
    status: int
    iterations: int
    relres: float
    history: np.ndarray = field(repr=False)

    @property
    def converged(self) -> bool:
        return self.status == L.SEM_OK

    def avg_rate(self) -> float:
        """rho = exp(log(||r_N|| / ||r_0||) / N) (average convergence rate)."""
        if self.iterations == 0 or self.history[0] == 0:
            return 0.0
        return float(np.exp(np.log(self.history[self.iterations] / self.history[0]) / self.iterations))


class _Base:
    def __init__(self):
        self._ctx = None
        self._lib = L.load()

    def close(self):
        if self._ctx:
            self._lib.sem_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self) -> int:
        n = C.c_int64()
        L.check(self._lib.sem_sizes(self._ctx, C.byref(n), None, None), self._ctx)
        return n.value

    @property
    def num_levels(self) -> int:
        nl = C.c_int32()
        L.check(self._lib.sem_sizes(self._ctx, None, C.byref(nl), None), self._ctx)
        return nl.value

    def level_info(self, j: int):
        o, n, lm = C.c_int32(), C.c_int64(), C.c_double()
        L.check(self._lib.sem_level_info(self._ctx, j, C.byref(o), C.byref(n), C.byref(lm)), self._ctx)
        return o.value, n.value, lm.value

    def lambda_max(self):
        return [self.level_info(j)[2] for j in range(self.num_levels - 1)]

    def host_array(self, what: str, level: int = 0) -> np.ndarray:
        need = C.c_int64()
        self._lib.sem_host_array(self._ctx, what.encode(), level, None, -1, C.byref(need))
        out = np.empty(max(need.value, 0))
        L.check(self._lib.sem_host_array(self._ctx, what.encode(), level,
                                         out.ctypes.data_as(C.POINTER(C.c_double)), out.size, None), self._ctx)
        return out

    def set_smoothing(self, smoother, pre: int, post: int):
        """Change the Chebyshev kind and the (m, n) orders; hierarchy and lambda_max are kept."""
        kind = L.SMOOTHERS[smoother] if isinstance(smoother, str) else int(smoother)
        L.check(self._lib.sem_set_smoothing(self._ctx, kind, int(pre), int(post)), self._ctx)

    def apply_counts(self):
        nl = self.num_levels
        buf = (C.c_int64 * nl)()
        L.check(self._lib.sem_apply_counts(self._ctx, buf, nl), self._ctx)
        return list(buf)

    def reset_counts(self):
        L.check(self._lib.sem_reset_counts(self._ctx), self._ctx)

    # ---- device entry points
    def apply_A(self, u, out=None):
        torch = _torch()
        n = self.n
        up = _ptr(u, n, "u")
        out = torch.empty_like(u) if out is None else out
        L.check(self._lib.sem_apply_A(self._ctx, up, _ptr(out, n, "out"), _stream()), self._ctx)
        return out

    def vcycle(self, r, out=None):
        torch = _torch()
        n = self.n
        rp = _ptr(r, n, "r")
        out = torch.empty_like(r) if out is None else out
        L.check(self._lib.sem_vcycle(self._ctx, rp, _ptr(out, n, "out"), _stream()), self._ctx)
        return out

    def solve(self, b, x0=None, rtol: float = 1e-8, maxit: int = 500, raise_on_fail: bool = False, out=None):
        """Returns (u, SolveInfo). u starts from x0 (zero when None). out: optional preallocated
        tensor like b that receives u (no allocation inside the call)."""
        torch = _torch()
        n = self.n
        _ptr(b, n, "b")
        if x0 is not None:
            _ptr(x0, n, "x0")
        if out is not None:
            _ptr(out, n, "out")
            u = out.zero_() if x0 is None else out.copy_(x0)
        else:
            u = torch.zeros_like(b) if x0 is None else x0.clone()
        its, rel = C.c_int32(), C.c_double()
        hist = np.zeros(maxit + 1)
        st = self._lib.sem_solve(self._ctx, _ptr(b, n, "b"), _ptr(u, n, "u"), float(rtol), int(maxit), C.byref(its),
                                 C.byref(rel), hist.ctypes.data_as(C.POINTER(C.c_double)), _stream())
        if st not in (L.SEM_OK, L.SEM_ENOTCONV) or (raise_on_fail and st != L.SEM_OK):
            L.check(st, self._ctx)
        return u, SolveInfo(st, its.value, rel.value, hist[: its.value + 1].copy())


class SemSolver(_Base):
    """Chebyshev-smoothed p-multigrid PCG for the SEM Poisson problem on a box mesh.

    verts: (nez+1, ney+1, nex+1, 3) float64 vertex coordinates (x fastest).
    schwarz: None (Jacobi), "asm" or "ras": the basic smoother inside the Chebyshev algorithms.
    krylov: "pcg", "fcg", "gmres" (GMRES(restart)) or "mg" (multigrid as the solver).
    geometry: "stored" (factors read from HBM) or "trilinear" (formed in the operator).
    coarse_storage: "fp64" or, with precision="mixed", "mixed" (the cycle reads FP32 copies of the
    coarse factor blocks).
    coarse: "exact" (exact order-1 solve) or "lattice" (the cycle continues on the vertex lattice
    with Galerkin levels down to dense_max unknowns, 0 = 4096; FP64 in every precision).
    """

    def __init__(self, verts, N=7, smoother="cheb4opt", pre=4, post=0, precision="fp64",
                 krylov="fcg", orders=None, lambda_max=None, lambda_scale=1.0, device=0,
                 coarse_planes=0, restart=30, schwarz=None, geometry="stored", coarse_storage="fp64",
                 coarse="exact", dense_max=0):
        super().__init__()
        verts = np.ascontiguousarray(np.asarray(verts, dtype=np.float64))
        if verts.ndim != 4 or verts.shape[3] != 3:
            raise ValueError("verts must have shape (nez+1, ney+1, nex+1, 3)")
        self.verts = verts
        mesh = L.SemBoxMesh(verts.shape[2] - 1, verts.shape[1] - 1, verts.shape[0] - 1,
                            verts.ctypes.data_as(C.POINTER(C.c_double)))
        opt = L.make_options(N, smoother, pre, post, precision, krylov, orders, lambda_max,
                             lambda_scale, device, coarse_planes, restart, schwarz, geometry, coarse_storage,
                             coarse, dense_max)
        ctx = C.c_void_p()
        stream = _stream() if device >= 0 else C.c_void_p(0)
        L.check(self._lib.sem_setup_box(C.byref(mesh), C.byref(opt), stream, C.byref(ctx)))
        self._ctx = ctx
        self.N = N
        self.E = (verts.shape[0] - 1) * (verts.shape[1] - 1) * (verts.shape[2] - 1)

    @property
    def n_local(self) -> int:
        nl = C.c_int64()
        L.check(self._lib.sem_sizes(self._ctx, None, None, C.byref(nl)), self._ctx)
        return nl.value

    def apply_local(self, u, out=None):
        """Element-local operator (E-vector output); float64 u -> FP64 path,
        float32 u -> FP32 arithmetic with BF16 factors (mixed contexts)."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.n_local, dtype=u.dtype, device=u.device)
        prec = 0 if u.dtype == torch.float64 else 1
        if u.dtype not in (torch.float64, torch.float32) or out.dtype != u.dtype or not u.is_cuda:
            raise TypeError("u and out must be float64 or float32 device tensors")
        if not (u.is_contiguous() and out.is_contiguous() and out.is_cuda):
            raise TypeError("u and out must be contiguous device tensors")
        if u.numel() != self.n or out.numel() != self.n_local:
            raise ValueError(f"apply_local: u needs {self.n} and out {self.n_local} elements")
        L.check(self._lib.sem_apply_local(self._ctx, prec, C.c_void_p(u.data_ptr()), C.c_void_p(out.data_ptr()),
                                          _stream()), self._ctx)
        return out

    def coords(self):
        torch = _torch()
        out = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        L.check(self._lib.sem_coords(self._ctx, _ptr(out, 3 * self.n, "xyz"), _stream()), self._ctx)
        return out

    def mass_apply(self, f, out=None):
        torch = _torch()
        n = self.n
        fp = _ptr(f, n, "f")
        out = torch.empty_like(f) if out is None else out
        L.check(self._lib.sem_mass_apply(self._ctx, fp, _ptr(out, n, "out"), _stream()), self._ctx)
        return out

    def factors(self):
        torch = _torch()
        out = torch.empty((self.E, 6, self.N + 1, self.N + 1, self.N + 1), dtype=torch.float64, device="cuda")
        L.check(self._lib.sem_get_factors(self._ctx, _ptr(out, self._factor_count(), "G"), _stream()), self._ctx)
        return out

    def _factor_count(self) -> int:
        return self.E * 6 * (self.N + 1) ** 3

    def set_factors(self, G):
        G = G.contiguous()
        L.check(self._lib.sem_set_factors(self._ctx, _ptr(G, self._factor_count(), "G"), _stream()), self._ctx)

    def adjoint_contract(self, lam, u, want_dG=True, want_df=True):
        torch = _torch()
        n = self.n
        lp = _ptr(lam, n, "lambda")
        upp = _ptr(u, n, "u") if u is not None else None
        dG = torch.empty((self.E, 6, self.N + 1, self.N + 1, self.N + 1), dtype=torch.float64,
                         device="cuda") if want_dG else None
        df = torch.empty_like(lam) if want_df else None
        L.check(self._lib.sem_adjoint_contract(self._ctx, lp, upp,
                                               _ptr(dG) if dG is not None else None,
                                               _ptr(df) if df is not None else None, _stream()), self._ctx)
        return dG, df


class MeshSolver(SemSolver):
    """The same solver on an unstructured conforming hexahedral mesh (sem_setup).

    vertex_xyz: (num_vertices, 3); elem_vertices: (E, 8) corner vertices per element in
    lexicographic reference order (corner ci + 2 cj + 4 ck at (2ci-1, 2cj-1, 2ck-1));
    vertex_dirichlet: (num_vertices,) flags, or None for a Dirichlet condition on the whole
    boundary. Unknowns are numbered by first appearance over the element-local nodes."""

    def __init__(self, vertex_xyz, elem_vertices, N=7, vertex_dirichlet=None, smoother="cheb4opt", pre=4, post=0,
                 precision="fp64", krylov="fcg", orders=None, lambda_max=None, lambda_scale=1.0, device=0,
                 restart=30):
        _Base.__init__(self)
        xyz = np.ascontiguousarray(np.asarray(vertex_xyz, dtype=np.float64))
        ev = np.ascontiguousarray(np.asarray(elem_vertices, dtype=np.int32))
        if xyz.ndim != 2 or xyz.shape[1] != 3 or ev.ndim != 2 or ev.shape[1] != 8:
            raise ValueError("vertex_xyz must be (num_vertices, 3) and elem_vertices (E, 8)")
        flags = None if vertex_dirichlet is None else np.ascontiguousarray(np.asarray(vertex_dirichlet, np.uint8))
        if flags is not None and flags.shape != (xyz.shape[0],):
            raise ValueError("vertex_dirichlet needs one flag per vertex")
        self._arrays = (xyz, ev, flags)
        mesh = L.SemMesh(ev.shape[0], xyz.shape[0], xyz.ctypes.data_as(C.POINTER(C.c_double)),
                         ev.ctypes.data_as(C.POINTER(C.c_int32)),
                         flags.ctypes.data_as(C.POINTER(C.c_uint8)) if flags is not None else None)
        opt = L.make_options(N, smoother, pre, post, precision, krylov, orders, lambda_max, lambda_scale, device,
                             0, restart)
        ctx = C.c_void_p()
        stream = _stream() if device >= 0 else C.c_void_p(0)
        L.check(self._lib.sem_setup(C.byref(mesh), C.byref(opt), stream, C.byref(ctx)))
        self._ctx = ctx
        self.N = N
        self.E = ev.shape[0]


class FdSolver(_Base):
    """2D finite-difference Poisson with Galerkin geometric multigrid (the paper's Sec. 3 problem).

    krylov: "pcg", "fcg", "gmres" (GMRES(restart)) or "mg" (multigrid as the solver).
    """

    def __init__(self, n=64, Lx=1.0, Ly=1.0, factor=2, coarsest_n=8, smoother="cheb4", pre=4, post=0,
                 krylov="fcg", lambda_max=None, lambda_scale=1.0, device=0, restart=30):
        super().__init__()
        opt = L.make_options(1, smoother, pre, post, "fp64", krylov, None, lambda_max, lambda_scale, device,
                             0, restart)
        ctx = C.c_void_p()
        stream = _stream() if device >= 0 else C.c_void_p(0)
        L.check(self._lib.sem_setup_fd2d(int(n), float(Lx), float(Ly), int(factor), int(coarsest_n),
                                         C.byref(opt), stream, C.byref(ctx)))
        self._ctx = ctx

    def sparse(self, what: str, level: int):
        """(rowptr, col, val) of A_j (what="csr") or of P_j, level j+1 -> j (what="interp")."""
        rp = self.host_array(what + "_rowptr", level).astype(np.int64)
        col = self.host_array(what + "_col", level).astype(np.int64)
        return rp, col, self.host_array(what + "_val", level)


class BatchedSolver(_Base):
    """Many independent SEM systems (own meshes and orders) solved together: every
    kernel launch of a solve covers all systems that have not converged.

    verts_list: list of (nez+1, ney+1, nex+1, 3) vertex arrays; orders: list of N.
    Vectors are concatenated over the systems (see `offsets`).
    """

    def __init__(self, verts_list, orders, smoother="cheb4opt", pre=4, post=0, krylov="fcg",
                 lambda_scale=1.0, device=0):
        super().__init__()
        nsys = len(verts_list)
        self._verts = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in verts_list]
        meshes = (L.SemBoxMesh * nsys)()
        for q, v in enumerate(self._verts):
            meshes[q] = L.SemBoxMesh(v.shape[2] - 1, v.shape[1] - 1, v.shape[0] - 1,
                                     v.ctypes.data_as(C.POINTER(C.c_double)))
        ords = (C.c_int32 * nsys)(*[int(o) for o in orders])
        opt = L.make_options(int(orders[0]), smoother, pre, post, "mixed", krylov, None, None,
                             lambda_scale, device)
        ctx = C.c_void_p()
        L.check(self._lib.sem_setup_batched(nsys, meshes, ords, C.byref(opt), _stream(), C.byref(ctx)))
        self._ctx = ctx
        self.nsys = nsys
        offs = (C.c_int64 * (nsys + 1))()
        L.check(self._lib.sem_batch_info(self._ctx, None, offs), self._ctx)
        self.offsets = list(offs)

    @property
    def n(self) -> int:
        return self.offsets[-1]

    def solve(self, b, rtol: float = 1e-8, maxit: int = 500):
        """Returns (u, status, iterations per system, relative residual per system)."""
        torch = _torch()
        bp = _ptr(b, self.n, "b")
        u = torch.empty_like(b)
        its = (C.c_int32 * self.nsys)()
        rel = (C.c_double * self.nsys)()
        st = self._lib.sem_solve_batched(self._ctx, bp, _ptr(u, self.n, "u"), float(rtol), int(maxit), its, rel,
                                         _stream())
        if st not in (L.SEM_OK, L.SEM_ENOTCONV):
            L.check(st, self._ctx)
        return u, st, list(its), list(rel)


def beta_table(k: int) -> list:
    lib = L.load()
    out = (C.c_double * k)()
    L.check(lib.sem_beta_table(k, out))
    return list(out)
