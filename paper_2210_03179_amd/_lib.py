"""ctypes binding of libsemcheb.so (the C ABI declared in include/semcheb.h).

Only argument marshalling lives here; every step of the solve runs in the HIP
kernels of the library. Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# SEMCHEB_LIB selects another build of the same library (the host-sanitizer test uses it)
LIB_PATH = os.environ.get("SEMCHEB_LIB", os.path.join(_HERE, "libsemcheb.so"))

SEM_OK, SEM_EINVAL, SEM_ENOMEM, SEM_EHIP, SEM_EMESH = 0, -1, -2, -3, -4
SEM_ENOTCONV, SEM_EBREAKDOWN, SEM_ENAN, SEM_ENODEV = -5, -6, -7, -8
STATUS_NAMES = {0: "SEM_OK", -1: "SEM_EINVAL", -2: "SEM_ENOMEM", -3: "SEM_EHIP", -4: "SEM_EMESH",
                -5: "SEM_ENOTCONV", -6: "SEM_EBREAKDOWN", -7: "SEM_ENAN", -8: "SEM_ENODEV"}
SMOOTHERS = {"cheb1": 1, "cheb1opt": 2, "cheb4": 4, "cheb4opt": 5}
PRECISIONS = {"fp64": 0, "mixed": 1}
KRYLOV = {"pcg": 0, "fcg": 1, "gmres": 2, "mg": 3}
SCHWARZ = {None: 0, "jacobi": 0, "asm": 1, "ras": 2}
GEOMETRY = {"stored": 0, "trilinear": 1}
COARSE = {"exact": 0, "lattice": 1}
MAX_LEVELS = 8

# exported entry points, as declared in include/semcheb.h
EXPORTS = (
    "sem_options_default", "sem_setup_box", "sem_setup", "sem_setup_fd2d", "sem_sizes", "sem_level_info",
    "sem_apply_A", "sem_apply_A_noalloc", "sem_apply_local", "sem_vcycle", "sem_solve", "sem_coords", "sem_mass_apply", "sem_get_factors",
    "sem_set_factors", "sem_adjoint_contract", "sem_apply_counts", "sem_reset_counts",
    "sem_host_array", "sem_set_smoothing", "sem_beta_table", "sem_destroy", "sem_last_error", "sem_global_error",
    "sem_setup_batched", "sem_batch_info", "sem_solve_batched",
)


class SemOptions(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("num_levels", C.c_int32), ("orders", C.c_int32 * MAX_LEVELS),
        ("smoother", C.c_int32), ("pre_order", C.c_int32), ("post_order", C.c_int32),
        ("precision", C.c_int32), ("krylov", C.c_int32), ("num_lambda_max", C.c_int32),
        ("lambda_max", C.c_double * MAX_LEVELS), ("lambda_scale", C.c_double), ("device", C.c_int32),
        ("coarse_planes", C.c_int32), ("gmres_restart", C.c_int32), ("schwarz", C.c_int32),
        ("geometry", C.c_int32), ("coarse_storage", C.c_int32), ("coarse_solver", C.c_int32),
        ("coarse_dense_max", C.c_int32),
    ]


class SemBoxMesh(C.Structure):
    _fields_ = [("nex", C.c_int32), ("ney", C.c_int32), ("nez", C.c_int32),
                ("vertex_xyz", C.POINTER(C.c_double))]


class SemMesh(C.Structure):
    _fields_ = [("num_elements", C.c_int32), ("num_vertices", C.c_int32),
                ("vertex_xyz", C.POINTER(C.c_double)), ("elem_vertices", C.POINTER(C.c_int32)),
                ("vertex_dirichlet", C.POINTER(C.c_uint8))]


class SemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2210_03179_amd.build")
    try:
        # torch ships its own HIP runtime; loading it first makes the library bind to that same
        # runtime instance (one runtime per process), whichever module the caller imported first
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "sem_options_default": (None, [P(SemOptions)]),
        "sem_setup_box": (i32, [P(SemBoxMesh), P(SemOptions), vp, P(vp)]),
        "sem_setup": (i32, [P(SemMesh), P(SemOptions), vp, P(vp)]),
        "sem_setup_fd2d": (i32, [i32, dbl, dbl, i32, i32, P(SemOptions), vp, P(vp)]),
        "sem_sizes": (i32, [vp, P(i64), P(i32), P(i64)]),
        "sem_level_info": (i32, [vp, i32, P(i32), P(i64), P(dbl)]),
        "sem_apply_A": (i32, [vp, vp, vp, vp]),
        "sem_apply_A_noalloc": (i32, [vp, vp, vp, vp]),
        "sem_apply_local": (i32, [vp, i32, vp, vp, vp]),
        "sem_vcycle": (i32, [vp, vp, vp, vp]),
        "sem_solve": (i32, [vp, vp, vp, dbl, i32, P(i32), P(dbl), P(dbl), vp]),
        "sem_coords": (i32, [vp, vp, vp]),
        "sem_mass_apply": (i32, [vp, vp, vp, vp]),
        "sem_get_factors": (i32, [vp, vp, vp]),
        "sem_set_factors": (i32, [vp, vp, vp]),
        "sem_adjoint_contract": (i32, [vp, vp, vp, vp, vp, vp]),
        "sem_apply_counts": (i32, [vp, P(i64), i32]),
        "sem_reset_counts": (i32, [vp]),
        "sem_host_array": (i32, [vp, C.c_char_p, i32, P(dbl), i64, P(i64)]),
        "sem_set_smoothing": (i32, [vp, i32, i32, i32]),
        "sem_beta_table": (i32, [i32, P(dbl)]),
        "sem_setup_batched": (i32, [i32, P(SemBoxMesh), P(i32), P(SemOptions), vp, P(vp)]),
        "sem_batch_info": (i32, [vp, P(i32), P(i64)]),
        "sem_solve_batched": (i32, [vp, vp, vp, dbl, i32, P(i32), P(dbl), vp]),
        "sem_destroy": (i32, [vp]),
        "sem_last_error": (C.c_char_p, [vp]),
        "sem_global_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, ctx=None) -> int:
    """Raise SemError for a failing status (SEM_ENOTCONV is returned to the caller)."""
    if status == SEM_OK:
        return status
    lib = load()
    msg = (lib.sem_last_error(ctx) if ctx else lib.sem_global_error()) or b""
    raise SemError(status, msg.decode())


def make_options(N=7, smoother="cheb4opt", pre=4, post=0, precision="fp64", krylov="fcg",
                 orders=None, lambda_max=None, lambda_scale=1.0, device=0, coarse_planes=0,
                 restart=30, schwarz=None, geometry="stored", coarse_storage="fp64", coarse="exact",
                 dense_max=0) -> SemOptions:
    lib = load()
    o = SemOptions()
    lib.sem_options_default(C.byref(o))
    o.N = N
    if orders is not None:
        o.num_levels = len(orders)
        for j, v in enumerate(orders):
            o.orders[j] = int(v)
    o.smoother = SMOOTHERS[smoother] if isinstance(smoother, str) else int(smoother)
    o.pre_order, o.post_order = int(pre), int(post)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.krylov = KRYLOV[krylov] if isinstance(krylov, str) else int(krylov)
    if lambda_max is not None:
        o.num_lambda_max = len(lambda_max)
        for j, v in enumerate(lambda_max):
            o.lambda_max[j] = float(v)
    o.lambda_scale = float(lambda_scale)
    o.device = int(device)
    o.coarse_planes = int(coarse_planes)
    o.gmres_restart = int(restart)
    o.schwarz = SCHWARZ[schwarz] if (schwarz is None or isinstance(schwarz, str)) else int(schwarz)
    o.geometry = GEOMETRY[geometry] if isinstance(geometry, str) else int(geometry)
    o.coarse_storage = PRECISIONS[coarse_storage] if isinstance(coarse_storage, str) else int(coarse_storage)
    o.coarse_solver = COARSE[coarse] if isinstance(coarse, str) else int(coarse)
    o.coarse_dense_max = int(dense_max)
    return o
