"""The host side of the library (set-up, validation, mesh numbering, coarse factorisation,
beta solver, host arrays) under AddressSanitizer and UndefinedBehaviorSanitizer: a build with
both sanitizers on the host pass runs host-only contexts (device = -1) of every kind in a
child process with the sanitizer runtime preloaded; any report fails the test. No GPU."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.modules["torch"] = None          # host-only: the binding must not need torch here
sys.path.insert(0, ROOT)
import numpy as np
import workload as wl
from paper_2210_03179_amd import _lib as L
from paper_2210_03179_amd.solver import SemSolver, MeshSolver, FdSolver, beta_table
V = wl.deformed_box((4, 4, 4), 0.05)
for kw in ({}, {"coarse": "lattice", "dense_max": 8}, {"geometry": "trilinear"}, {"schwarz": "ras", "orders": [5, 3, 1]},
           {"precision": "mixed", "coarse_storage": "mixed"}):
    s = SemSolver(V, N=5, device=-1, lambda_max=[2.0] * 4, **kw)
    for j in range(s.num_levels):
        s.level_info(j)
    s.host_array("diag", 0); s.host_array("coarse_matrix")
    s.close()
s = SemSolver(wl.deformed_box((3, 2, 5), 0.05), N=7, device=-1, lambda_max=[2.0] * 2, coarse_planes=1)
s.close()
xyz, ev = wl.box_as_mesh(V)
xyz, ev, _ = wl.shuffled_mesh(xyz, ev, 1)
m = MeshSolver(xyz, ev, N=4, vertex_dirichlet=wl.face_flags(xyz, ("x0", "z1")), device=-1, lambda_max=[2.0] * 2)
m.host_array("coords", 0); m.host_array("coarse_matrix")
m.close()
f = FdSolver(n=64, factor=2, coarsest_n=2, device=-1, lambda_max=[1.0] * 5)
f.sparse("csr", 1); f.close()
for k in range(1, 33):
    assert len(beta_table(k)) == k
for bad in (dict(N=13), dict(pre=0, post=0), dict(smoother="cheb4opt", pre=40)):
    try:
        SemSolver(V, device=-1, **bad)
    except L.SemError:
        pass
    else:
        raise SystemExit("accepted " + str(bad))
print("SANITIZED RUN OK")
"""


def _runtime(name):
    hits = glob.glob(f"/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.{name}-x86_64.so")
    return hits[0] if hits else None


@pytest.mark.slow
def test_host_code_under_sanitizers(tmp_path):
    asan, ubsan = _runtime("asan"), _runtime("ubsan_standalone")
    if asan is None:
        pytest.skip("no clang AddressSanitizer runtime in this image")
    from paper_2210_03179_amd.build import build_host_sanitized
    lib = build_host_sanitized(str(tmp_path))
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms   # the host code is instrumented
    env = dict(os.environ, SEMCHEB_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", SCRIPT.replace("ROOT", repr(ROOT))], env=env, capture_output=True,
                       text=True, timeout=900)
    report = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0, report
    assert "SANITIZED RUN OK" in r.stdout, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
