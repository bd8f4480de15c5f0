"""sem_apply_A_noalloc, the allocation-free form of sem_apply_A (its element-local
products live in the library's static device array), through the C ABI: bitwise equal to
sem_apply_A on two calls in a row, the second on a smaller problem (the array keeps the
first call's contents), and a clear refusal above the array's size."""
import ctypes as C

import numpy as np
import pytest
import torch

import workload as wl
from paper_2210_03179_amd import _lib as L
from paper_2210_03179_amd.solver import FdSolver, SemSolver

pytestmark = pytest.mark.gpu


def _noalloc(s, u, w):
    lib = L.load()
    return lib.sem_apply_A_noalloc(s._ctx, C.c_void_p(u.data_ptr()), C.c_void_p(w.data_ptr()),
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_apply_A_noalloc_matches_apply_A():
    # the larger case first: the second, smaller call runs on what the first left in the array
    for m, N, seed in [((10, 9, 8), 7, 3), ((2, 3, 2), 4, 4)]:
        print(f"noalloc apply m={m} N={N}", flush=True)
        V = wl.deformed_box(m, 0.05)
        s = SemSolver(V, N=N, lambda_max=[2.0, 2.0])
        u = torch.from_numpy(wl.uniform_noise(s.n, seed)).cuda()
        ref = s.apply_A(u)
        w = torch.full_like(u, float("nan"))
        assert _noalloc(s, u, w) == L.SEM_OK
        torch.cuda.synchronize()
        assert torch.equal(w, ref)
        # a second call into the same output, and counts like sem_apply_A
        s.reset_counts()
        assert _noalloc(s, u, w) == L.SEM_OK
        torch.cuda.synchronize()
        assert torch.equal(w, ref) and s.apply_counts()[0] == 1
        s.close()


def test_apply_A_noalloc_refuses_above_its_scratch():
    V = wl.deformed_box(21, 0.05)             # 21^3 (N+1)^3 = 4,741,632 > 2^22 element-local nodes
    s = SemSolver(V, N=7, lambda_max=[2.0, 2.0])
    assert s.n_local > 1 << 22
    u = torch.zeros(s.n, dtype=torch.float64, device="cuda")
    w = torch.zeros_like(u)
    assert _noalloc(s, u, w) == L.SEM_EINVAL
    assert b"scratch maximum" in L.load().sem_last_error(s._ctx)
    fd = FdSolver(n=16, factor=2, coarsest_n=2, lambda_max=[1, 1, 1])
    v = torch.zeros(fd.n, dtype=torch.float64, device="cuda")
    assert _noalloc(fd, v, torch.zeros_like(v)) == L.SEM_EINVAL   # FD contexts have no scratch use
