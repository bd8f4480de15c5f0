"""Writes tests/golden/cfg3_fcg_fp64.txt and tests/golden/cfg3_fcg_fp64_lattice.txt: the
oracle's FP64 flexible-CG solve of the 32^3-element, order-7 box (11,089,567 unknowns;
p-multigrid 7/3/1, optimised 4th-kind Chebyshev-Jacobi (4,0) one-sided cycle, relative
residual 1e-8, x0 = 0), with the exact order-1 solve and with the lattice multigrid below
order 1 (one smoothed lattice level of 29,791 unknowns, dense 3,375-unknown last level).

lambda_max of every smoothed level is the oracle's Lanczos estimate, run to a relative
change below 1e-10 (the accuracy the library's own estimator stops at). The script calls
only oracle/ and workload/ (seeded inputs) and runs on the CPU for about half an hour:
    python tests/golden/make_cfg3_golden.py

Recorded per file: lambda_max per level, ||b||, the iteration count, the residual norm
history, ||x||_2, ||x||_inf, and x at 64 seeded sample indices.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workload as wl  # noqa: E402
from oracle import chebyshev as cheb, krylov, mg  # noqa: E402
from oracle.lanczos import lambda_max_SA  # noqa: E402
from oracle.sem import SemBox  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
M, N = 32, 7


def sample_indices(n: int) -> np.ndarray:
    return np.sort(np.random.Generator(np.random.PCG64(314)).choice(n, 64, replace=False))


def write(path, title, box, lmax, b, res):
    idx = sample_indices(box.n)
    with open(path, "w") as f:
        f.write(f"# Oracle FP64 flexible-CG solve, {title}: 32^3 deformed box (amplitude 0.05), N = 7,\n")
        f.write("# schedule 7/3/1, opt. 4th-kind Chebyshev-Jacobi (4,0) one-sided cycle,\n")
        f.write("# b = B f (f = 3 pi^2 sin sin sin) + 1e-3 max|B f| U[-1,1] (seed 0), tol 1e-8, x0 = 0.\n")
        f.write("# Written by tests/golden/make_cfg3_golden.py (oracle only).\n")
        f.write(f"n {box.n}\n")
        for j, v in enumerate(lmax):
            f.write(f"lambda_max {j} {v!r}\n")
        f.write(f"bnorm {float(np.linalg.norm(b))!r}\n")
        f.write(f"iterations {res.iterations}\n")
        for k, v in enumerate(res.history):
            f.write(f"history {k} {float(v)!r}\n")
        f.write(f"xnorm2 {float(np.linalg.norm(res.x))!r}\n")
        f.write(f"xnorminf {float(np.max(np.abs(res.x)))!r}\n")
        for i in idx:
            f.write(f"x {int(i)} {float(res.x[i])!r}\n")
    print("wrote", path, flush=True)


def main():
    t0 = time.time()
    V = wl.deformed_box(M, 0.05)
    lmax = []
    for order in (N, N // 2):
        bx = SemBox(V, order)
        lmax.append(lambda_max_SA(bx.apply, 1.0 / bx.diag(), bx.n, tol=1e-10, maxit=300))
        print(f"lambda_max order {order}: {lmax[-1]!r} ({time.time() - t0:.0f} s)", flush=True)
        del bx
    h = mg.sem_hierarchy(V, N, cheb.CHEB4_OPT, 4, 0, lmax=lmax)
    box = h.extra["boxes"][0]
    b0 = box.mass() * wl.manufactured_load(box.coords())
    b = b0 + 1e-3 * np.max(np.abs(b0)) * wl.uniform_noise(box.n, 0)
    res = krylov.pcg(box.apply, b, h.vcycle, 1e-8, 100, flexible=True)
    print(f"exact order-1 solve: {res.iterations} iterations ({time.time() - t0:.0f} s)", flush=True)
    write(os.path.join(HERE, "cfg3_fcg_fp64.txt"), "exact order-1 solve", box, lmax, b, res)
    # the lattice level's lambda_max from the same estimator, then the same solve
    A1 = mg.q1_lattice_levels(h.extra["boxes"][-1], 4096)[0][0]
    lm1 = lambda_max_SA(lambda x: A1 @ x, 1.0 / A1.diagonal(), A1.shape[0], tol=1e-10, maxit=300)
    lmax_l = lmax + [lm1]
    del h
    hl = mg.sem_hierarchy(V, N, cheb.CHEB4_OPT, 4, 0, lmax=lmax_l, coarse="lattice")
    assert [lev.n for lev in hl.levels[2:]] == [31 ** 3, 15 ** 3]
    boxl = hl.extra["boxes"][0]
    resl = krylov.pcg(boxl.apply, b, hl.vcycle, 1e-8, 100, flexible=True)
    print(f"lattice multigrid: {resl.iterations} iterations ({time.time() - t0:.0f} s)", flush=True)
    write(os.path.join(HERE, "cfg3_fcg_fp64_lattice.txt"), "lattice multigrid below order 1", boxl, lmax_l, b,
          resl)


if __name__ == "__main__":
    main()
