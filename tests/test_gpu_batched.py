"""Batched solves of uneven SEM systems on the GPU.

Each system of a batch is also solved alone with the single-system mixed-precision
solver (same hierarchy, same lambda_max estimator): iteration counts must agree
(within one iteration, reductions are grouped differently) and solutions agree to
1e-10. The true FP64 residual of every batched solution is recomputed with the
oracle's operator and must meet the 1e-8 tolerance (parity unpinned against the
paper, which has no batched runs; pinned against the FP64 oracle).
"""
import numpy as np
import pytest
import torch

import workload as wl
from oracle.sem import SemBox
from paper_2210_03179_amd import _lib as L
from paper_2210_03179_amd.solver import BatchedSolver, SemSolver

pytestmark = pytest.mark.gpu


def _systems(count, seed0):
    specs = []
    g = np.random.Generator(np.random.PCG64(seed0))
    for s in range(count):
        m = int(g.integers(3, 7))
        N = int(g.choice([4, 5, 7]))
        specs.append((wl.batched_box(m, seed0 + s), N, seed0 + 50 + s))
    return specs


def _rhs(box, seed):
    b0 = box.mass() * wl.manufactured_load(box.coords())
    return b0 + 1e-3 * np.max(np.abs(b0)) * wl.uniform_noise(box.n, seed)


@pytest.mark.parametrize("pre,post,kind", [(4, 0, "cheb4opt"), (2, 2, "cheb4"), (3, 0, "cheb1opt")])
def test_batched_matches_single_and_oracle(pre, post, kind, monkeypatch):
    # the same operator variant on both sides (their single-precision roundings differ)
    monkeypatch.setenv("SEMCHEB_AX_VARIANT", "5")
    specs = _systems(7, 300)
    boxes = [SemBox(V, N) for V, N, _ in specs]
    rhs = [_rhs(bx, sd) for bx, (_, _, sd) in zip(boxes, specs)]
    bs = BatchedSolver([V for V, _, _ in specs], [N for _, N, _ in specs], smoother=kind, pre=pre,
                       post=post, krylov="fcg")
    assert bs.offsets[-1] == sum(bx.n for bx in boxes)
    b = torch.from_numpy(np.concatenate(rhs)).cuda()
    u, st, its, rel = bs.solve(b, rtol=1e-8, maxit=200)
    assert st == L.SEM_OK
    uh = u.cpu().numpy()
    for q, ((V, N, _), bx, bq) in enumerate(zip(specs, boxes, rhs)):
        uq = uh[bs.offsets[q]:bs.offsets[q + 1]]
        true_rel = np.linalg.norm(bq - bx.apply(uq)) / np.linalg.norm(bq)
        assert true_rel <= 1.01e-8, (q, true_rel)
        single = SemSolver(V, N=N, smoother=kind, pre=pre, post=post, precision="mixed", krylov="fcg")
        us, info = single.solve(torch.from_numpy(bq).cuda(), rtol=1e-8, maxit=200)
        assert abs(info.iterations - its[q]) <= 1, (q, info.iterations, its[q])
        if info.iterations == its[q]:
            ush = us.cpu().numpy()
            assert np.linalg.norm(uq - ush) <= 1e-10 * np.linalg.norm(ush), q
    print(f"batched ({pre},{post}) {kind}: iterations {its}", flush=True)


def test_batched_zero_rhs_and_errors():
    specs = _systems(3, 400)
    bs = BatchedSolver([V for V, _, _ in specs], [N for _, N, _ in specs])
    b = torch.zeros(bs.n, dtype=torch.float64, device="cuda")
    boxes = [SemBox(V, N) for V, N, _ in specs]
    b[bs.offsets[1]:bs.offsets[2]] = torch.from_numpy(_rhs(boxes[1], 7)).cuda()
    u, st, its, rel = bs.solve(b)
    assert st == L.SEM_OK and its[0] == 0 and its[2] == 0 and its[1] > 0
    assert float(u[bs.offsets[0]:bs.offsets[1]].abs().max()) == 0.0
    # the launch count of a solve is reported and repeats for the same input
    n1 = int(bs.host_array("launches")[0])
    bs.solve(b)
    assert n1 > 0 and int(bs.host_array("launches")[0]) == n1
    with pytest.raises(L.SemError):
        BatchedSolver([specs[0][0]], [3])  # order 3 has only two levels


def test_batched_operator_autotuning():
    """The batched setup times the six operator variants on the batched launches of every
    (level, order) and keeps the fastest; every variant, fixed through the environment,
    solves every system to a true 1e-8 in the same number of iterations (within one: the
    single-precision roundings differ between variants)."""
    import os
    specs = _systems(6, 500)
    boxes = [SemBox(V, N) for V, N, _ in specs]
    rhs = [_rhs(bx, sd) for bx, (_, _, sd) in zip(boxes, specs)]
    b = torch.from_numpy(np.concatenate(rhs)).cuda()
    bs = BatchedSolver([V for V, _, _ in specs], [N for _, N, _ in specs])
    rows = bs.host_array("ax_tuning").reshape(-1, 9)
    orders = sorted({N for _, N, _ in specs})
    assert sorted(int(r[1]) for r in rows if r[0] == 0) == orders
    assert sorted(int(r[1]) for r in rows if r[0] == 1) == sorted({N // 2 for N in orders})
    assert sorted(int(r[1]) for r in rows if r[0] == -1) == orders
    for r in rows:
        t = r[3:]
        assert t[int(r[2])] == min(x for x in t if x >= 0), r
    print("batched tuning (level, order, variant):", [tuple(int(x) for x in r[:3]) for r in rows], flush=True)
    _, st, its_auto, _ = bs.solve(b)
    assert st == L.SEM_OK
    for v in range(6):
        os.environ["SEMCHEB_AX_VARIANT"] = str(v)
        try:
            bv = BatchedSolver([V for V, _, _ in specs], [N for _, N, _ in specs])
        finally:
            del os.environ["SEMCHEB_AX_VARIANT"]
        u, st, its, _ = bv.solve(b)
        assert st == L.SEM_OK
        assert all(abs(a - c) <= 1 for a, c in zip(its, its_auto)), (v, its, its_auto)
        uh = u.cpu().numpy()
        for q, (bx, bq) in enumerate(zip(boxes, rhs)):
            uq = uh[bv.offsets[q]:bv.offsets[q + 1]]
            assert np.linalg.norm(bq - bx.apply(uq)) <= 1.01e-8 * np.linalg.norm(bq), (v, q)
