#!/usr/bin/env python
"""Benchmark: PCG-to-1e-8 solves of the SEM Poisson problem on one MI355X.

Workload (default): 32x32x32 hexahedral box of [0,1]^3, vertices moved by
0.05 sin(pi x) sin(pi y) sin(pi z), order N = 7 (11,089,567 unknowns), p-multigrid
schedule (7,3,1), optimised 4th-kind Chebyshev-Jacobi smoothing of order 4 in a
one-sided V-cycle, exact order-1 coarse solve, flexible CG to ||r|| <= 1e-8 ||b||,
load 3 pi^2 sin sin sin plus 1e-3 relative U[-1,1] noise (seed 0).

One step = one full solve from x0 = 0 with the right-hand side resident in HBM.
Both forms are timed on the same GPU: the mixed-precision form (FP32 smoothing
with BF16 geometric factors inside an FP64 flexible CG, FP64 coarse solve) is
the reported `value`; the all-FP64 form is reported beside it.

Prints one JSON line (see the fields below). `roofline` is for the dominant
kernel, the FP64 element operator of apply_A, priced with the byte model's
apply_A bytes 48 L + 16 n (FP64 factors per local node, u and w once per unknown)
and timed with HIP events on the stream the library launches on, around each of
its launches inside the last timed FP64 solve (`us`; a loop of back-to-back
launches gives `us_back_to_back`); the complete apply_A (operator + direct-stiffness
summation) and the mixed cycle's BF16 operator are timed as back-to-back loops
and reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=32, help="elements per direction")
    ap.add_argument("--order", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-system batched measurement")
    ap.add_argument("--no-schwarz", action="store_true", help="skip the Chebyshev-Schwarz measurement")
    ap.add_argument("--no-trilinear", action="store_true",
                    help="skip the measurement with factors formed in the operator")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 64-system batched measurement (for profiler runs)")
    ap.add_argument("--solve-only", action="store_true",
                    help="set up the FP64 and mixed contexts and run --steps solves of each, nothing else "
                         "(short runs for profilers)")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--kernel-only", action="store_true",
                    help="set up the FP64 and mixed contexts with fixed lambda_max and only launch the "
                         "element-local operator --kernel-reps times each (short runs for profilers)")
    return ap.parse_args()


def kernel_only(args):
    import torch

    import workload as wl
    from paper_2210_03179_amd.solver import SemSolver
    V = wl.deformed_box(args.m, 0.05)
    lam = [2.0, 2.0]  # operator launches do not use lambda_max; skips the estimator's launches
    s64 = SemSolver(V, N=args.order, precision="fp64", lambda_max=lam)
    smx = SemSolver(V, N=args.order, precision="mixed", lambda_max=lam)
    n, nloc = s64.n, s64.n_local
    u = torch.rand(n, dtype=torch.float64, device="cuda")
    w = torch.empty(nloc, dtype=torch.float64, device="cuda")
    u32, w32 = u.float(), torch.empty(nloc, dtype=torch.float32, device="cuda")
    t64 = time_kernel(lambda: s64.apply_local(u, w), args.kernel_reps)
    tmx = time_kernel(lambda: smx.apply_local(u32, w32), args.kernel_reps)
    wg = torch.empty(n, dtype=torch.float64, device="cuda")
    tap = time_kernel(lambda: s64.apply_A(u, wg), args.kernel_reps)  # operator + summation
    # the same operator with factors formed in the kernel (trilinear geometry option)
    st64 = SemSolver(V, N=args.order, precision="fp64", lambda_max=lam, geometry="trilinear")
    stmx = SemSolver(V, N=args.order, precision="mixed", lambda_max=lam, geometry="trilinear")
    tt64 = time_kernel(lambda: st64.apply_local(u, w), args.kernel_reps)
    ttmx = time_kernel(lambda: stmx.apply_local(u32, w32), args.kernel_reps)
    # plain device copy of a known size (1 GiB read + 1 GiB written per launch): the reference
    # against which the profiler's FETCH_SIZE / WRITE_SIZE counters are scaled
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    tcp = time_kernel(lambda: dst.copy_(src), 3)
    print(json.dumps({"kernel_only": True, "unknowns": n, "local_nodes": nloc,
                      "copy_bytes": 2 * src.numel() * 8, "copy_us": tcp * 1e6,
                      "copy_GBs": 2 * src.numel() * 8 / tcp / 1e9,
                      "apply_A_fp64_us": tap * 1e6, "apply_A_fp64_GBs": (48.0 * nloc + 16.0 * n) / tap / 1e9,
                      "ax_fp64_us": t64 * 1e6, "ax_fp64_GBs": (56.0 * nloc + 8.0 * n) / t64 / 1e9,
                      "ax_bf16_us": tmx * 1e6, "ax_bf16_GBs": (16.0 * nloc + 4.0 * n) / tmx / 1e9,
                      "ax_trilinear_fp64_us": tt64 * 1e6, "ax_trilinear_fp32_us": ttmx * 1e6}), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_solves(solver, b, steps, warmup):
    """Mean time per solve over `steps` back-to-back solves, plus each solve's own wall time
    (a solve ends with a stream synchronisation, so the per-solve times are exact)."""
    import torch
    info = None
    u = torch.empty_like(b)  # preallocated: no device allocation inside the timed region
    for _ in range(warmup):
        _, info = solver.solve(b, rtol=1e-8, maxit=500, out=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, each = [], []
    for _ in range(steps):
        t1 = time.perf_counter()
        u, info = solver.solve(b, rtol=1e-8, maxit=500, out=u)
        each.append(time.perf_counter() - t1)
        its.append(info.iterations)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return u, info, dt, its, each


# operator variant index -> (prefetch, occupancy, tile) template arguments; N <= 7 asks for 4 waves
def _variant_args(variant, N, fp64=False):
    mw = 4 if N <= 7 else 2
    if variant == 5 and fp64:  # the FP64 factor ring (N = 7); other orders launch variant 0
        return (0, mw, 3) if N == 7 else (1, 1, 0)
    if variant == 6 and fp64:  # variant 2 with elements in launch order
        return (1, mw, 5)
    if variant == 6 and N == 7:  # matrix-core contractions (BF16 factors at N = 7)
        return (0, mw, 4)
    return {0: (1, 1, 0), 1: (0, mw, 0), 2: (1, mw, 0), 3: (1, 1, 1), 4: (0, mw, 1), 5: (0, mw, 2),
            6: (0, mw, 2)}[variant]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE in KiB per dispatch, scaled by the factors a 1 GiB copy gives); None when the
    summary does not cover this kernel."""
    path = os.path.join(ROOT, "profiles", "ax_n7_hbm_counters.md")
    if not os.path.exists(path):
        return None
    sf = sw = None
    row = None
    for line in open(path):
        if line.startswith("Calibration:"):
            mt = re.search(r"FETCH_SIZE is scaled by ([0-9.]+) and WRITE_SIZE by ([0-9.]+?)\.?\s*$", line)
            if mt:
                sf, sw = float(mt.group(1)), float(mt.group(2))
        if row is None and line.startswith(f"| `{kernel}`"):  # first table: FETCH / WRITE KiB
            row = [c.strip() for c in line.strip().strip("|").split("|")]
    if sf is None or row is None:
        return None
    return float(row[1]) * 1024 * sf + float(row[2]) * 1024 * sw


def time_kernel(fn, reps):
    """Average duration of fn() (one kernel launch) with events on the current stream."""
    import torch
    fn()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps * 1e-3


def bench_batched(steps, nsys=64):
    """64 independent systems (m ~ U{4..16}, N ~ U{5,7,9}, per-system random deformation and
    rhs): one batched mixed-precision solve of all systems versus the plain FP64 form (every
    system solved on its own, one after the other) on the same GPU."""
    import torch

    import workload as wl
    from paper_2210_03179_amd.solver import BatchedSolver, SemSolver
    specs = wl.batched_specs(nsys, 1000)
    verts = [wl.batched_box(sp.m, sp.mesh_seed) for sp in specs]
    t0 = time.perf_counter()
    singles = [SemSolver(V, N=sp.N, smoother="cheb4opt", pre=4, post=0, precision="fp64", krylov="fcg")
               for V, sp in zip(verts, specs)]
    t_setup64 = time.perf_counter() - t0
    rhs = []
    for s, sp in zip(singles, specs):
        f = wl.manufactured_load(s.coords().cpu().numpy())
        b0 = s.mass_apply(torch.from_numpy(f).cuda()).cpu().numpy()
        rhs.append(b0 + 1e-3 * np.max(np.abs(b0)) * wl.uniform_noise(s.n, sp.rhs_seed))
    t0 = time.perf_counter()
    bs = BatchedSolver(verts, [sp.N for sp in specs], smoother="cheb4opt", pre=4, post=0, krylov="fcg")
    t_setupb = time.perf_counter() - t0
    b = torch.from_numpy(np.concatenate(rhs)).cuda()
    bs.solve(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u, st, its, rel = bs.solve(b)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    bdev = [torch.from_numpy(r).cuda() for r in rhs]
    for s, bq in zip(singles, bdev):
        s.solve(bq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its64 = []
    for s, bq in zip(singles, bdev):
        _, info = s.solve(bq)
        its64.append(info.iterations)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    # true FP64 residual of every batched solution with each system's FP64 operator
    worst = 0.0
    for q, (s, bq) in enumerate(zip(singles, bdev)):
        uq = u[bs.offsets[q]:bs.offsets[q + 1]].contiguous()
        worst = max(worst, float(torch.linalg.vector_norm(bq - s.apply_A(uq)) / torch.linalg.vector_norm(bq)))
    ns = [bs.offsets[q + 1] - bs.offsets[q] for q in range(nsys)]
    # operator variants chosen by the batched autotuner: (level, order) -> (variant, us); level -1
    # is the FP64 Krylov operator
    tune = {f"{int(r[0])}:{int(r[1])}": [int(r[2]), round(float(r[3 + int(r[2])]), 1)]
            for r in bs.host_array("ax_tuning").reshape(-1, 9)}
    return {"systems": nsys, "unknowns": bs.n, "ms_per_batch_solve": round(t_batch * 1e3, 3),
            "ms_fp64_one_by_one": round(t_seq * 1e3, 3), "speedup_vs_fp64": round(t_seq / t_batch, 3),
            "gdof_iter_per_s": round(sum(n * i for n, i in zip(ns, its)) / t_batch / 1e9, 4),
            "iterations_min_max": [min(its), max(its)], "fp64_iterations_min_max": [min(its64), max(its64)],
            "worst_true_relres": worst, "status": st, "operator_variants": tune,
            "launches_per_solve": int(bs.host_array("launches")[0]),
            "setup_s": {"fp64_systems": round(t_setup64, 1), "batched": round(t_setupb, 1)}}


def cpu_baseline(m, N, n_global):
    """The oracle (numpy FP64) on the same workload, one thread: exactly one flexible-CG
    iteration, i.e. one operator application w = A p, the residual and iterate updates with
    their dot products, and one V-cycle z = M r, each timed on the host with the oracle's
    own functions and summed. BLAS is limited to one thread for the timed calls; numpy's
    einsum contractions, the oracle's main cost, run on one thread anyway. lambda_max does
    not change the cost and is set to 2 (no Lanczos run)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import workload as wl
    from oracle import chebyshev as cheb, mg
    with threadpool_limits(limits=1):
        threads = max([1] + [int(d.get("num_threads", 1)) for d in threadpool_info()])
        V = wl.deformed_box(m, 0.05)
        h = mg.sem_hierarchy(V, N, cheb.CHEB4_OPT, 4, 0, lmax=[2.0, 2.0])
        box = h.extra["boxes"][0]
        b = box.mass() * wl.manufactured_load(box.coords())
        r, p, x, r_old = b.copy(), b.copy(), np.zeros_like(b), b.copy()
        rz = float(b @ b)
        t0 = time.perf_counter()
        w = box.apply(p)                      # w = A p
        t1 = time.perf_counter()
        alpha = rz / float(p @ w)             # vector part of the iteration (as oracle.krylov.pcg)
        x = x + alpha * p
        r_old, r = r, r - alpha * w
        float(np.linalg.norm(r))
        t2 = time.perf_counter()
        z = h.vcycle(r)                       # z = M r
        t3 = time.perf_counter()
        beta = float(z @ (r - r_old)) / rz
        rz = float(r @ z)
        p = z + beta * p
        t4 = time.perf_counter()
    dt = t4 - t0
    return {"value": round(n_global / dt / 1e9, 6), "unit": "GDOF-iter/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one flexible-CG iteration on the full {m}^3 N={N} box ({n_global} unknowns), "
                      f"single thread: operator {t1 - t0:.2f} s + V-cycle {t3 - t2:.2f} s + vector "
                      f"updates {t2 - t1 + t4 - t3:.2f} s = {dt:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is a design only",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import workload as wl
    from paper_2210_03179_amd.solver import SemSolver

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if args.kernel_only:
        kernel_only(args)
        return
    if args.batched_only:
        print(json.dumps({"batched": bench_batched(max(1, args.steps // 2))}), flush=True)
        return
    m, N = args.m, args.order
    V = wl.deformed_box(m, 0.05)
    t0 = time.perf_counter()
    s64 = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, precision="fp64", krylov="fcg")
    t_setup64 = time.perf_counter() - t0
    log(f"fp64 setup {t_setup64:.1f} s, lambda_max {s64.lambda_max()}")
    t0 = time.perf_counter()
    smx = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, precision="mixed", krylov="fcg")
    t_setupmx = time.perf_counter() - t0
    log(f"mixed setup {t_setupmx:.1f} s")
    n = s64.n
    nloc = s64.n_local
    f = wl.manufactured_load(s64.coords().cpu().numpy())
    b0 = s64.mass_apply(torch.from_numpy(f).cuda()).cpu().numpy()
    bh = b0 + 1e-3 * np.max(np.abs(b0)) * wl.uniform_noise(n, 0)
    b = torch.from_numpy(bh).cuda()
    if args.solve_only:
        _, i64, d64, _, _ = time_solves(s64, b, args.steps, 0)
        _, imx, dmx, _, _ = time_solves(smx, b, args.steps, 0)
        print(json.dumps({"solve_only": True, "unknowns": n, "fp64": {"iterations": i64.iterations,
                                                                     "ms_per_solve": d64 * 1e3},
                          "mixed": {"iterations": imx.iterations, "ms_per_solve": dmx * 1e3}}), flush=True)
        return

    # the FP64 solves also time their Krylov operator launches: an event pair around each launch
    # on the library's stream, inside the timed region (two stream markers per iteration)
    os.environ["SEMCHEB_TIME_KRYLOV_OP"] = "1"
    try:
        u64, info64, dt64, its64, each64 = time_solves(s64, b, args.steps, args.warmup)
    finally:
        del os.environ["SEMCHEB_TIME_KRYLOV_OP"]
    kop_us = s64.host_array("krylov_operator_us")  # the last timed solve, one value per iteration
    log(f"fp64: {info64.iterations} its, {dt64 * 1e3:.2f} ms/solve")
    umx, infomx, dtmx, itsmx, eachmx = time_solves(smx, b, args.steps, args.warmup)
    log(f"mixed: {infomx.iterations} its, {dtmx * 1e3:.2f} ms/solve")

    def true_rel(u):
        r = b - s64.apply_A(u)
        return float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))

    rel64, relmx = true_rel(u64), true_rel(umx)
    err_mx = float(torch.linalg.vector_norm(umx - u64) / torch.linalg.vector_norm(u64))

    # apply_A as the byte model counts it (48 B of FP64 factors per local node, u read and
    # w written once per unknown: 48 L + 16 n), timed as the complete sem_apply_A (element
    # operator + direct-stiffness summation) and as the element operator alone; FLOPs of the
    # tensor-product operator: 12 (N+1)^4 + 17 (N+1)^3 per element (three derivatives and their
    # transposes, 15 flops of factor products and 2 of sums per node). The mixed cycle's apply:
    # 12 L + 8 n (BF16 factors, FP32 vectors).
    E = nloc // (N + 1) ** 3
    alg64 = 48.0 * nloc + 16.0 * n
    algmx = 12.0 * nloc + 8.0 * n
    flops = float(12 * (N + 1) ** 4 + 17 * (N + 1) ** 3) * E
    u_rand = torch.rand(n, dtype=torch.float64, device="cuda")
    w_glob = torch.empty(n, dtype=torch.float64, device="cuda")
    w_loc = torch.empty(nloc, dtype=torch.float64, device="cuda")
    t_apply = time_kernel(lambda: s64.apply_A(u_rand, w_glob), args.kernel_reps)
    t_ax64_loop = time_kernel(lambda: s64.apply_local(u_rand, w_loc), args.kernel_reps)
    # the roofline duration is the operator's own inside the timed FP64 solves (its input then
    # comes from the update that has just written it), the back-to-back loop is reported beside it
    t_ax64 = float(np.mean(kop_us)) * 1e-6 if len(kop_us) else t_ax64_loop
    u32 = u_rand.float()
    w32 = torch.empty(nloc, dtype=torch.float32, device="cuda")
    t_axmx = time_kernel(lambda: smx.apply_local(u32, w32), args.kernel_reps)
    # achievable streaming bandwidth on this device: a 2 GiB device-to-device copy
    # (1 GiB read + 1 GiB written), the reference the operator's fraction can also be read against
    cpy_src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    cpy_dst = torch.empty_like(cpy_src)
    t_copy = time_kernel(lambda: cpy_dst.copy_(cpy_src), 10)
    copy_gbs = 2.0 * cpy_src.numel() * 8 / t_copy / 1e9
    del cpy_src, cpy_dst
    log(f"apply_A fp64 {t_apply * 1e6:.1f} us ({alg64 / t_apply / 1e9:.0f} GB/s), element operator fp64 "
        f"{t_ax64 * 1e6:.1f} us, bf16 {t_axmx * 1e6:.1f} us ({algmx / t_axmx / 1e9:.0f} GB/s)")

    gdof_mx = n * infomx.iterations / dtmx / 1e9
    gdof_64 = n * info64.iterations / dt64 / 1e9
    ach = alg64 / t_apply / 1e9
    tune64 = s64.host_array("ax_tuning", 0)
    tunemx = smx.host_array("ax_tuning", 0)
    nvar = (len(tune64) // s64.num_levels - 2) // 2  # per level: variant, times (FP64), variant, times
    v64, vmx = int(tune64[0]), int(tunemx[1 + nvar])
    k64 = "ax_local_kernel<%d, double, double, %d, %d, %d>" % ((N,) + _variant_args(v64, N, fp64=True))
    kmx = "ax_local_kernel<%d, float, unsigned short, %d, %d, %d>" % ((N,) + _variant_args(vmx, N))  # BF16 storage
    log(f"operator variants (us) fp64 {[round(x, 1) for x in tune64[1:1 + nvar]]} -> {v64}, "
        f"bf16 {[round(x, 1) for x in tunemx[2 + nvar:2 + 2 * nvar]]} -> {vmx}")
    per = 2 * (1 + nvar)
    for j in range(1, s64.num_levels - 1):  # the smoothed lower levels
        t64, tmx = tune64[j * per:(j + 1) * per], tunemx[j * per:(j + 1) * per]
        log(f"level {j} operator variants (us) fp64 {[round(x, 1) for x in t64[1:1 + nvar]]} -> {int(t64[0])}, "
            f"bf16 {[round(x, 1) for x in tmx[2 + nvar:2 + 2 * nvar]]} -> {int(tmx[1 + nvar])}")
    kdss = "dss_kernel<double, double, 2>"
    tr_ax = measured_traffic(k64) if N == 7 and m == 32 else None
    tr_dss = measured_traffic(kdss) if N == 7 and m == 32 else None
    tr_apply = tr_ax + tr_dss if (tr_ax is not None and tr_dss is not None) else None
    trmx = measured_traffic(kmx) if N == 7 and m == 32 else None
    out = {
        "metric": "PCG-to-1e-8 solve time & GDOF-iter/s; mixed/batched vs plain FP64 same GPU",
        "value": round(gdof_mx, 4),
        "unit": "GDOF-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dtmx * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16 V-cycle / f64 Krylov",
        "data": "synthetic",
        "config": {"workload": f"SEM Poisson {m}^3 deformed hex box, N={N}, pMG ({N},{N // 2},1), "
                               f"opt-4th Chebyshev (4,0) one-sided, FCG to 1e-8",
                   "unknowns": n, "local_nodes": nloc, "parallelism": "single GPU"},
        "iterations": infomx.iterations,
        "true_relres": relmx,
        "rel_diff_to_fp64_solution": err_mx,
        "ms_min": round(min(eachmx) * 1e3, 4),
        "ms_median": round(float(np.median(eachmx)) * 1e3, 4),
        "fp64": {"ms_per_solve": round(dt64 * 1e3, 4), "ms_min": round(min(each64) * 1e3, 4),
                 "ms_median": round(float(np.median(each64)) * 1e3, 4), "iterations": info64.iterations,
                 "gdof_iter_per_s": round(gdof_64, 4), "true_relres": rel64},
        "speedup_mixed_vs_fp64": round(dt64 / dtmx, 4),
        "setup_s": {"fp64": round(t_setup64, 2), "mixed": round(t_setupmx, 2)},
        # roofline of the dominant kernel, the FP64 element operator of apply_A: achieved = the byte
        # model's apply_A bytes (48 L + 16 n: the factors, u read and w written once per unknown)
        # over its duration (HIP events on the library's stream); traffic = HBM bytes the profiler
        # counted for the same kernel (committed counter summary, FETCH_SIZE and WRITE_SIZE scaled by
        # a copy of known size) over the same duration, null when the summary does not cover it.
        # complete_apply_A prices the whole sem_apply_A (operator + summation) the same way.
        "roofline": {"bound": "hbm", "achieved": round(alg64 / t_ax64 / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(alg64 / t_ax64 / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": round(tr_ax / t_ax64 / 1e9, 1) if tr_ax else None,
                     "kernel": k64, "us": round(t_ax64 * 1e6, 2),
                     "us_source": "in-solve" if len(kop_us) else "back-to-back",
                     "launches_timed": int(len(kop_us)), "us_back_to_back": round(t_ax64_loop * 1e6, 2),
                     "algorithmic_bytes": alg64,
                     "traffic_bytes": tr_ax, "copy_GBs": round(copy_gbs, 1),
                     "frac_of_copy": round(alg64 / t_ax64 / 1e9 / copy_gbs, 4),
                     "flops": flops, "TFLOPs": round(flops / t_ax64 / 1e12, 3), "fp64_peak_TFLOPs": 78.6,
                     "flop_frac": round(flops / t_ax64 / 1e12 / 78.6, 4),
                     "complete_apply_A": {"kernels": f"{k64} + {kdss}", "us": round(t_apply * 1e6, 2),
                                          "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                                          "traffic": round(tr_apply / t_apply / 1e9, 1) if tr_apply else None,
                                          "TFLOPs": round(flops / t_apply / 1e12, 3)},
                     "mixed_operator": {"kernel": kmx, "us": round(t_axmx * 1e6, 2),
                                        "achieved": round(algmx / t_axmx / 1e9, 1),
                                        "frac": round(algmx / t_axmx / 1e9 / HBM_PEAK_GBS, 4),
                                        "algorithmic_bytes": algmx,
                                        "TFLOPs": round(flops / t_axmx / 1e12, 3), "fp32_peak_TFLOPs": 157.3,
                                        "traffic": round(trmx / t_axmx / 1e9, 1) if trmx else None}},
    }
    # Table ksp-comparison analogue: time per iteration of GMRES(30) (classical Gram-Schmidt)
    # against flexible CG, same mixed-precision preconditioner
    sgm = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, precision="mixed", krylov="gmres",
                    restart=30, lambda_max=smx.lambda_max())
    _, infogm, dtgm, _, eachgm = time_solves(sgm, b, max(1, args.steps // 2), 1)
    out["gmres30"] = {"ms_per_solve": round(dtgm * 1e3, 4), "iterations": infogm.iterations,
                      "ms_per_iteration": round(dtgm * 1e3 / max(infogm.iterations, 1), 4),
                      "fcg_ms_per_iteration": round(dtmx * 1e3 / max(infomx.iterations, 1), 4)}
    log(f"gmres(30): {out['gmres30']}")
    del sgm
    if not args.no_schwarz:
        # Chebyshev-accelerated RAS smoothing with FDM local solves (Sec. 4.1), 4th kind (2,0),
        # same hierarchy and mixed precision, GMRES(30) as in the paper's Schwarz runs
        t0 = time.perf_counter()
        ssw = SemSolver(V, N=N, smoother="cheb4", pre=2, post=0, precision="mixed", krylov="gmres", restart=30,
                        schwarz="ras")
        t_sw_setup = time.perf_counter() - t0
        _, infosw, dtsw, _, _ = time_solves(ssw, b, max(1, args.steps // 2), 1)
        out["schwarz_ras_cheb4_2_0"] = {"ms_per_solve": round(dtsw * 1e3, 4), "iterations": infosw.iterations,
                                        "ms_per_iteration": round(dtsw * 1e3 / max(infosw.iterations, 1), 4),
                                        "setup_s": round(t_sw_setup, 2), "lambda_max": ssw.lambda_max()}
        log(f"schwarz RAS: {out['schwarz_ras_cheb4_2_0']}")
        del ssw
    if not args.no_trilinear:
        # the same solves with the geometric factors formed inside the operator from the
        # trilinear element geometry (36 edge values per element) instead of read from HBM;
        # not the headline: it holds for trilinear elements only
        stm = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, precision="mixed", geometry="trilinear",
                        lambda_max=smx.lambda_max())
        st64 = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, precision="fp64", geometry="trilinear",
                         lambda_max=s64.lambda_max())
        utm, infotm, dttm, _, _ = time_solves(stm, b, max(1, args.steps // 2), 1)
        ut64, infot64, dtt64, _, _ = time_solves(st64, b, max(1, args.steps // 2), 1)
        t_tax64 = time_kernel(lambda: st64.apply_local(u_rand, w_loc), args.kernel_reps)
        t_tax32 = time_kernel(lambda: stm.apply_local(u32, w32), args.kernel_reps)
        E = nloc // (N + 1) ** 3
        out["trilinear_geometry"] = {
            "mixed": {"ms_per_solve": round(dttm * 1e3, 4), "iterations": infotm.iterations,
                      "gdof_iter_per_s": round(n * infotm.iterations / dttm / 1e9, 4),
                      "true_relres": true_rel(utm)},
            "fp64": {"ms_per_solve": round(dtt64 * 1e3, 4), "iterations": infot64.iterations,
                     "gdof_iter_per_s": round(n * infot64.iterations / dtt64 / 1e9, 4),
                     "true_relres": true_rel(ut64)},
            # algorithmic bytes: u gathered once per unknown, w stored per local node, 36 edge
            # values per element
            "ax_fp64_us": round(t_tax64 * 1e6, 2),
            "ax_fp64_GBs": round((8.0 * n + 8.0 * nloc + 288.0 * E) / t_tax64 / 1e9, 1),
            "ax_fp32_us": round(t_tax32 * 1e6, 2),
            "ax_fp32_GBs": round((4.0 * n + 4.0 * nloc + 144.0 * E) / t_tax32 / 1e9, 1),
            "variants_fp64_us": [round(x, 1) for x in st64.host_array("ax_tuning", 0)[1:4]],
            "variants_fp32_us": [round(x, 1) for x in stm.host_array("ax_tuning", 0)[2 + nvar:5 + nvar]],
        }
        log(f"trilinear geometry: {out['trilinear_geometry']}")
        stm.close()
        st64.close()
    # the cycle continued below order 1 on the vertex lattice (one smoothed lattice level of
    # 29,791 unknowns, dense 3,375-unknown last level) instead of the exact order-1 solve, in
    # both precisions; the lattice levels run in FP64 in both
    slm = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, precision="mixed", coarse="lattice")
    sl64 = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, precision="fp64", coarse="lattice",
                     lambda_max=slm.lambda_max())
    ulm, infolm, dtlm, _, eachlm = time_solves(slm, b, args.steps, 1)
    ul64, infol64, dtl64, _, eachl64 = time_solves(sl64, b, args.steps, 1)
    out["lattice_coarse"] = {
        "levels": [sl64.level_info(j)[1] for j in range(sl64.num_levels)],
        "mixed": {"ms_per_solve": round(dtlm * 1e3, 4), "ms_min": round(min(eachlm) * 1e3, 4),
                  "iterations": infolm.iterations, "gdof_iter_per_s": round(n * infolm.iterations / dtlm / 1e9, 4),
                  "true_relres": true_rel(ulm)},
        "fp64": {"ms_per_solve": round(dtl64 * 1e3, 4), "ms_min": round(min(eachl64) * 1e3, 4),
                 "iterations": infol64.iterations, "gdof_iter_per_s": round(n * infol64.iterations / dtl64 / 1e9, 4),
                 "true_relres": true_rel(ul64)},
        "speedup_mixed_vs_fp64": round(dtl64 / dtlm, 4)}
    log(f"lattice coarse: {out['lattice_coarse']}")
    slm.close()
    sl64.close()
    if not args.no_trilinear:
        # option: the mixed cycle's coarse solve reads FP32 copies of its factor blocks (FP64
        # vectors, products and sums); the headline keeps FP64 factors
        scs = SemSolver(V, N=N, smoother="cheb4opt", pre=4, post=0, precision="mixed", coarse_storage="mixed",
                        lambda_max=smx.lambda_max())
        ucs, infocs, dtcs, _, _ = time_solves(scs, b, max(1, args.steps // 2), 1)
        out["mixed_fp32_coarse_factors"] = {"ms_per_solve": round(dtcs * 1e3, 4), "iterations": infocs.iterations,
                                            "gdof_iter_per_s": round(n * infocs.iterations / dtcs / 1e9, 4),
                                            "true_relres": true_rel(ucs)}
        log(f"mixed, FP32 coarse factors: {out['mixed_fp32_coarse_factors']}")
        scs.close()
    if not args.no_schwarz:
        # Table ksp-comparison's preconditioner: 1st-kind Chebyshev with Jacobi, symmetric (3,3)
        # cycle over the (7,5,3,1) schedule, FP64, under CG and under GMRES(30); the paper's run
        # is a Kershaw mesh of 16M unknowns on 6 V100s, 1.26e-2 s per CG iteration at eps = 1
        sk = SemSolver(V, N=N, smoother="cheb1", pre=3, post=3, precision="fp64", krylov="pcg",
                       orders=[7, 5, 3, 1] if N == 7 else None)
        _, infok, dtk, _, _ = time_solves(sk, b, max(1, args.steps // 2), 1)
        skg = SemSolver(V, N=N, smoother="cheb1", pre=3, post=3, precision="fp64", krylov="gmres", restart=30,
                        orders=[7, 5, 3, 1] if N == 7 else None, lambda_max=sk.lambda_max())
        _, infokg, dtkg, _, _ = time_solves(skg, b, max(1, args.steps // 2), 1)
        out["ksp_comparison_cheb1_3_3_fp64"] = {
            "cg": {"ms_per_solve": round(dtk * 1e3, 4), "iterations": infok.iterations,
                   "ms_per_iteration": round(dtk * 1e3 / max(infok.iterations, 1), 4),
                   "gdof_iter_per_s": round(n * infok.iterations / dtk / 1e9, 4)},
            "gmres30": {"ms_per_solve": round(dtkg * 1e3, 4), "iterations": infokg.iterations,
                        "ms_per_iteration": round(dtkg * 1e3 / max(infokg.iterations, 1), 4)}}
        log(f"ksp comparison (1st-kind Jacobi (3,3), 7/5/3/1, fp64): {out['ksp_comparison_cheb1_3_3_fp64']}")
        sk.close()
        skg.close()
    if not args.no_batched:
        log("batched systems ...")
        out["batched"] = bench_batched(max(1, args.steps // 2))
        log(f"batched: {out['batched']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(m, N, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
