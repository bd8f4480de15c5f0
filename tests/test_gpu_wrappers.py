"""The Python binding checks every tensor against the context's sizes before it calls
the library: a tensor of the wrong length raises ValueError and nothing is launched
(the C ABI reads and writes the context's sizes, so a short tensor would be overrun)."""
import pytest

import workload as wl

pytestmark = pytest.mark.gpu


def test_wrong_sizes_raise_before_any_launch():
    import torch
    from paper_2210_03179_amd.solver import SemSolver, BatchedSolver

    V = wl.deformed_box(2, 0.05)
    s = SemSolver(V, N=3, lambda_max=[2.0, 2.0])
    n, nl, E = s.n, s.n_local, s.E
    good = torch.ones(n, dtype=torch.float64, device="cuda")
    short = torch.ones(n - 1, dtype=torch.float64, device="cuda")
    elem = torch.ones(E, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for call in (lambda: s.apply_A(short), lambda: s.apply_A(good, out=short),
                 lambda: s.vcycle(elem), lambda: s.vcycle(good, out=elem),
                 lambda: s.solve(short), lambda: s.solve(good, x0=short),
                 lambda: s.solve(good, out=short), lambda: s.mass_apply(short),
                 lambda: s.mass_apply(good, out=elem),
                 lambda: s.set_factors(torch.zeros(E * 6 * 64 - 1, dtype=torch.float64, device="cuda")),
                 lambda: s.adjoint_contract(short, good), lambda: s.adjoint_contract(good, short),
                 lambda: s.apply_local(short),
                 lambda: s.apply_local(good, out=torch.empty(nl - 1, dtype=torch.float64, device="cuda"))):
        with pytest.raises(ValueError):
            call()
    # the right sizes still work after the refusals
    w = s.apply_A(good)
    torch.cuda.synchronize()
    assert torch.isfinite(w).all()
    bs = BatchedSolver([wl.deformed_box(2, 0.05)], [5])
    with pytest.raises(ValueError):
        bs.solve(torch.ones(bs.n + 1, dtype=torch.float64, device="cuda"))
