"""The allocation-free solve (sbm_solve_noalloc) against sbm_solve, through the C ABI.

Same arithmetic on the same inputs, only the workspace differs (the library's
fixed device scratch array instead of buffers the problem allocates): the
solutions and statistics agree to the FP64 parity bar (1e-10 relative; in
practice bit for bit).  Two calls in a row, the second on a smaller problem,
check that the shared array's leftover contents do not matter; a problem too
large for the array is refused before any device work.
"""
import numpy as np
import pytest
import torch

from paper_2506_12899_amd import native, workloads

pytestmark = pytest.mark.gpu


def _problem(geo, n, p, **kw):
    from paper_2506_12899_amd.problem import Problem
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Problem(geo, n, p, device=0, **kw)


def _rel(a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


CALLS = [
    # (geometry, n, p, options): the second is smaller than the first
    (workloads.balls([[0.0, 0.0]], [0.7]), 32, 2, {"coarse_dofs": 256}),
    (workloads.balls([[0.03, -0.02]], [0.6]), 16, 1, {"coarse_dofs": 64}),
]


@pytest.mark.parametrize("fp32", [0, 1])
def test_noalloc_solve_matches_solve_twice(fp32):
    sol = workloads.problem("disk32_q1").solution
    sizes = []
    for geo, n, p, kw in CALLS:
        print(f"[no-alloc] n={n} p={p} {kw} fp32={fp32}", flush=True)
        pb = _problem(geo, n, p, vcycle_fp32=fp32, **kw)
        sizes.append(pb.n_dofs)
        need = native.lib().sbm_solve_noalloc_doubles(pb._h, 30)
        assert 0 < need * 8 <= native.NOALLOC_SCRATCH_BYTES
        b = pb.rhs(sol.f, sol.u)
        x0, st0 = pb.solve(b, tol=1e-8)
        x1, st1 = pb.solve(b, tol=1e-8, noalloc=True)
        torch.cuda.synchronize()
        assert st0["converged"] and st1["converged"]
        assert st1["iterations"] == st0["iterations"]
        assert abs(st1["rel_residual"] - st0["rel_residual"]) <= 1e-10 * st0["rel_residual"]
        assert _rel(x1, x0) <= 1e-10
        # a restart shorter than the problem's own workspace was sized for
        x2, st2 = pb.solve(b, tol=1e-8, restart=7, noalloc=True)
        x3, st3 = pb.solve(b, tol=1e-8, restart=7)
        assert st2["iterations"] == st3["iterations"] and _rel(x2, x3) <= 1e-10
        del pb
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_a_problem_beyond_the_scratch_size():
    prob = workloads.problem("star512_q2")       # 687,654 DoFs: FGMRES(30) needs ~330 MiB
    pb = _problem(prob.geometry, prob.n, prob.p)
    need = native.lib().sbm_solve_noalloc_doubles(pb._h, 30)
    assert need * 8 > native.NOALLOC_SCRATCH_BYTES
    b = torch.ones(pb.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(native.SbmError) as e:
        pb.solve(b, tol=1e-8, noalloc=True)
    assert e.value.status == native.SBM_EINVAL and "scratch" in str(e.value)
    # a short enough restart fits
    assert native.lib().sbm_solve_noalloc_doubles(pb._h, 10) * 8 <= native.NOALLOC_SCRATCH_BYTES
