"""The paper's own setting (paper_2506_12899_amd.paper_mode) against the
iteration counts the paper prints (tests/golden/paper_iterations.txt).

Parity unpinned in the strict sense: this build orders the cell-wise smoother
red-black instead of sequentially and restarts FGMRES every 30 iterations,
and the penalty scaling is a reading, so equal counts are not expected.  The
test holds the p = 1, 2 unit-disk and unit-sphere studies to converge where the
paper converges, within 2 x the printed count + 4 iterations, and prints the
side-by-side table.
"""
import os

import pytest
import torch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_iterations.txt")


def _paper():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            src, kind, d, p, lam, lv, its = line.split()
            rows[(kind, int(d), int(p), float(lam), int(lv))] = int(its)
    return rows


CASES = [("ball", 2, 1, range(1, 6)), ("ball", 2, 2, range(1, 6)), ("ball", 3, 1, range(1, 4)),
         ("ball", 3, 2, range(1, 3))]


@pytest.mark.parametrize("kind,d,p,levels", CASES)
def test_iterations_against_printed_figures(kind, d, p, levels):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_12899_amd import paper_mode
    ref = _paper()
    rows = paper_mode.iterations(kind, d, p, list(levels), lambdas=(1.0, 0.75, 0.5, 0.25))
    for r in rows:
        key = (kind, d, p, r["lam"], r["level"])
        pits = ref.get(key)
        print(f"[paper] {kind} {d}D p={p} lambda={r['lam']} level {r['level']}: ours {r.get('iterations')} "
              f"(converged {r.get('converged')}), paper {pits}", flush=True)
        if pits is None or pits >= 100:
            continue
        assert "error" not in r and r["converged"], r
        assert r["iterations"] <= 2 * pits + 4, (r, pits)


@pytest.mark.parametrize("p", [1, 2])
def test_deformed_domain_solves(p):
    """Sec. 5.4 deformed domain (callback level set, Lagrangian-Newton closest
    points), lambda = 0.5, levels 3-5: the GPU solve reaches 1e-12 within the
    paper's 100-iteration budget, and at level 3 the oracle's matrix and
    right-hand side confirm the true residual (1e-8 solve)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import numpy as np
    from oracle import dg
    from paper_2506_12899_amd import paper_mode
    from paper_2506_12899_amd.problem import Problem
    from tests.oracle_geom import oracle_geometry
    rows = paper_mode.iterations("deformed", 2, p, [3, 4, 5], lambdas=(0.5,))
    for r in rows:
        print(f"[paper] deformed 2D p={p} lambda=0.5 level {r['level']}: {r.get('iterations')} its "
              f"(converged {r.get('converged')})", flush=True)
        assert "error" not in r and r["converged"], r
    pr = paper_mode.problem("deformed", 2, 3, p, 0.5)
    pb = Problem(pr.geometry, pr.n, pr.p, device=0, **pr.opts)
    b = pb.rhs(pr.solution.f, pr.solution.u)
    x, st = pb.solve(b, tol=1e-8)
    assert st["converged"]
    o = {k: v for k, v in pr.opts.items() if k in ("lo", "hi", "lambda_frac", "c_F", "c_G")}
    L = dg.Level(oracle_geometry(pr.geometry), 2, pr.n, p, **o)
    bo = L.rhs(pr.solution.f, pr.solution.u)
    assert np.linalg.norm(b.cpu().numpy() - bo) <= 1e-10 * np.linalg.norm(bo)
    assert np.linalg.norm(bo - L.A @ x.cpu().numpy()) <= 1e-8 * np.linalg.norm(bo) * (1 + 1e-6)
