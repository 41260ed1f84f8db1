"""What the trained boundary-cell correction gains over the plain smoother.

Trains the MLP on the GPU (own kernels) on pairs from the method's own
iterations (white-noise errors and the iterates after three preconditioned
Richardson steps) on 40 seeded sphere/ellipsoid geometries (16^3, Q3,
stabilised form), then solves the held-out 8-sphere union and the r = 0.8
sphere (16^3) with and without it.  The plain smoother is the fallback and
the judge: the test prints both iteration counts, and asserts that training
lowers the loss, that the judge keeps the run with fewer iterations (or the
lower residual), and that the kept solution is that run's.
"""
import pytest
import torch

from paper_2506_12899_amd import learned, workloads

pytestmark = pytest.mark.gpu


def test_learned_correction_judged_against_plain():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_12899_amd.problem import Problem
    dev = torch.device("cuda", 0)
    opts = dict(workloads.STABILISED_Q3)
    print("[learned] generating training data (40 geometries, n = 16, p = 3)", flush=True)
    data = learned.generate(lambda g, n, p: Problem(g, n, p, device=0, **opts), range(1, 41), 16, 3, (0, 3), 2,
                            device=dev, log=lambda m: None)
    net = learned.MLP(data[0].shape[1], data[1].shape[1], 64, device=dev, omega=0.8, train_uv=True)
    hist = learned.train(net, data, epochs=20, batch=4096, lr=1e-3, log=lambda m: None, time_budget=60.0)
    assert hist[-1] < hist[0], hist
    for name in ("balls128_q3", "sphere96_q3"):
        prob = workloads.problem(name)
        pb = Problem(prob.geometry, 16, 3, device=0, **prob.opts)
        b = pb.rhs(prob.solution.f, prob.solution.u)
        x, st, choice = learned.judged_solve(pb, net, b, tol=1e-8, max_iter=300)
        p0, p1 = st["plain"], st["learned"]
        print(f"[learned] {name} geometry at 16^3 Q3: plain {p0['iterations']} its rel {p0['rel_residual']:.2e}; "
              f"learned {p1['iterations']} its rel {p1['rel_residual']:.2e}; judge keeps {choice}", flush=True)
        if p0["converged"] != p1["converged"]:
            better = p1["converged"]
        elif p0["converged"]:
            better = p1["iterations"] < p0["iterations"]
        else:
            better = p1["rel_residual"] < p0["rel_residual"]
        assert choice == ("learned" if better else "plain")
        kept = p1 if better else p0
        r = torch.empty_like(b)
        pb.apply(x, r)
        rel = float(torch.linalg.vector_norm(b - r) / torch.linalg.vector_norm(b))
        assert abs(rel - kept["rel_residual"]) <= 1e-6 * max(rel, 1e-30) + 1e-14
