"""What the trained boundary-cell correction gains over the plain smoother.

Trains the MLP on the GPU (own kernels) from the method's own smoothing on
200 seeded sphere/ellipsoid geometries (16^3, Q3), then solves a held-out
8-sphere union (16^3, Q3, omega = 0.8) with and without it.  The plain
smoother stalls there; the test prints both residuals and asserts that the
learned form reaches a lower true residual, and that the judge keeps the
better of the two.
"""
import pytest
import torch

from paper_2506_12899_amd import learned, workloads

pytestmark = pytest.mark.gpu


def test_learned_correction_gain_on_held_out_union():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_12899_amd.problem import Problem
    dev = torch.device("cuda", 0)
    print("[learned] generating training data (200 geometries, n = 16, p = 3)", flush=True)
    data = learned.generate(lambda g, n, p: Problem(g, n, p, device=0), range(1, 201), 16, 3, 1, 4,
                            device=dev, log=lambda m: None)
    net = learned.MLP(data[0].shape[1], data[1].shape[1], 64, device=dev, omega=0.8, train_uv=True)
    hist = learned.train(net, data, epochs=30, batch=4096, lr=1e-3, log=lambda m: None, time_budget=60.0)
    assert hist[-1] < 0.1 * hist[0], hist
    uni = workloads.problem("balls128_q3")
    pb = Problem(uni.geometry, 16, 3, device=0)
    b = pb.rhs(uni.solution.f, uni.solution.u)
    x, st, choice = learned.judged_solve(pb, net, b, tol=1e-8, max_iter=150)
    p0, p1 = st["plain"], st["learned"]
    print(f"[learned] 8-ball union 16^3 Q3: plain {p0['iterations']} its rel {p0['rel_residual']:.2e}; "
          f"learned {p1['iterations']} its rel {p1['rel_residual']:.2e}; judge keeps {choice}", flush=True)
    assert not p0["converged"]
    assert p1["rel_residual"] < 0.5 * p0["rel_residual"]
    assert choice == "learned"
    # the kept solution is the learned run's: its true residual is the learned one
    r = torch.empty_like(b)
    pb.apply(x, r)
    rel = float(torch.linalg.vector_norm(b - r) / torch.linalg.vector_norm(b))
    assert abs(rel - p1["rel_residual"]) <= 1e-6 * max(rel, 1e-30) + 1e-14
