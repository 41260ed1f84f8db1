"""Pins of the oracle's learned-smoother reference (forward, loss, backward, Adam)."""
import numpy as np
import pytest

from oracle import mg, mlp
from paper_2506_12899_amd import workloads
from tests.oracle_geom import oracle_geometry

N_IN, WIDTH, NC = 12, 16, 8


def _sample(seed=0, S=7):
    rng = np.random.default_rng(seed)
    n_out = 1 + 2 * NC * 4
    theta = rng.standard_normal(mlp.n_params(N_IN, WIDTH, n_out)) * 0.3
    X = rng.standard_normal((S, N_IN))
    r = rng.standard_normal((S, NC))
    Br = rng.standard_normal((S, NC))
    e = rng.standard_normal((S, NC))
    return theta, X, r, Br, e


def test_gradient_matches_central_differences():
    theta, X, r, Br, e = _sample()
    L, g = mlp.loss_grad(theta, X, r, Br, e, 0.8, N_IN, WIDTH, NC)
    rng = np.random.default_rng(1)
    idx = rng.choice(len(theta), 60, replace=False)
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (mlp.loss_grad(tp, X, r, Br, e, 0.8, N_IN, WIDTH, NC)[0]
              - mlp.loss_grad(tm, X, r, Br, e, 0.8, N_IN, WIDTH, NC)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_output_gradient_directional_derivative():
    """dL/do against a directional finite difference in output space."""
    theta, X, r, Br, e = _sample(2)
    n_out = 1 + 2 * NC * 4
    o, _ = mlp.forward(theta, X, N_IN, WIDTH, n_out)
    L, dout = mlp.loss_and_dout(o, r, Br, e, 0.8, NC)
    dirn = np.random.default_rng(3).standard_normal(o.shape)
    eps = 1e-6
    fd = (mlp.loss_and_dout(o + eps * dirn, r, Br, e, 0.8, NC)[0]
          - mlp.loss_and_dout(o - eps * dirn, r, Br, e, 0.8, NC)[0]) / (2 * eps)
    assert abs(fd - np.sum(dout * dirn)) <= 1e-7 * abs(fd)


def test_zero_head_is_plain_smoother():
    theta = mlp.init(N_IN, WIDTH, NC)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((5, N_IN))
    o, _ = mlp.forward(theta, X, N_IN, WIDTH, 1 + 2 * NC * 4)
    w, U, V = mlp.head(o, NC)
    assert np.all(w == 1.0) and np.all(U == 0.0) and np.any(V != 0.0)
    # loss with exact local solve: pred = omega * Br
    r = rng.standard_normal((5, NC))
    Br = rng.standard_normal((5, NC))
    e = 0.8 * Br
    L, _ = mlp.loss_and_dout(o, r, Br, e, 0.8, NC)
    assert L == 0.0


def test_zero_head_vcycle_bitwise_equal():
    """Hierarchy with a learned correction of zero head equals the plain one bit for bit."""
    prob = workloads.problem("sphere96_q3")
    H = mg.Hierarchy(oracle_geometry(prob.geometry), 3, 6, 3)
    r = np.random.default_rng(5).standard_normal(H.fine.n_dofs)
    z0 = H.vcycle(r)
    nb = len(H.fine.boundary_cells)
    N = H.fine.N
    H.learned = (np.ones(nb), np.zeros((nb, N, 4)), np.random.default_rng(6).standard_normal((nb, N, 4)),
                 H.fine.boundary_cells)
    z1 = H.vcycle(r)
    assert np.array_equal(z0, z1)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(7)
    th = rng.standard_normal(20)
    g = rng.standard_normal(20)
    t1, m, v = mlp.adam(th, g, np.zeros(20), np.zeros(20), 1, lr=1e-2, eps=1e-12)
    assert np.allclose(t1, th - 1e-2 * np.sign(g), atol=1e-12)


def test_feature_layout():
    C, d, nq = 3, 3, 16
    rng = np.random.default_rng(8)
    sh = rng.uniform(-0.05, 0.05, (C, 2 * d, nq, d))
    mask = np.zeros((C, 2 * d))
    mask[:, 1] = 1
    sh[mask == 0] = 0
    nrm = rng.standard_normal((C, 2 * d, d))
    F = mlp.boundary_features(sh, mask, nrm, 0.1)
    assert F.shape == (C, 60)
    assert np.all(F[:, 0:10] == 0)       # face 0 (k = 0, s = 0) is interior
    assert np.all(F[:, 10] == 1)         # face 1 mask
    assert np.allclose(F[:, 11], sh[:, 1, :, 0].mean(1) / 0.1)   # mean d . n~ / h, outward +x
