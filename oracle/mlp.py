"""Reference of the learned boundary-cell smoother correction (oracle; test infrastructure only).

Not part of the paper.  The paper reports that the cell-wise smoother loses
effectiveness for p = 3 in 3D (Sec. 5.3) and leaves better smoothers to future
work (Sec. 6).  The correction here keeps the successive cell-wise update of
Sec. 3.1 and only modifies the local solve on cells next to the surrogate
boundary:

    z_K += omega * w_K * (B_K + U_K V_K^T) r_K,    w_K = 2 sigmoid(o_0)

with (o_0, U_K, V_K) the output of a small MLP on per-cell geometric features
(shift statistics per face).  A zero output head gives w_K = 1 and U_K = 0, i.e.
exactly the plain smoother.

Network: three dense layers, tanh after the first two.
    h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  o = W3 h2 + b3
Flat parameter layout: W1 (width x n_in, row-major), b1, W2 (width x width),
b2, W3 (n_out x width), b3;  n_out = 1 + 2 * N * rank, o = [o_0, U (N x rank,
row-major), V (N x rank, row-major)].

Loss over samples s (e = error, r = residual, Br = B_K r on the sample's cell):
    pred_s = omega * w * (Br + U (V^T r)),   L = mean_s |pred_s - e_s|^2 / |e_s|^2
"""
import numpy as np


def dims(n_in, width, n_cell, rank=4):
    return n_in, width, 1 + 2 * n_cell * rank


def n_params(n_in, width, n_out):
    return width * n_in + width + width * width + width + n_out * width + n_out


def unpack(theta, n_in, width, n_out):
    o = 0
    out = []
    for shape in ((width, n_in), (width,), (width, width), (width,), (n_out, width), (n_out,)):
        sz = int(np.prod(shape))
        out.append(theta[o:o + sz].reshape(shape))
        o += sz
    return out


def forward(theta, X, n_in, width, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, width, n_out)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    o = h2 @ W3.T + b3
    return o, (X, h1, h2)


def head(o, n_cell, rank=4):
    w = 2.0 / (1.0 + np.exp(-o[:, 0]))
    U = o[:, 1:1 + n_cell * rank].reshape(-1, n_cell, rank)
    V = o[:, 1 + n_cell * rank:].reshape(-1, n_cell, rank)
    return w, U, V


def loss_and_dout(o, r, Br, e, omega, n_cell, rank=4):
    """Loss and its gradient with respect to the network output o."""
    w, U, V = head(o, n_cell, rank)
    q = np.einsum('sja,sj->sa', V, r)
    P = Br + np.einsum('sia,sa->si', U, q)
    pred = omega * w[:, None] * P
    res = pred - e
    ne = np.sum(e * e, axis=1)
    # a sample with e = 0 has no relative error: it contributes zero
    inv = np.divide(1.0, ne, out=np.zeros_like(ne), where=ne > 0)
    S = o.shape[0]
    L = np.mean(np.sum(res * res, axis=1) * inv)
    g = 2.0 * res * inv[:, None] / S                     # dL/dpred
    sig = w / 2.0
    dw = omega * np.sum(g * P, axis=1)                   # dL/dw
    do0 = dw * 2.0 * sig * (1.0 - sig)
    dP = omega * w[:, None] * g
    dU = np.einsum('si,sa->sia', dP, q)
    dq = np.einsum('si,sia->sa', dP, U)
    dV = np.einsum('sa,sj->sja', dq, r)
    dout = np.concatenate([do0[:, None], dU.reshape(S, -1), dV.reshape(S, -1)], axis=1)
    return L, dout


def backward(theta, cache, dout, n_in, width, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, width, n_out)
    X, h1, h2 = cache
    gW3 = dout.T @ h2
    gb3 = dout.sum(0)
    d2 = (dout @ W3) * (1.0 - h2 * h2)
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * (1.0 - h1 * h1)
    gW1 = d1.T @ X
    gb1 = d1.sum(0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def loss_grad(theta, X, r, Br, e, omega, n_in, width, n_cell, rank=4):
    n_out = 1 + 2 * n_cell * rank
    o, cache = forward(theta, X, n_in, width, n_out)
    L, dout = loss_and_dout(o, r, Br, e, omega, n_cell, rank)
    return L, backward(theta, cache, dout, n_in, width, n_out)


def adam(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba), t = 1-based step count."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init(n_in, width, n_cell, rank=4, seed=0, scale_v=0.05):
    """Hidden layers ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)); output rows of o_0
    and U zero (plain smoother at start), rows of V small random so that the
    U-gradient is not identically zero."""
    n_out = 1 + 2 * n_cell * rank
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (width, n_in)) / np.sqrt(n_in)
    W2 = rng.uniform(-1, 1, (width, width)) / np.sqrt(width)
    W3 = np.zeros((n_out, width))
    W3[1 + n_cell * rank:] = rng.uniform(-1, 1, (n_cell * rank, width)) * scale_v / np.sqrt(width)
    b3 = np.zeros(n_out)
    return np.concatenate([W1.ravel(), np.zeros(width), W2.ravel(), np.zeros(width), W3.ravel(), b3])


def boundary_features(shifts_per_face, mask, normals_per_face, h):
    """Per boundary cell feature vector (60 values for d = 3).

    shifts_per_face: (cells, 2d, nq, d) physical shifts of the cell's surrogate
    faces (zeros where the face is interior); mask: (cells, 2d) 1 = surrogate;
    normals_per_face: (cells, 2d, d) mean unit normal of Gamma at the
    projections.  Per face, in face order (k, s): mask, mean / min / max of
    d . n~ / h, mean d / h (d values), mean true normal (d values).
    """
    C, F, Q, d = shifts_per_face.shape
    out = []
    for f in range(F):
        k, s = f // 2, f % 2
        sg = 1.0 if s == 1 else -1.0
        dn = shifts_per_face[:, f, :, k] * sg / h
        m = mask[:, f]
        out.append(m[:, None])
        out.append((np.stack([dn.mean(1), dn.min(1), dn.max(1)], 1)) * m[:, None])
        out.append(shifts_per_face[:, f].mean(1) / h * m[:, None])
        out.append(normals_per_face[:, f] * m[:, None])
    return np.concatenate(out, axis=1)
