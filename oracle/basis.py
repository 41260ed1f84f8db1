"""1D reference-element data on [0, 1] (oracle; test infrastructure only).

The paper discretises with a nodal Lagrange basis on tensor-product cells
(Sec. 2.2, closing paragraph).  The node set is not stated; this oracle uses the
Gauss-Lobatto-Legendre (GLL) points for every degree, which coincide with the
equispaced points for p <= 2.  The quadrature rule is not stated either; the
oracle uses (p+1)-point Gauss-Legendre per direction for the cell, the faces
and the right-hand side (exact for the degree-2p integrands of the unshifted
form), and p+3 points for the L2 error.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(p):
    """GLL nodes on [0,1]: the end points plus the roots of P_p' (Legendre)."""
    if p < 1:
        raise ValueError("p >= 1 required")
    c = np.zeros(p + 1)
    c[p] = 1.0
    interior = np.sort(np.real(npleg.legroots(npleg.legder(c)))) if p > 1 else np.array([])
    x = np.concatenate([[-1.0], interior, [1.0]])
    return 0.5 * (x + 1.0)


def gauss(nq):
    """nq-point Gauss-Legendre rule mapped to [0,1] (weights sum to 1)."""
    x, w = npleg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange(nodes, x):
    """Values and derivatives of the Lagrange polynomials through `nodes` at x.

    Returns (V, D) with V[m, a] = l_a(x_m) and D[m, a] = l_a'(x_m), computed
    from the product formula l_a(x) = prod_{b != a} (x - x_b) / (x_a - x_b).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    D = np.zeros((len(x), n))
    for a in range(n):
        den = 1.0
        for b in range(n):
            if b != a:
                den *= nodes[a] - nodes[b]
        for b in range(n):
            if b == a:
                continue
            V[:, a] *= x - nodes[b]
            term = np.ones(len(x))
            for c in range(n):
                if c != a and c != b:
                    term *= x - nodes[c]
            D[:, a] += term
        V[:, a] /= den
        D[:, a] /= den
    return V, D


def multi_indices(n1, d):
    """All d-tuples in [0, n1)^d, first component fastest (x fastest)."""
    idx = np.indices((n1,) * d).reshape(d, -1).T  # last axis fastest
    return idx[:, ::-1].copy()  # reverse so component 0 (x) is fastest


def tabulate(p, pts):
    """Tensor-product basis values and reference gradients at points of [0,1]^d.

    pts: (Q, d) reference coordinates.  Returns (Phi, G) with Phi[q, i] the value
    of basis function i (lexicographic, x fastest) at point q and G[q, i, c] its
    derivative in reference direction c.
    """
    pts = np.atleast_2d(pts)
    Q, d = pts.shape
    nodes = gll_nodes(p)
    mi = multi_indices(p + 1, d)  # (N, d)
    vals = []
    ders = []
    for c in range(d):
        V, D = lagrange(nodes, pts[:, c])
        vals.append(V)
        ders.append(D)
    N = mi.shape[0]
    Phi = np.ones((Q, N))
    for c in range(d):
        Phi *= vals[c][:, mi[:, c]]
    G = np.ones((Q, N, d))
    for c in range(d):
        for cc in range(d):
            G[:, :, c] *= (ders[cc] if cc == c else vals[cc])[:, mi[:, cc]]
    return Phi, G


def volume_points(nq, d):
    """Tensor Gauss points/weights on [0,1]^d, x fastest."""
    x, w = gauss(nq)
    mi = multi_indices(nq, d)
    pts = x[mi]
    wts = np.prod(w[mi], axis=1)
    return pts, wts


def face_points(nq, d, k, s):
    """Tensor Gauss points on the reference face {xi_k = s}, s in {0,1}.

    The tangential directions are the remaining ones in increasing order, the
    first remaining direction fastest.  Returns (pts (Q,d), weights (Q,)).
    """
    x, w = gauss(nq)
    if d == 1:
        pts = np.array([[float(s)]])
        return pts, np.array([1.0])
    mi = multi_indices(nq, d - 1)
    tang = [c for c in range(d) if c != k]
    pts = np.zeros((mi.shape[0], d))
    for j, c in enumerate(tang):
        pts[:, c] = x[mi[:, j]]
    pts[:, k] = float(s)
    wts = np.prod(w[mi], axis=1)
    return pts, wts
