"""Maps the shared workload geometries onto the oracle's geometry classes."""
import numpy as np

from oracle import geometry


def oracle_geometry(g):
    if g.kind == "balls":
        return geometry.Balls(g.centers, g.radii)
    if g.kind == "ellipsoid":
        c, a, R = g.centers[0], g.radii, g.rotation
        Ainv2 = R @ np.diag(1.0 / a ** 2) @ R.T          # phi = (x-c)^T Ainv2 (x-c) - 1

        def phi(X):
            Y = X - c
            return np.einsum('ni,ij,nj->n', Y, Ainv2, Y) - 1.0

        def grad(X):
            return 2.0 * (X - c) @ Ainv2

        def hess(X):
            return np.broadcast_to(2.0 * Ainv2, (X.shape[0], 3, 3))
        return geometry.LevelSet(phi, grad, hess, 3)
    if g.kind == "callback":
        return geometry.LevelSet(g.phi, g.grad, g.hess, g.dim)
    return geometry.Star2D(g.star_r0, g.star_a, g.star_k)
