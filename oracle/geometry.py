"""Level sets and closest-point projections (oracle; test infrastructure only).

The domain is Omega = {phi < 0} and Gamma = {phi = 0} (Sec. 4.1).  Each
surrogate-boundary quadrature point x~ is mapped to its closest point x on
Gamma, and the shift is d = x - x~ (Sec. 2.1, definition of the extension
operator).  For balls and their unions the projection is computed exactly,
as the paper allows where that is possible (Sec. 4.2); for the 2D star it is a
1D minimisation over the curve parameter; for a general level set it is the
Newton iteration on the Lagrangian of the constrained distance problem
(Sec. 4.2, stationarity conditions of L(x, mu) = |x - x~|^2 + mu phi(x)).

Readings (where the paper is silent):
  * the closest point is the global one on Gamma, not a search restricted to
    the adjacent cells;
  * union of balls: the candidates are the radial projections onto each
    sphere, the nearest points of every pairwise intersection circle (2D: the
    two intersection points) and, in 3D, the triple intersection points; a
    candidate strictly inside another ball (by more than 1e-12) is dropped;
    the nearest remaining candidate wins, ties to the first in that order;
  * star r(theta) = r0 + a sin(k theta): 4096 equispaced samples of theta,
    the nearest sample (ties to the smallest theta) seeds a safeguarded
    Newton iteration on the derivative of the squared distance.
"""
import numpy as np

_INSIDE_TOL = 1e-12


class Balls:
    """Union of balls |x - c_j| < r_j (one ball = disk / sphere).  phi is the
    minimum of the balls' signed distances: 1-Lipschitz."""

    lipschitz = True

    def __init__(self, centers, radii):
        self.centers = np.atleast_2d(np.asarray(centers, dtype=np.float64))
        self.radii = np.atleast_1d(np.asarray(radii, dtype=np.float64))
        self.d = self.centers.shape[1]

    def phi(self, X):
        X = np.atleast_2d(X)
        dist = np.linalg.norm(X[:, None, :] - self.centers[None], axis=2)
        return np.min(dist - self.radii[None], axis=1)

    def grad_phi(self, X):
        """Gradient of the active (minimising) ball's distance function."""
        X = np.atleast_2d(X)
        dist = np.linalg.norm(X[:, None, :] - self.centers[None], axis=2)
        j = np.argmin(dist - self.radii[None], axis=1)
        v = X - self.centers[j]
        return v / np.linalg.norm(v, axis=1, keepdims=True)

    def _outside_others(self, Y, skip):
        """Mask of candidate points Y (M, d) not strictly inside a ball outside `skip`."""
        ok = np.ones(Y.shape[0], dtype=bool)
        for m in range(len(self.radii)):
            if m in skip:
                continue
            ok &= ~(np.linalg.norm(Y - self.centers[m], axis=1) < self.radii[m] - _INSIDE_TOL)
        return ok

    def closest(self, X):
        """Nearest point of Gamma for each row of X (candidate order: spheres,
        pairwise circles / points, triple points; ties go to the first)."""
        X = np.atleast_2d(np.asarray(X, dtype=np.float64))
        C, R, d = self.centers, self.radii, self.d
        M = X.shape[0]
        cands, valid = [], []
        for j in range(len(R)):
            v = X - C[j]
            nv = np.linalg.norm(v, axis=1)
            z = nv == 0.0
            v[z] = 0.0
            v[z, 0] = 1.0
            nv[z] = 1.0
            Y = C[j] + R[j] * v / nv[:, None]
            cands.append(Y)
            valid.append(self._outside_others(Y, (j,)))
        for j in range(len(R)):
            for k in range(j + 1, len(R)):
                L = np.linalg.norm(C[k] - C[j])
                if not (abs(R[j] - R[k]) < L < R[j] + R[k]):
                    continue
                e = (C[k] - C[j]) / L
                a = (L * L + R[j] ** 2 - R[k] ** 2) / (2.0 * L)
                rho = np.sqrt(max(R[j] ** 2 - a * a, 0.0))
                mc = C[j] + a * e
                if d == 2:
                    perp = np.array([-e[1], e[0]])
                    pts = [np.broadcast_to(mc + rho * perp, X.shape), np.broadcast_to(mc - rho * perp, X.shape)]
                else:
                    w = (X - mc) - ((X - mc) @ e)[:, None] * e
                    nw = np.linalg.norm(w, axis=1)
                    z = nw == 0.0
                    if np.any(z):
                        ax = np.argmin(np.abs(e))
                        t = np.zeros(3)
                        t[ax] = 1.0
                        t = t - np.dot(t, e) * e
                        w[z] = t
                        nw[z] = np.linalg.norm(t)
                    pts = [mc + rho * w / nw[:, None]]
                for Y in pts:
                    cands.append(np.array(Y))
                    valid.append(self._outside_others(Y, (j, k)))
        if d == 3:
            for j in range(len(R)):
                for k in range(j + 1, len(R)):
                    for l in range(k + 1, len(R)):
                        for y in _triple_points(C[j], R[j], C[k], R[k], C[l], R[l]):
                            Y = np.broadcast_to(y, X.shape)
                            cands.append(np.array(Y))
                            valid.append(self._outside_others(Y, (j, k, l)))
        P = np.stack(cands, axis=1)                  # (M, n_cand, d)
        ok = np.stack(valid, axis=1)
        dist = np.linalg.norm(P - X[:, None, :], axis=2)
        dist[~ok] = np.inf
        best = np.argmin(dist, axis=1)              # first minimum on ties
        return P[np.arange(M), best]


def _triple_points(c1, r1, c2, r2, c3, r3):
    """Points common to three spheres (0 or 2 points, 1 if tangent)."""
    # |y-ci|^2 = ri^2; subtracting the first from the others gives two planes.
    a2 = 2.0 * (c2 - c1)
    a3 = 2.0 * (c3 - c1)
    b2 = r1 ** 2 - r2 ** 2 + np.dot(c2, c2) - np.dot(c1, c1)
    b3 = r1 ** 2 - r3 ** 2 + np.dot(c3, c3) - np.dot(c1, c1)
    u = np.cross(a2, a3)
    nu = np.dot(u, u)
    if nu < 1e-30:
        return []
    # particular point on the line {a2.y=b2, a3.y=b3}, in the span of a2, a3
    y0 = (b2 * np.cross(a3, u) + b3 * np.cross(u, a2)) / nu
    uu = u / np.sqrt(nu)
    w = y0 - c1
    bq = np.dot(w, uu)
    cq = np.dot(w, w) - r1 ** 2
    disc = bq * bq - cq
    if disc < 0.0:
        return []
    s = np.sqrt(disc)
    return [y0 + (-bq - s) * uu, y0 + (-bq + s) * uu]


class Star2D:
    """2D star {|x| < r(theta)}, r(theta) = r0 + a sin(k theta)."""

    def __init__(self, r0, a, k):
        self.r0, self.a, self.k = float(r0), float(a), int(k)
        self.d = 2

    def radius(self, th):
        return self.r0 + self.a * np.sin(self.k * th)

    def phi(self, X):
        X = np.atleast_2d(X)
        th = np.arctan2(X[:, 1], X[:, 0])
        return np.linalg.norm(X, axis=1) - self.radius(th)

    def grad_phi(self, X):
        """Unit outward normal of the curve at the closest point of X."""
        X = np.atleast_2d(X)
        Y = self.closest(X)
        out = np.empty_like(Y)
        for i, y in enumerate(Y):
            th = np.arctan2(y[1], y[0])
            r = self.radius(th)
            dr = self.a * self.k * np.cos(self.k * th)
            # curve c(th) = r e_th ; tangent c' = dr e_th + r e_th'
            t = np.array([dr * np.cos(th) - r * np.sin(th), dr * np.sin(th) + r * np.cos(th)])
            n = np.array([t[1], -t[0]])
            out[i] = n / np.linalg.norm(n)
        return out

    def _F(self, x, th):
        """Squared distance F, and F', F'' with respect to theta."""
        a, k = self.a, self.k
        r = self.r0 + a * np.sin(k * th)
        r1 = a * k * np.cos(k * th)
        r2 = -a * k * k * np.sin(k * th)
        c, s = np.cos(th), np.sin(th)
        xe = x[0] * c + x[1] * s       # x . e_th
        xe1 = -x[0] * s + x[1] * c     # x . e_th'
        F = np.dot(x, x) - 2.0 * r * xe + r * r
        F1 = -2.0 * r1 * xe - 2.0 * r * xe1 + 2.0 * r * r1
        F2 = -2.0 * r2 * xe - 4.0 * r1 * xe1 + 2.0 * r * xe + 2.0 * r1 * r1 + 2.0 * r * r2
        return F, F1, F2

    def closest_theta(self, x, nsamp=4096):
        th = 2.0 * np.pi * np.arange(nsamp) / nsamp
        F, _, _ = self._F(x, th)
        m = int(np.argmin(F))
        dth = 2.0 * np.pi / nsamp
        lo, hi = th[m] - dth, th[m] + dth
        t = th[m]
        for _ in range(100):
            _, F1, F2 = self._F(x, t)
            if abs(F1) < 1e-15:
                break
            if F1 > 0.0:
                hi = t
            else:
                lo = t
            tn = t - F1 / F2 if F2 > 0.0 else 0.5 * (lo + hi)
            if not (lo < tn < hi):
                tn = 0.5 * (lo + hi)
            if tn == t or hi - lo < 1e-16:
                t = tn
                break
            t = tn
        return t

    def closest(self, X):
        X = np.atleast_2d(np.asarray(X, dtype=np.float64))
        Y = np.empty_like(X)
        for i, x in enumerate(X):
            t = self.closest_theta(x)
            r = self.radius(t)
            Y[i] = [r * np.cos(t), r * np.sin(t)]
        return Y


class LevelSet:
    """General level set given by phi, its gradient and Hessian (vectorised).

    The closest point solves the stationarity system of the Lagrangian
    L(x, mu) = |x - x~|^2 + mu phi(x) with Newton's method (Sec. 4.2).
    """

    def __init__(self, phi, grad, hess, d):
        self._phi, self._grad, self._hess, self.d = phi, grad, hess, d

    def phi(self, X):
        return self._phi(np.atleast_2d(X))

    def grad_phi(self, X):
        g = self._grad(np.atleast_2d(X))
        return g / np.linalg.norm(g, axis=1, keepdims=True)

    def closest(self, X, maxit=100):
        X = np.atleast_2d(np.asarray(X, dtype=np.float64))
        d = X.shape[1]
        Y = np.empty_like(X)
        for i, xt in enumerate(X):
            f = self._phi(xt[None])[0]
            g = self._grad(xt[None])[0]
            x = xt - f * g / np.dot(g, g)
            g = self._grad(x[None])[0]
            mu = -2.0 * np.dot(x - xt, g) / np.dot(g, g)
            for _ in range(maxit):
                f = self._phi(x[None])[0]
                g = self._grad(x[None])[0]
                H = self._hess(x[None])[0]
                res = np.concatenate([2.0 * (x - xt) + mu * g, [f]])
                if abs(f) < 1e-14 and np.linalg.norm(res[:d]) < 1e-13:
                    break
                J = np.zeros((d + 1, d + 1))
                J[:d, :d] = 2.0 * np.eye(d) + mu * H
                J[:d, d] = g
                J[d, :d] = g
                step = np.linalg.solve(J, -res)
                x = x + step[:d]
                mu = mu + step[d]
            Y[i] = x
        return Y
