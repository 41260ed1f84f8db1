"""Restarted flexible GMRES, right-preconditioned (oracle; test infrastructure only).

The paper solves its non-symmetric DG-SBM system with GMRES preconditioned by
one multigrid V-cycle per iteration and stops on the relative residual
(Sec. 3 opening, Sec. 5 opening).  The variant is not stated; this oracle takes
flexible GMRES(m) with right preconditioning, x0 = 0, modified Gram-Schmidt
Arnoldi and Givens rotations, and stops on the TRUE relative residual
||b - A x|| / ||b||, which is checked whenever the Arnoldi estimate reaches the
tolerance and at every restart.
"""
import numpy as np


def fgmres(A, M, b, tol=1e-8, restart=30, max_iter=1000):
    """Returns (x, iterations, true_relative_residual, converged, history)."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, 0.0, True, []
    its = 0
    hist = []
    r = b.copy()
    while True:
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        gvec = np.zeros(restart + 1)
        gvec[0] = beta
        j = 0
        while j < restart and its < max_iter:
            z = M(V[j])
            w = A(z)
            for i in range(j + 1):                 # modified Gram-Schmidt
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            Z.append(z)
            V.append(w / H[j + 1, j] if H[j + 1, j] != 0.0 else w)
            for i in range(j):                     # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            j += 1
            its += 1
            est = abs(gvec[j]) / nb
            hist.append(est)
            if est <= tol:
                break
        y = np.linalg.solve(np.triu(H[:j, :j]), gvec[:j])
        for i in range(j):
            x = x + y[i] * Z[i]
        r = b - A(x)
        rel = np.linalg.norm(r) / nb
        if rel <= tol:
            return x, its, rel, True, hist
        if its >= max_iter:
            return x, its, rel, False, hist
