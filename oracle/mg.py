"""hp-multigrid V-cycle with the cell-wise red-black SSOR smoother (oracle).

Test infrastructure only.  Follows Sec. 3 of the paper:
  * hierarchy (Sec. 3 opening): the finest mesh carries p, p-1, ..., 1, then
    the mesh is coarsened with p = 1; every level has its own active set,
    surrogate faces, shifts and re-discretised operator (Sec. 4.3);
  * smoother (Sec. 3.1): successive subspace correction over the cell
    subspaces, u <- u + omega R_i^T A_i^{-1} R_i (f - A u), with A_i the
    diagonal cell block, used as a symmetric (SSOR) sweep;
  * transfers (Sec. 3.2): prolongation = embedding on the background mesh
    (fine nodes take the coarse polynomial's value), restriction = transpose.

Readings (listed in the design notes):
  * coarsening: halve n while n is even, n/2 >= coarse_min (3) and the level
    still has more than coarse_dofs (2048) active DoFs (the coarse solver and
    coarsest mesh are not specified for the experiments);
  * the smoother visits the two colours (i+j+k mod 2) in the order 0,1,1,0 per
    step; cells of one colour do not couple, so a colour is updated at once;
  * omega = 1 for p <= 2 and 0.8 for p = 3 on every level;
  * V(1,1), a pre-smoothing step starting from zero;
  * inactive DoFs are identically zero: restriction into an inactive coarse
    cell is dropped, prolongation from an inactive parent gives zero;
  * coarse solver: a direct solve with the dense matrix of the coarsest level;
  * min_neighbours (the k-core rule of the active set) shapes the finest mesh
    only; the h-coarsened levels keep the plain active-cell rule;
  * smoother = 1: the additive variant of Sec. 3.1 (block Jacobi) inside a
    Chebyshev iteration (Sec. 5.3 mentions both): the interval of B A is
    [lmax / cheb_range, lmax], lmax = 1.2 x the dominant eigenvalue modulus
    from 25 power iterations started at the all-ones vector (range 20, degree
    3 by default: the values the interval is taken with are a reading).
"""
import numpy as np
import scipy.sparse as sp

from . import basis, dg


def level_shapes(n, p, coarse_min=3):
    """(n, p) of every level by the mesh rule alone, finest first."""
    out = [(n, q) for q in range(p, 0, -1)]
    while n % 2 == 0 and n // 2 >= coarse_min:
        n //= 2
        out.append((n, 1))
    return out


def default_omega(p):
    return 0.8 if p >= 3 else 1.0


def cell_inverses(L, D, stab=0.0):
    """Smoother inverses of the cell blocks D (k, N, N) of level L.

    B_K = D_K^{-1} by LU with partial pivoting (LAPACK getrf/getri).
    stab > 0: the stabilisation of near-singular cell blocks that Sec. 3.1
    calls for (reading: a singular-value floor).  With D_K = U S V^T and the
    floor f = stab * (smallest singular value of the level's interior block),
    B_K = V diag(1 / max(s_i, f)) U^T; blocks whose singular values all reach
    f keep the exact inverse."""
    B = np.linalg.inv(D)
    if stab > 0.0 and len(D):
        floor = stab * np.linalg.svd(L.interior_block(), compute_uv=False)[-1]
        U, s, Vt = np.linalg.svd(D)
        low = s[:, -1] < floor
        B[low] = np.einsum('kji,kj,klj->kil', Vt[low], 1.0 / np.maximum(s[low], floor), U[low])
    return B


class Hierarchy:
    """Levels coarsest first.  Geometric coarsening (p = 1) continues while n is
    even, n/2 >= coarse_min and the current level has more than coarse_dofs
    active DoFs; the last level is solved exactly."""

    def __init__(self, geom, d, n, p, coarse_min=3, coarse_dofs=2048, omega=None, nu_pre=1, nu_post=1,
                 stab=0.0, smoother=0, cheb_degree=3, cheb_range=20.0, **kw):
        fine_first = [dg.Level(geom, d, n, q, **kw) for q in range(p, 0, -1)]
        ckw = {k: v for k, v in kw.items() if k != "min_neighbours"}   # finest mesh only
        nn = n
        while nn % 2 == 0 and nn // 2 >= coarse_min and fine_first[-1].n_dofs > coarse_dofs:
            nn //= 2
            fine_first.append(dg.Level(geom, d, nn, 1, **ckw))
        self.levels = fine_first[::-1]
        self.d = d
        self.omega = default_omega(p) if omega is None else float(omega)
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.stab = float(stab)
        self.inv = [self._block_inverses(L, self.stab) for L in self.levels]
        self.P = [None] + [self._prolongation(self.levels[l - 1], self.levels[l])
                           for l in range(1, len(self.levels))]
        A0 = self.levels[0].A.toarray()
        self.A0inv = np.linalg.inv(A0) if A0.size else A0
        self.learned = None   # optional (omega_K, U_K, V_K) on the finest level
        self.smoother, self.cheb_degree, self.cheb_range = int(smoother), int(cheb_degree), float(cheb_range)
        self.cheb_lmax = [None] + [self._largest_eigenvalue(l) for l in range(1, len(self.levels))] \
            if self.smoother == 1 else None

    @staticmethod
    def _block_inverses(L, stab=0.0):
        if L.n_act == 0:
            return np.zeros((0, L.N, L.N))
        return cell_inverses(L, L.D, stab)

    @staticmethod
    def _prolongation(Lc, Lf):
        """Embedding of the coarse DG space into the fine one on the background mesh."""
        d = Lf.d
        nodes_f = basis.gll_nodes(Lf.p)
        mi_f = basis.multi_indices(Lf.p + 1, d)
        ref_f = nodes_f[mi_f]                                   # fine nodes, fine reference coords
        rows, cols, vals = [], [], []
        ratio = Lf.n // Lc.n                                    # 1 (p-level) or 2 (h-level)
        for K in range(Lf.n_act):
            mi = Lf.cells[K]
            parent = mi // ratio
            pc = Lc.cell_of[Lc.lin_index(parent)[0]]
            if pc < 0:
                continue
            off = mi - parent * ratio
            xc = (off[None, :] + ref_f) / ratio                 # fine nodes in coarse reference coords
            Phi, _ = basis.tabulate(Lc.p, xc)                    # (Nf, Nc)
            r = K * Lf.N + np.arange(Lf.N)
            c = pc * Lc.N + np.arange(Lc.N)
            rows.append(np.repeat(r, Lc.N))
            cols.append(np.tile(c, Lf.N))
            vals.append(Phi.reshape(-1))
        if not rows:
            return sp.csr_matrix((Lf.n_dofs, Lc.n_dofs))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(Lf.n_dofs, Lc.n_dofs))

    # ------------------------------------------------------------ smoother
    def colour_update(self, l, z, b, c):
        """z_K += omega B_K (b - A z)_K for every active cell K of colour c."""
        L = self.levels[l]
        r = (b - L.A @ z).reshape(L.n_act, L.N)
        zz = z.reshape(L.n_act, L.N)
        cells = np.arange(L.n_col0) if c == 0 else np.arange(L.n_col0, L.n_act)
        corr = self.omega * np.einsum('kij,kj->ki', self.inv[l][cells], r[cells])
        if self.learned is not None and l == len(self.levels) - 1:
            w, U, V, idx = self.learned                     # per boundary cell of the finest level
            pos = -np.ones(L.n_act, dtype=np.int64)
            pos[idx] = np.arange(len(idx))
            sel = pos[cells] >= 0
            kk = cells[sel]
            j = pos[kk]
            Br = np.einsum('kij,kj->ki', self.inv[l][kk], r[kk])
            UVr = np.einsum('kia,kja,kj->ki', U[j], V[j], r[kk])
            corr[sel] = (self.omega * w[j])[:, None] * (Br + UVr)
        zz[cells] += corr
        return z

    def ssor_step(self, l, z, b):
        for c in (0, 1, 1, 0):
            z = self.colour_update(l, z, b, c)
        return z

    # ------------------------------------------ additive smoother + Chebyshev
    def block_jacobi(self, l, r):
        """B r: every cell's inverse on its residual at once (Sec. 3.1,
        additive subspace correction without the weight)."""
        L = self.levels[l]
        return np.einsum('kij,kj->ki', self.inv[l], r.reshape(L.n_act, L.N)).ravel()

    def _largest_eigenvalue(self, l):
        """1.2 x the modulus of the dominant eigenvalue of B A, by 25 power
        iterations from the normalised all-ones vector."""
        L = self.levels[l]
        v = np.full(L.n_dofs, 1.0 / np.sqrt(L.n_dofs))
        lam = 0.0
        for _ in range(25):
            t = self.block_jacobi(l, L.A @ v)
            lam = np.linalg.norm(t)
            v = t / lam
        return 1.2 * lam

    def chebyshev_step(self, l, z, b):
        """cheb_degree additive block-Jacobi updates with Chebyshev weights
        for the interval [lmax / range, lmax] of B A (Sec. 5.3: the additive
        smoother wrapped in a Chebyshev iteration): the Chebyshev iteration for
        A x = b preconditioned by B, started from z."""
        lmax = self.cheb_lmax[l]
        lmin = lmax / self.cheb_range
        theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
        sigma = theta / delta
        L = self.levels[l]
        d = self.block_jacobi(l, b - L.A @ z) / theta
        z = z + d
        rho_old = 1.0 / sigma
        for _ in range(1, self.cheb_degree):
            rho = 1.0 / (2.0 * sigma - rho_old)
            d = rho * rho_old * d + 2.0 * rho / delta * self.block_jacobi(l, b - L.A @ z)
            z = z + d
            rho_old = rho
        return z

    def smoothing_step(self, l, z, b):
        return self.chebyshev_step(l, z, b) if self.smoother == 1 else self.ssor_step(l, z, b)

    # ------------------------------------------------------------ V-cycle
    def vcycle(self, b, l=None):
        if l is None:
            l = len(self.levels) - 1
        if l == 0:
            return self.A0inv @ b if b.size else b.copy()
        L = self.levels[l]
        z = np.zeros_like(b)
        for _ in range(self.nu_pre):
            z = self.smoothing_step(l, z, b)
        r = b - L.A @ z
        zc = self.vcycle(self.P[l].T @ r, l - 1)
        z = z + self.P[l] @ zc
        for _ in range(self.nu_post):
            z = self.smoothing_step(l, z, b)
        return z

    @property
    def fine(self):
        return self.levels[-1]
