"""DG-SBM discrete operator by direct quadrature (oracle; test infrastructure only).

Follows the paper's Sec. 2 (weak form with the extension operator, SIPG form,
full DG-SBM bilinear form and right-hand side) on a Cartesian background mesh.

Readings of the paper used here (each is listed in the design notes):
  * extension operator (ext = 0) E u = u + d . grad u: the
    printed definition carries the opposite sign, but only this sign gives the
    stated consistency E u*(x~) = u*(x~ + d) = g; the linear patch test pins
    it.  First-order Taylor limits the L2 rate to about h^2 for p >= 2, while
    Fig. 5 shows h^(p+1); ext = 1 evaluates the cell polynomial at x~ + d
    (Taylor to all orders), which restores h^(p+1) and coincides with ext = 0
    on linear functions;
  * sigma_F = c_F (p+1)^2 / h and sigma_Gamma = c_G (p+1)^2 / h, c_F = 2, c_G = 5;
  * a background cell is active iff phi(cell centre) < 0 (a cheap surrogate of
    the volume-fraction rule of Sec. 2.1), on every level; or, with
    lambda_frac > 0, iff its volume fraction inside Omega exceeds lambda, the
    fraction taken by the midpoint rule on frac_m^d equal sub-cells (Sec. 4.1
    uses cut-cell quadrature);
  * penalty_p > 0: the penalties use that degree on every level (one constant
    across the p-levels of a hierarchy) instead of the level's own degree;
  * min_neighbours = k > 0: the active set is then reduced to its k-core (cells
    with fewer than k active face neighbours dropped until none is left);
  * the trial function carries the shift in the Nitsche terms, the test
    function does not (quasi-symmetric form, alpha = 1);
  * quadrature: (p+1)^d Gauss points per cell, (p+1)^(d-1) per face.

Layout: active cells are ordered colour 0 first, then colour 1, colour =
(i+j+k) mod 2, each colour lexicographic with i fastest; inside a cell the
(p+1)^d GLL nodes are lexicographic with x fastest.
"""
import numpy as np
import scipy.sparse as sp

from . import basis


class Level:
    """One mesh level: active cells, faces, shifts and the DG-SBM matrix."""

    def __init__(self, geom, d, n, p, lo=-1.0, hi=1.0, c_F=2.0, c_G=5.0, alpha=1.0,
                 ext=1, zero_shift=False, shifts=None, build_matrix=True,
                 penalty_p=0, lambda_frac=0.0, frac_m=16, min_neighbours=0):
        if ext not in (0, 1):
            raise ValueError("ext must be 0 (first-order Taylor) or 1 (polynomial extrapolation)")
        self.geom, self.d, self.n, self.p = geom, d, n, p
        self.ext = ext
        self.lo, self.hi = float(lo), float(hi)
        self.h = (self.hi - self.lo) / n
        self.alpha = float(alpha)
        # penalty degree: the level's own p, or one degree for the whole hierarchy
        q = penalty_p if penalty_p > 0 else p
        self.sigma_F = c_F * (q + 1) ** 2 / self.h
        self.sigma_G = c_G * (q + 1) ** 2 / self.h
        self.lambda_frac, self.frac_m = float(lambda_frac), int(frac_m)
        self.min_neighbours = int(min_neighbours)
        self.N = (p + 1) ** d
        self._classify()
        self._faces()
        if shifts is not None:
            self.shifts = np.asarray(shifts, dtype=np.float64).reshape(self.face_points.shape)
        elif zero_shift:
            self.shifts = np.zeros_like(self.face_points)
        else:
            self._compute_shifts()
        if build_matrix:
            self.assemble()

    # ---------------------------------------------------------------- mesh
    def volume_fractions(self, idx):
        """Share of the frac_m^d midpoints of equal sub-cells of each cell that
        lie in Omega (phi < 0): the midpoint-rule value of the volume fraction
        that the active-cell rule of Sec. 2.1 thresholds."""
        d, h, m = self.d, self.h, self.frac_m
        sub = (basis.multi_indices(m, d) + 0.5) / m
        out = np.zeros(len(idx))
        todo = np.arange(len(idx))
        if getattr(self.geom, "lipschitz", False) and len(idx):
            # |phi| is at most the distance to Gamma: a cell whose centre is
            # farther than half its diagonal from Gamma lies on one side
            pc = self.geom.phi(self.lo + h * (idx + 0.5))
            far = np.abs(pc) > 0.5 * np.sqrt(d) * h * (1 + 1e-12)
            out[far] = (pc[far] < 0.0).astype(float)
            todo = np.nonzero(~far)[0]
        for a in range(0, len(todo), 256):
            cc = todo[a:a + 256]
            X = (self.lo + h * idx[cc])[:, None, :] + h * sub[None]
            out[cc] = (self.geom.phi(X.reshape(-1, d)).reshape(-1, len(sub)) < 0.0).mean(axis=1)
        return out

    def _classify(self):
        d, n, h = self.d, self.n, self.h
        idx = basis.multi_indices(n, d)          # every background cell, x fastest
        lin = np.arange(idx.shape[0])            # = i + n j + n^2 k
        centres = self.lo + h * (idx + 0.5)
        if self.lambda_frac > 0.0:
            # Sec. 2.1: active iff the volume fraction inside Omega exceeds
            # lambda (lambda = 1: the whole cell)
            frac = self.volume_fractions(idx)
            active = frac >= 1.0 if self.lambda_frac >= 1.0 else frac > self.lambda_frac
        else:
            active = self.geom.phi(centres) < 0.0 if idx.shape[0] else np.zeros(0, bool)
        if self.min_neighbours > 0:
            active = self._k_core(active, self.min_neighbours)
        colour = idx.sum(axis=1) % 2
        sel = np.nonzero(active)[0]
        order = sel[np.lexsort((lin[sel], colour[sel]))]
        self.cells = idx[order]                  # (n_act, d) multi-indices in DoF order
        self.colour = colour[order]
        self.n_act = len(order)
        self.n_col0 = int(np.sum(self.colour == 0))
        self.cell_of = -np.ones(n ** d, dtype=np.int64)
        self.cell_of[order] = np.arange(self.n_act)
        self.n_dofs = self.n_act * self.N

    def _k_core(self, active, k):
        """Largest subset of the active cells in which every cell has at least
        k active face neighbours (cells below k dropped until none is left)."""
        d, n = self.d, self.n
        act = active.reshape((n,) * d).copy()              # axis 0 = last coordinate
        while True:
            cnt = np.zeros(act.shape, dtype=int)
            for ax in range(d):
                pad = [(0, 0)] * d
                pad[ax] = (1, 1)
                p = np.pad(act, pad)
                lo = [slice(None)] * d
                hi = [slice(None)] * d
                lo[ax] = slice(0, n)
                hi[ax] = slice(2, n + 2)
                cnt += p[tuple(lo)].astype(int) + p[tuple(hi)].astype(int)
            drop = act & (cnt < k)
            if not drop.any():
                return act.reshape(-1)
            act &= ~drop

    def lin_index(self, mi):
        mi = np.atleast_2d(mi)
        w = self.n ** np.arange(self.d)
        return mi @ w

    def neighbour(self, cells, k, s):
        """Active index of the neighbour across face (k, s) or -1."""
        mi = self.cells[cells].copy()
        mi[:, k] += 2 * s - 1
        inside = (mi[:, k] >= 0) & (mi[:, k] < self.n)
        out = -np.ones(len(cells), dtype=np.int64)
        out[inside] = self.cell_of[self.lin_index(mi[inside])]
        return out

    def _faces(self):
        d = self.d
        allc = np.arange(self.n_act)
        self.nbr = np.zeros((self.n_act, 2 * d), dtype=np.int64)
        for k in range(d):
            for s in (0, 1):
                self.nbr[:, 2 * k + s] = self.neighbour(allc, k, s)
        # interior faces, recorded once from the lower cell: (minus, plus, k)
        self.int_faces = []
        for k in range(d):
            nb = self.nbr[:, 2 * k + 1]
            m = np.nonzero(nb >= 0)[0]
            self.int_faces.append((m, nb[m]))
        # surrogate faces, ordered by (cell, k, s)
        cell, kk, ss = np.nonzero(self.nbr.reshape(self.n_act, d, 2) < 0)
        self.surr_cell, self.surr_k, self.surr_s = cell, kk, ss
        self.n_surr = len(cell)
        nq = self.p + 1
        nf = nq ** (d - 1)
        self.face_points = np.zeros((self.n_surr, nf, d))
        for k in range(d):
            for s in (0, 1):
                sel = np.nonzero((kk == k) & (ss == s))[0]
                if len(sel) == 0:
                    continue
                pts, _ = basis.face_points(nq, d, k, s)
                origin = self.lo + self.h * self.cells[cell[sel]]
                self.face_points[sel] = origin[:, None, :] + self.h * pts[None]
        self.boundary_cells = np.unique(cell)

    def _compute_shifts(self):
        flat = self.face_points.reshape(-1, self.d)
        if flat.shape[0] == 0:
            self.shifts = np.zeros_like(self.face_points)
            return
        cp = self.geom.closest(flat)
        self.shifts = (cp - flat).reshape(self.face_points.shape)

    # ---------------------------------------------------------------- blocks
    def volume_block(self):
        """int_K grad phi_j . grad phi_i (Sec. 2.2, volume term of a_h)."""
        d, p, h = self.d, self.p, self.h
        pts, w = basis.volume_points(p + 1, d)
        _, G = basis.tabulate(p, pts)
        return h ** d * np.einsum('q,qic,qjc->ij', w, G / h, G / h)

    def interior_block(self):
        """Diagonal block of a cell whose 2d neighbours are all active: the
        volume term plus both sides' self terms of its 2d SIPG faces."""
        D = self.volume_block()
        for k in range(self.d):
            B = self.interior_face_blocks(k)
            D = D + B[0][0] + B[1][1]
        return D

    def interior_face_blocks(self, k):
        """SIPG face terms on a face normal to e_k (Sec. 2.2, SIPG bilinear form).

        Returns blocks[a][b] (a = test side, b = trial side; 0 = minus, the cell
        with the lower coordinate, 1 = plus), with [w] = (w- - w+) e_k and
        {dw/dx_k} = (dw-/dx_k + dw+/dx_k) / 2.
        """
        d, p, h = self.d, self.p, self.h
        pm, w = basis.face_points(p + 1, d, k, 1)
        pp, _ = basis.face_points(p + 1, d, k, 0)
        Phi = [None, None]
        Dk = [None, None]
        Phi[0], G0 = basis.tabulate(p, pm)
        Phi[1], G1 = basis.tabulate(p, pp)
        Dk[0], Dk[1] = G0[:, :, k] / h, G1[:, :, k] / h
        js = (1.0, -1.0)
        area = h ** (d - 1)
        blocks = [[None, None], [None, None]]
        for a in (0, 1):
            for b in (0, 1):
                # v = phi_i on side a, u = phi_j on side b
                t = (-0.5 * js[a] * np.einsum('q,qj,qi->ij', w, Dk[b], Phi[a])
                     - 0.5 * js[b] * np.einsum('q,qi,qj->ij', w, Dk[a], Phi[b])
                     + self.sigma_F * js[a] * js[b] * np.einsum('q,qi,qj->ij', w, Phi[a], Phi[b]))
                blocks[a][b] = area * t
        return blocks

    def extension(self, k, s, faces):
        """E phi_j at the Gauss points of the given surrogate faces, (f, q, j).

        ext = 0: first-order Taylor extension E u = u + d . grad u (Sec. 2.1,
                 sign fixed by the stated consistency E u* (x~) = u*(x~ + d));
        ext = 1: the cell polynomial evaluated at the true-boundary point,
                 E u(x~) = u|_K(x~ + d), i.e. the Taylor series of the cell
                 polynomial summed to all orders.
        """
        d, p, h = self.d, self.p, self.h
        pts, _ = basis.face_points(p + 1, d, k, s)
        dq = self.shifts[faces]                              # (f, q, d) physical
        if self.ext == 0:
            Phi, G = basis.tabulate(p, pts)
            return Phi[None] + np.einsum('fqc,qjc->fqj', dq, G / h)
        out = np.empty((len(faces), len(pts), self.N))
        for a in range(len(faces)):
            out[a], _ = basis.tabulate(p, pts + dq[a] / h)
        return out

    def surrogate_blocks(self, faces=None):
        """Nitsche-SBM terms on surrogate faces (Sec. 2.1 weak form, Sec. 2.2).

        For test phi_i, trial phi_j at the face Gauss points x~_q with outward
        normal n~ and shift d_q:
          -(grad phi_j . n~) phi_i - alpha (grad phi_i . n~) E phi_j
          + sigma_Gamma E phi_j phi_i       (E: see `extension`).
        Returns (n_faces, N, N).
        """
        d, p, h = self.d, self.p, self.h
        if faces is None:
            faces = np.arange(self.n_surr)
        out = np.zeros((len(faces), self.N, self.N))
        area = h ** (d - 1)
        for k in range(d):
            for s in (0, 1):
                sel = np.nonzero((self.surr_k[faces] == k) & (self.surr_s[faces] == s))[0]
                if len(sel) == 0:
                    continue
                pts, w = basis.face_points(p + 1, d, k, s)
                Phi, G = basis.tabulate(p, pts)
                G = G / h
                ns = 2.0 * s - 1.0
                dn = G[:, :, k] * ns                      # (q, i) outward normal derivative
                Eu = self.extension(k, s, faces[sel])     # (f, q, j)
                t = (-np.einsum('q,qj,qi->ij', w, dn, Phi)[None]
                     - self.alpha * np.einsum('q,qi,fqj->fij', w, dn, Eu)
                     + self.sigma_G * np.einsum('q,fqj,qi->fij', w, Eu, Phi))
                out[sel] = area * t
        return out

    def assemble(self):
        """Global matrix (active DoFs only) as a block-sparse matrix."""
        N = self.N
        D = np.broadcast_to(self.volume_block(), (self.n_act, N, N)).copy()
        rows, cols, data = [], [], []
        self.coupling = []
        for k in range(self.d):
            m, pl = self.int_faces[k]
            B = self.interior_face_blocks(k)
            self.coupling.append(B)
            np.add.at(D, m, B[0][0])
            np.add.at(D, pl, B[1][1])
            rows += [m, pl]
            cols += [pl, m]
            data += [np.broadcast_to(B[0][1], (len(m), N, N)), np.broadcast_to(B[1][0], (len(m), N, N))]
        if self.n_surr:
            np.add.at(D, self.surr_cell, self.surrogate_blocks())
        self.D = D
        rows = np.concatenate(rows + [np.arange(self.n_act)]) if self.n_act else np.zeros(0, int)
        cols = np.concatenate(cols + [np.arange(self.n_act)]) if self.n_act else np.zeros(0, int)
        data = np.concatenate(data + [D], axis=0) if self.n_act else np.zeros((0, N, N))
        order = np.lexsort((cols, rows))
        rows, cols, data = rows[order], cols[order], data[order]
        indptr = np.zeros(self.n_act + 1, dtype=np.int64)
        np.add.at(indptr, rows + 1, 1)
        indptr = np.cumsum(indptr)
        self.A = sp.bsr_matrix((data, cols, indptr), shape=(self.n_dofs, self.n_dofs))

    def apply(self, x):
        return self.A @ x

    def _cell_blocks(self, K, X, V, Bf):
        """Diagonal block D_K and the neighbour part sum_F B_{K,nb} x_nb of cell
        K's rows, from the same element blocks as `assemble` (Sec. 2.2):
        volume, the SIPG blocks of each interior face (K is the minus side,
        index 0, when its neighbour lies at the higher coordinate), and the
        Nitsche-SBM blocks of its surrogate faces."""
        D = V.copy()
        off = np.zeros(self.N)
        for k in range(self.d):
            B = Bf[k]
            for s in (0, 1):
                nb = self.nbr[K, 2 * k + s]
                if nb >= 0:
                    me = 0 if s == 1 else 1
                    D += B[me][me]
                    if X is not None:
                        off += B[me][1 - me] @ X[nb]
        faces = np.nonzero(self.surr_cell == K)[0]
        if len(faces):
            D += self.surrogate_blocks(faces).sum(axis=0)
        return D, off

    def cell_apply(self, cells, x):
        """(A x)_K for the given active cells, one cell at a time without the
        global matrix (for sampled checks at sizes where A is too large)."""
        X = np.asarray(x, dtype=np.float64).reshape(self.n_act, self.N)
        out = np.zeros((len(cells), self.N))
        V, Bf = self.volume_block(), [self.interior_face_blocks(k) for k in range(self.d)]
        for a, K in enumerate(cells):
            D, off = self._cell_blocks(int(K), X, V, Bf)
            out[a] = D @ X[K] + off
        return out

    def cell_diag_blocks(self, cells):
        """D_K for the given active cells (the blocks the smoother inverts)."""
        if len(cells) == 0:
            return np.zeros((0, self.N, self.N))
        V, Bf = self.volume_block(), [self.interior_face_blocks(k) for k in range(self.d)]
        return np.stack([self._cell_blocks(int(K), None, V, Bf)[0] for K in cells])

    # ---------------------------------------------------------------- data
    def rhs(self, f, g):
        """Right-hand side of the DG-SBM system (Sec. 2.2):
        int_K f phi_i + sum_q w_q [-alpha grad phi_i . n~ + sigma_Gamma phi_i] g(x~_q + d_q)."""
        d, p, h = self.d, self.p, self.h
        pts, w = basis.volume_points(p + 1, d)
        Phi, _ = basis.tabulate(p, pts)
        b = np.zeros((self.n_act, self.N))
        if self.n_act:
            X = (self.lo + h * self.cells)[:, None, :] + h * pts[None]
            fv = f(X.reshape(-1, d)).reshape(self.n_act, -1)
            b += h ** d * np.einsum('q,kq,qi->ki', w, fv, Phi)
        area = h ** (d - 1)
        for k in range(d):
            for s in (0, 1):
                sel = np.nonzero((self.surr_k == k) & (self.surr_s == s))[0]
                if len(sel) == 0:
                    continue
                fp, wf = basis.face_points(p + 1, d, k, s)
                Phf, Gf = basis.tabulate(p, fp)
                dn = Gf[:, :, k] * (2.0 * s - 1.0) / h
                Y = self.face_points[sel] + self.shifts[sel]
                gv = g(Y.reshape(-1, d)).reshape(len(sel), -1)
                contrib = area * np.einsum('q,fq,qi->fi', wf, gv, -self.alpha * dn + self.sigma_G * Phf)
                np.add.at(b, self.surr_cell[sel], contrib)
        return b.reshape(-1)

    def interpolate(self, u):
        """Nodal interpolant of u on the active cells."""
        nodes = basis.gll_nodes(self.p)
        mi = basis.multi_indices(self.p + 1, self.d)
        X = (self.lo + self.h * self.cells)[:, None, :] + self.h * nodes[mi][None]
        return u(X.reshape(-1, self.d))

    def l2_error(self, uh, u):
        """|| u - u_h ||_{L2(surrogate domain)} with (p+3)^d Gauss points."""
        d, p, h = self.d, self.p, self.h
        pts, w = basis.volume_points(p + 3, d)
        Phi, _ = basis.tabulate(p, pts)
        X = (self.lo + h * self.cells)[:, None, :] + h * pts[None]
        ue = u(X.reshape(-1, d)).reshape(self.n_act, -1)
        uhq = uh.reshape(self.n_act, self.N) @ Phi.T
        return np.sqrt(h ** d * np.sum(w[None] * (ue - uhq) ** 2))
