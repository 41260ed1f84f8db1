"""Python handle over the C ABI: marshals torch tensors and numpy arrays.

No arithmetic of the method happens here; every call goes to libsbm.so.
"""
import ctypes as C

import numpy as np
import torch

from . import native as N


def _ptr(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous cuda tensor")
    return C.c_void_p(t.data_ptr())


_FLOATS = (torch.float32, torch.float64)


class Problem:
    """DG-SBM hierarchy for one geometry (see include/sbm.h, sbm_setup)."""

    def __init__(self, geometry, n, p, device=0, stream=None, **opts):
        self._h = None
        L = N.lib()
        o = N.default_options(geometry.dim, p)
        for k, v in opts.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        o.device = device
        if stream is None and device >= 0 and torch.cuda.is_available():
            stream = torch.cuda.current_stream(device).cuda_stream
        o.stream = stream
        g = N.Geometry()
        g.dim = geometry.dim
        self._keep = []
        if geometry.kind == "balls":
            c = np.ascontiguousarray(geometry.centers, dtype=np.float64)
            r = np.ascontiguousarray(geometry.radii, dtype=np.float64)
            self._keep += [c, r]
            g.kind = N.GEOM_BALLS
            g.n_balls = len(r)
            g.centers = c.ctypes.data_as(C.POINTER(C.c_double))
            g.radii = r.ctypes.data_as(C.POINTER(C.c_double))
        elif geometry.kind == "ellipsoid":
            c = np.ascontiguousarray(np.ravel(geometry.centers), dtype=np.float64)
            r = np.ascontiguousarray(geometry.radii, dtype=np.float64)
            R = np.ascontiguousarray(geometry.rotation, dtype=np.float64)
            self._keep += [c, r, R]
            g.kind = N.GEOM_ELLIPSOID
            g.centers = c.ctypes.data_as(C.POINTER(C.c_double))
            g.radii = r.ctypes.data_as(C.POINTER(C.c_double))
            g.rotation = R.ctypes.data_as(C.POINTER(C.c_double))
        elif geometry.kind == "star":
            g.kind = N.GEOM_STAR2D
            g.star_r0, g.star_a, g.star_k = geometry.star_r0, geometry.star_a, geometry.star_k
        elif geometry.kind == "callback":
            g.kind = N.GEOM_CALLBACK
            d = geometry.dim

            def phi(x, _u):
                return float(geometry.phi(np.ctypeslib.as_array(x, (1, d)))[0])

            def grad(x, out, _u):
                np.ctypeslib.as_array(out, (d,))[:] = geometry.grad(np.ctypeslib.as_array(x, (1, d)))[0]

            def hess(x, out, _u):
                np.ctypeslib.as_array(out, (d * d,))[:] = geometry.hess(np.ctypeslib.as_array(x, (1, d)))[0].ravel()
            cbs = (N.PHI_FN(phi), N.VEC_FN(grad), N.VEC_FN(hess))
            self._keep += list(cbs)
            g.phi, g.grad, g.hess = cbs
        else:
            raise ValueError(geometry.kind)
        h = C.c_void_p()
        st = L.sbm_setup(C.byref(g), n, p, C.byref(o), C.byref(h))
        if st < 0:
            msg = L.sbm_last_error(h).decode() if h.value else ""
            if h.value:
                L.sbm_destroy(h)
            raise N.SbmError(st, msg)
        self._h = h
        self.dim, self.n, self.p = geometry.dim, n, p
        self.device = torch.device("cuda", device) if device >= 0 else None
        lay = N.Layout()
        N.check(L.sbm_layout_info(h, C.byref(lay)), h)
        self.layout = lay
        self.n_dofs = lay.n_dofs
        self.n_levels = lay.n_levels

    def __del__(self):
        if getattr(self, "_h", None) is not None:
            try:
                N.lib().sbm_destroy(self._h)
            except Exception:  # interpreter shutdown: the library is already gone
                pass
            self._h = None

    close = __del__

    # ------------------------------------------------------------- metadata
    def level_info(self, level=-1):
        vals = [C.c_int() for _ in range(5)]
        N.check(N.lib().sbm_level_info(self._h, level, *[C.byref(v) for v in vals]), self._h)
        return dict(zip(("n", "p", "n_active", "n_colour0", "n_surrogate_faces"), [v.value for v in vals]))

    def level_blocks(self, level=-1):
        vals = [C.c_int() for _ in range(3)]
        N.check(N.lib().sbm_level_blocks(self._h, level, *[C.byref(v) for v in vals]), self._h)
        return dict(zip(("n_boundary", "n_clipped", "n_clipped_colour0"), [v.value for v in vals]))

    def active_cells(self, level=-1):
        info = self.level_info(level)
        out = np.zeros((info["n_active"], self.dim), dtype=np.int32)
        N.check(N.lib().sbm_active_cells(self._h, level, out.ctypes.data_as(C.POINTER(C.c_int)), out.size), self._h)
        return out

    def shifts(self, level=-1):
        info = self.level_info(level)
        nf = (info["p"] + 1) ** (self.dim - 1)
        out = np.zeros((info["n_surrogate_faces"], nf, self.dim))
        N.check(N.lib().sbm_shifts(self._h, level, out.ctypes.data_as(C.POINTER(C.c_double)), out.size), self._h)
        return out

    def set_shifts(self, shifts, level=-1):
        """Load externally supplied shifts (test hook, sbm_set_shifts)."""
        info = self.level_info(level)
        nf = (info["p"] + 1) ** (self.dim - 1)
        a = np.ascontiguousarray(shifts, dtype=np.float64)
        if a.shape != (info["n_surrogate_faces"], nf, self.dim):
            raise ValueError(f"shifts of shape {a.shape}, level {level} needs "
                             f"{(info['n_surrogate_faces'], nf, self.dim)}")
        N.check(N.lib().sbm_set_shifts(self._h, level, a.ctypes.data_as(C.POINTER(C.c_double)), a.size), self._h)

    def cell_block(self, cell, level=-1, inverse=False):
        info = self.level_info(level)
        nc = (info["p"] + 1) ** self.dim
        out = np.zeros((nc, nc))
        N.check(N.lib().sbm_cell_block(self._h, level, cell, int(inverse),
                                       out.ctypes.data_as(C.POINTER(C.c_double))), self._h)
        return out

    def coarse_matrix(self):
        info = self.level_info(0)
        nd = info["n_active"] * (info["p"] + 1) ** self.dim
        out = np.zeros((nd, nd))
        N.check(N.lib().sbm_coarse_matrix(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), out.size), self._h)
        return out

    def level_dofs(self, level=-1):
        info = self.level_info(level)
        return info["n_active"] * (info["p"] + 1) ** self.dim

    def _vectors(self, *pairs, dtype=None):
        """Check (tensor, level) pairs before any pointer reaches the library:
        the C side sees only addresses, so a wrong length, dtype or device
        would become an out-of-bounds device access.  Returns the common
        dtype's fp32 flag."""
        dt = dtype
        for t, level in pairs:
            if not isinstance(t, torch.Tensor):
                raise TypeError("expected a torch tensor")
            if t.dtype not in _FLOATS:
                raise ValueError(f"vectors must be float32 or float64, got {t.dtype}")
            if dt is None:
                dt = t.dtype
            elif t.dtype != dt:
                raise ValueError(f"mixed dtypes in one call ({t.dtype} and {dt})")
            if self.device is None or t.device != self.device:
                raise ValueError(f"vector on {t.device}, problem on {self.device}")
            if not t.is_contiguous():
                raise ValueError("vectors must be contiguous")
            want = self.level_dofs(level)
            if t.numel() != want:
                raise ValueError(f"vector of {t.numel()} entries where level {level} has {want} DoFs")
        return int(dt == torch.float32)

    # ------------------------------------------------------------- data
    def rhs(self, f, g):
        """b (FP64 cuda tensor) for vectorised callables f(X), g(X) on (npts, dim) arrays."""
        d = self.dim

        def wrap(fn):
            def cb(x, npts, out, _u):
                X = np.ctypeslib.as_array(x, (npts, d))
                np.ctypeslib.as_array(out, (npts,))[:] = fn(X)
            return N.FIELD_FN(cb)
        cf, cg = wrap(f), wrap(g)
        b = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        self._vectors((b, -1), dtype=torch.float64)
        N.check(N.lib().sbm_rhs(self._h, cf, cg, None, _ptr(b)), self._h)
        return b

    # ------------------------------------------------------------- operators
    def apply(self, x, y=None):
        y = torch.empty_like(x) if y is None else y
        f32 = self._vectors((x, -1), (y, -1))
        N.check(N.lib().sbm_apply(self._h, _ptr(x), _ptr(y), f32), self._h)
        return y

    def vcycle(self, r, z=None):
        z = torch.empty_like(r) if z is None else z
        f32 = self._vectors((r, -1), (z, -1))
        N.check(N.lib().sbm_vcycle(self._h, _ptr(r), _ptr(z), f32), self._h)
        return z

    def level_apply(self, level, x, y=None):
        y = torch.empty_like(x) if y is None else y
        f32 = self._vectors((x, level), (y, level))
        N.check(N.lib().sbm_level_apply(self._h, level, _ptr(x), _ptr(y), f32), self._h)
        return y

    def colour_update(self, level, colour, b, z):
        f32 = self._vectors((b, level), (z, level))
        N.check(N.lib().sbm_colour_update(self._h, level, colour, _ptr(b), _ptr(z), f32), self._h)
        return z

    def restrict(self, level, r, bc):
        f32 = self._vectors((r, level), (bc, self._coarser(level)))
        N.check(N.lib().sbm_restrict(self._h, level, _ptr(r), _ptr(bc), f32), self._h)
        return bc

    def prolong_add(self, level, zc, zf):
        f32 = self._vectors((zc, self._coarser(level)), (zf, level))
        N.check(N.lib().sbm_prolong_add(self._h, level, _ptr(zc), _ptr(zf), f32), self._h)
        return zf

    def _coarser(self, level):
        lv = self.n_levels - 1 if level == -1 else level
        if not 1 <= lv < self.n_levels:
            raise ValueError(f"level {level} has no coarser level")
        return lv - 1

    def sync(self):
        N.check(N.lib().sbm_sync(self._h), self._h)

    def set_vcycle_fp32(self, fp32):
        N.check(N.lib().sbm_set_vcycle_fp32(self._h, int(bool(fp32))), self._h)

    def solve(self, b, x=None, tol=1e-8, restart=30, max_iter=1000, vcycle_fp32=None, noalloc=False):
        """FGMRES solve (sbm_solve); noalloc=True takes the allocation-free
        entry point (sbm_solve_noalloc: workspace in the library's fixed
        device scratch array)."""
        if vcycle_fp32 is not None:
            self.set_vcycle_fp32(vcycle_fp32)
        x = torch.empty_like(b) if x is None else x
        self._vectors((b, -1), (x, -1), dtype=torch.float64)
        st = N.Stats()
        fn = N.lib().sbm_solve_noalloc if noalloc else N.lib().sbm_solve
        status = N.check(fn(self._h, _ptr(b), _ptr(x), tol, restart, max_iter, C.byref(st)), self._h)
        return x, dict(status=status, iterations=st.iterations, converged=bool(st.converged),
                       rel_residual=st.rel_residual_true, seconds=st.seconds)
