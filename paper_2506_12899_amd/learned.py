"""Training driver and runtime for the learned boundary-cell smoother correction.

Marshalling and orchestration only: data generation calls the library's
operator, colour-update, V-cycle and sample-gathering kernels; the network is
trained with the library's forward, loss, backward and Adam kernels; inference
runs through sbm_set_learned (BF16 on the matrix cores).  Torch provides device
memory only.

Data protocol (per seeded training geometry, p = 3, 3D): x* ~ N(0, 1), b = A x*;
from z = 0 and from the iterates after a few preconditioned Richardson steps
z += V-cycle(b - A z) (where the error modes the plain cycle handles badly
dominate), before each finest-level colour update of one smoothing step the
boundary cells of that colour contribute the pair (e_K = x*_K - z_K,
r_K = (b - A z)_K) together with B_K r_K and the cell's features, scaled to
|e_K| = 1 (sbm_collect_pairs, sbm_richardson).

Checkpoint format (little-endian): magic b"SBMMLP01", int32 n_in, width,
n_out, n_cell, int64 step, then params, Adam m, Adam v as float32.
"""
import ctypes as C
import struct
import time

import numpy as np
import torch

from . import native as N
from . import workloads

MAGIC = b"SBMMLP01"


def _p(t):
    return C.c_void_p(t.data_ptr())


class MLP:
    """Flat-parameter MLP trained with the library's kernels."""

    def __init__(self, n_in, n_cell, width=64, rank=4, seed=0, device="cuda", omega=0.8, train_uv=True):
        self.n_in, self.width, self.n_cell = n_in, width, n_cell
        self.train_uv = bool(train_uv)
        self.n_out = 1 + 2 * n_cell * rank
        self.omega = omega
        self.device = device
        self.params = torch.from_numpy(init_params(n_in, width, n_cell, rank, seed)).to(device, torch.float32)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = {}

    @property
    def n_params(self):
        return self.params.numel()

    def _work(self, S, dtype):
        key = (S, dtype)
        if key not in self._ws:
            w, no = self.width, self.n_out
            mk = lambda *s: torch.empty(*s, dtype=dtype, device=self.device)  # noqa: E731
            self._ws[key] = dict(H1=mk(S, w), H2=mk(S, w), O=mk(S, no), dO=mk(S, no), dH=mk(2 * S * w),
                                 loss_s=mk(S), loss=mk(1), grads=mk(self.n_params),
                                 work=mk(int(N.lib().sbm_mlp_work_elems(self.n_in, w, no, S))))
        return self._ws[key]

    def forward(self, X, params=None):
        params = self.params if params is None else params
        fp64 = int(X.dtype == torch.float64)
        ws = self._work(X.shape[0], X.dtype)
        N.check(N.lib().sbm_mlp_forward(fp64, self.n_in, self.width, self.n_out, X.shape[0], _p(params), _p(X),
                                        _p(ws["H1"]), _p(ws["H2"]), _p(ws["O"]), None))
        return ws

    def loss_grad(self, X, R, BR, E, params=None):
        """Returns (loss tensor (1,), grads tensor) computed on the device."""
        params = self.params if params is None else params
        fp64 = int(X.dtype == torch.float64)
        S = X.shape[0]
        ws = self.forward(X, params)
        L = N.lib()
        N.check(L.sbm_mlp_loss_grad(fp64, S, self.n_cell, int(self.train_uv), self.omega, _p(ws["O"]), _p(R), _p(BR),
                                    _p(E),
                                    _p(ws["dO"]), _p(ws["loss_s"]), _p(ws["loss"]), None))
        N.check(L.sbm_mlp_backward(fp64, self.n_in, self.width, self.n_out, S, _p(params), _p(X), _p(ws["H1"]),
                                   _p(ws["H2"]), _p(ws["dO"]), _p(ws["grads"]), _p(ws["dH"]), _p(ws["work"]), None))
        return ws["loss"], ws["grads"]

    def adam(self, grads, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        N.check(N.lib().sbm_adam(self.n_params, _p(self.params), _p(grads), _p(self.m), _p(self.v), self.step,
                                 lr, b1, b2, eps, None))

    def infer_bf16(self, X):
        O = torch.empty(X.shape[0], self.n_out, dtype=torch.float32, device=self.device)
        wb = torch.empty(int(N.lib().sbm_mlp_infer_wbuf_elems(self.n_out)), dtype=torch.int16, device=self.device)
        N.check(N.lib().sbm_mlp_infer_bf16(self.n_in, self.width, self.n_out, X.shape[0], _p(self.params), _p(X),
                                           _p(O), _p(wb), None))
        return O

    # ---------------------------------------------------------------- io
    def save(self, path):
        with open(path, "wb") as f:
            f.write(MAGIC)
            f.write(struct.pack("<iiiiq", self.n_in, self.width, self.n_out, self.n_cell, self.step))
            for t in (self.params, self.m, self.v):
                f.write(t.detach().cpu().numpy().astype("<f4").tobytes())

    @classmethod
    def load(cls, path, device="cuda", omega=0.8):
        with open(path, "rb") as f:
            if f.read(8) != MAGIC:
                raise ValueError("not an MLP checkpoint")
            n_in, width, n_out, n_cell, step = struct.unpack("<iiiiq", f.read(24))
            obj = cls(n_in, n_cell, width, device=device, omega=omega)
            n = obj.n_params
            for name in ("params", "m", "v"):
                arr = np.frombuffer(f.read(4 * n), dtype="<f4").copy()
                setattr(obj, name, torch.from_numpy(arr).to(device))
            obj.step = step
        return obj


def init_params(n_in, width, n_cell, rank=4, seed=0, scale_v=0.05):
    """Hidden layers uniform(+-1/sqrt(fan_in)); output rows of o_0 and U zero
    (the network starts as the plain smoother), rows of V small random."""
    n_out = 1 + 2 * n_cell * rank
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (width, n_in)) / np.sqrt(n_in)
    W2 = rng.uniform(-1, 1, (width, width)) / np.sqrt(width)
    W3 = np.zeros((n_out, width))
    W3[1 + n_cell * rank:] = rng.uniform(-1, 1, (n_cell * rank, width)) * scale_v / np.sqrt(width)
    return np.concatenate([W1.ravel(), np.zeros(width), W2.ravel(), np.zeros(width), W3.ravel(),
                           np.zeros(n_out)]).astype(np.float32)


# -------------------------------------------------------------------- data
def boundary_info(pb):
    L = N.lib()
    nb = C.c_int()
    N.check(L.sbm_boundary_cells(pb._h, C.byref(nb), None, 0), pb._h)
    cells = np.zeros(nb.value, dtype=np.int32)
    N.check(L.sbm_boundary_cells(pb._h, C.byref(nb), cells.ctypes.data_as(C.POINTER(C.c_int)), nb.value), pb._h)
    F = np.zeros((nb.value, L.sbm_feature_dim(pb.dim)))
    N.check(L.sbm_boundary_features(pb._h, F.ctypes.data_as(C.POINTER(C.c_double)), F.size), pb._h)
    return cells, F


def boundary_samples(pb, r, e):
    nb = pb.layout.n_boundary_cells
    nc = pb.layout.dofs_per_cell
    R = torch.empty(nb, nc, dtype=torch.float64, device=r.device)
    BR, E = torch.empty_like(R), torch.empty_like(R)
    N.check(N.lib().sbm_boundary_samples(pb._h, _p(r), _p(e), _p(R), _p(BR), _p(E)), pb._h)
    return R, BR, E


def collect_pairs(pb, xs, b, z):
    """(R, BR, E, valid) of every finest-level boundary cell for the iterate z
    (sbm_collect_pairs: residual, error, block product and the per-sample
    normalisation |E| = 1 run in the library)."""
    nb = pb.layout.n_boundary_cells
    nc = pb.layout.dofs_per_cell
    R = torch.empty(nb, nc, dtype=torch.float64, device=b.device)
    BR, E = torch.empty_like(R), torch.empty_like(R)
    valid = torch.empty(nb, dtype=torch.int32, device=b.device)
    N.check(N.lib().sbm_collect_pairs(pb._h, _p(xs), _p(b), _p(z), _p(R), _p(BR), _p(E), _p(valid)), pb._h)
    return R, BR, E, valid


def richardson(pb, b, z, steps):
    """z <- z + V-cycle(b - A z), `steps` times, in the library."""
    if steps > 0:
        N.check(N.lib().sbm_richardson(pb._h, _p(b), _p(z), int(steps)), pb._h)


def generate(problem_factory, seeds, n, p=3, iterates=(0,), draws=4, device="cuda", log=print, geometry=None):
    """Training samples from the method's own iterations on seeded geometries.

    For each geometry (workloads.training_geometry(seed), or geometry(seed)),
    `draws` random discrete solutions x* (b = A x*), and for each count k in
    `iterates` the iterate z after k preconditioned Richardson steps from
    z = 0 (k = 0: white-noise error; larger k: the error modes the V-cycle
    reduces slowly dominate); from that iterate one smoothing step (colours 0,
    1, 1, 0) runs, and before each finest-level colour update the boundary
    cells of that colour give a pair (e_K, r_K) with B_K r_K and the cell's
    features.  Every piece of the method's arithmetic runs in the library;
    torch selects rows and concatenates."""
    Xs, Rs, BRs, Es = [], [], [], []
    for s in seeds:
        geo = workloads.training_geometry(s) if geometry is None else geometry(s)
        pb = problem_factory(geo, n, p)
        cells, F = boundary_info(pb)
        if len(cells) == 0:
            pb.close()
            continue
        n_col0 = pb.layout.n_colour0
        lf = pb.n_levels - 1
        Ft = torch.from_numpy(F).to(device)
        col = torch.from_numpy((cells >= n_col0).astype(np.int64)).to(device)
        for dr in range(draws):
            g = torch.Generator(device="cpu").manual_seed(10_000 + 97 * s + dr)
            xs = torch.randn(pb.n_dofs, dtype=torch.float64, generator=g).to(device)
            b = pb.apply(xs)
            z = torch.zeros_like(b)
            done = 0
            for k in sorted(iterates):
                richardson(pb, b, z, k - done)
                done = k
                zz = z.clone()
                for c in (0, 1, 1, 0):
                    R, BR, E, valid = collect_pairs(pb, xs, b, zz)
                    sel = (col == c) & (valid != 0)
                    Xs.append(Ft[sel])
                    Rs.append(R[sel])
                    BRs.append(BR[sel])
                    Es.append(E[sel])
                    pb.colour_update(lf, c, b, zz)
        pb.close()
        log(f"[learned] geometry {s}: {len(cells)} boundary cells")
    return (torch.cat(Xs).float(), torch.cat(Rs).float(), torch.cat(BRs).float(), torch.cat(Es).float())


def train(mlp, data, epochs=20, batch=4096, lr=1e-3, seed=0, log=print, time_budget=None):
    X, R, BR, E = data
    S = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.time()
    n0 = min(S, 8 * batch)
    loss0, _ = mlp.loss_grad(X[:n0].contiguous(), R[:n0].contiguous(), BR[:n0].contiguous(), E[:n0].contiguous())
    log(f"[learned] initial loss (plain smoother) {float(loss0.item()):.5f}")
    hist.append(float(loss0.item()))
    for ep in range(epochs):
        perm = torch.randperm(S, generator=g).to(X.device)
        tot, nb = 0.0, 0
        for i in range(0, S - batch + 1, batch):
            idx = perm[i:i + batch]
            loss, grads = mlp.loss_grad(X[idx].contiguous(), R[idx].contiguous(), BR[idx].contiguous(),
                                        E[idx].contiguous())
            mlp.adam(grads, lr=lr)
            tot += float(loss.item())
            nb += 1
        hist.append(tot / max(nb, 1))
        log(f"[learned] epoch {ep}: loss {hist[-1]:.5f}")
        if time_budget and time.time() - t0 > time_budget:
            break
    return hist


def install(pb, mlp):
    """BF16 inference on pb's finest boundary cells; enables the correction."""
    N.check(N.lib().sbm_set_learned(pb._h, _p(mlp.params), mlp.width), pb._h)


def use(pb, on):
    N.check(N.lib().sbm_use_learned(pb._h, int(bool(on))), pb._h)


def judged_solve(pb, mlp, b, x=None, tol=1e-8, max_iter=300, restart=30):
    """Solve with and without the learned correction and keep the better run.

    The plain smoother is the fallback and the judge: the learned form wins
    only if it reaches tol in fewer iterations, or, when neither converges, a
    lower true residual.  The winner stays enabled on pb.  Returns
    (x, stats, choice) with choice "learned" or "plain" and stats of both."""
    use(pb, False)
    x0, st0 = pb.solve(b, None, tol=tol, restart=restart, max_iter=max_iter)
    install(pb, mlp)
    x1, st1 = pb.solve(b, None, tol=tol, restart=restart, max_iter=max_iter)
    if st1["converged"] != st0["converged"]:
        better = st1["converged"]
    elif st0["converged"]:
        better = st1["iterations"] < st0["iterations"]
    else:
        better = st1["rel_residual"] < st0["rel_residual"]
    use(pb, better)
    xb = x1 if better else x0
    if x is not None:
        x.copy_(xb)
        xb = x
    return xb, {"plain": st0, "learned": st1}, ("learned" if better else "plain")
