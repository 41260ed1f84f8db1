"""Host-side setup of the C library (no GPU) against the oracle.

The library is set up in host-only mode (device = -1): active sets, order,
surrogate faces, closest points, cell blocks, their LU inverses and the
coarsest-level matrix are compared with the oracle's independent
construction by direct quadrature.
"""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import dg, geometry, mg
from paper_2506_12899_amd import native, workloads
from tests.oracle_geom import oracle_geometry

pytestmark = pytest.mark.skipif(not os.path.exists(native.LIBPATH), reason="libsbm.so not built")


def _problem(geo, n, p, **kw):
    from paper_2506_12899_amd.problem import Problem
    return Problem(geo, n, p, device=-1, **kw)


CASES = [
    ("disk", workloads.balls([[0.03, -0.02]], [0.7]), 16, 1),
    ("disk", workloads.balls([[0.03, -0.02]], [0.7]), 16, 3),
    ("star", workloads.star(0.6, 0.15, 5), 24, 2),
    ("union2", workloads.balls([[-0.2, 0.0], [0.25, 0.1], [0.0, -0.3]], [0.45, 0.4, 0.35]), 16, 2),
    ("sphere", workloads.balls([[0.03, -0.02, 0.01]], [0.75]), 8, 2),
    ("union3", workloads.eight_balls(0), 10, 1),
    ("union3", workloads.eight_balls(0), 8, 3),
]


@pytest.mark.parametrize("name,geo,n,p", CASES)
@pytest.mark.parametrize("ext", [0, 1])
def test_levels_shifts_blocks_match_oracle(name, geo, n, p, ext):
    pb = _problem(geo, n, p, ext=ext)
    H = mg.Hierarchy(oracle_geometry(geo), geo.dim, n, p, ext=ext)
    assert pb.n_levels == len(H.levels)
    rng = np.random.default_rng(0)
    for l, L in enumerate(H.levels):
        info = pb.level_info(l)
        assert (info["n"], info["p"], info["n_active"], info["n_colour0"], info["n_surrogate_faces"]) == \
            (L.n, L.p, L.n_act, L.n_col0, L.n_surr)
        assert np.array_equal(pb.active_cells(l), L.cells)
        sh = pb.shifts(l)
        assert np.abs(sh - L.shifts).max(initial=0.0) <= 1e-12
        cells = rng.choice(L.n_act, size=min(L.n_act, 12), replace=False) if L.n_act else []
        bcells = L.boundary_cells[:8]
        for K in list(cells) + list(bcells):
            D = pb.cell_block(int(K), l)
            ref = L.D[K]
            assert np.abs(D - ref).max() <= 1e-12 * np.abs(ref).max(), (l, K)
            B = pb.cell_block(int(K), l, inverse=True)
            Bref = H.inv[l][K]
            assert np.abs(B - Bref).max() <= 1e-10 * np.abs(Bref).max(), (l, K)
    A0 = pb.coarse_matrix()
    assert np.abs(A0 - H.levels[0].A.toarray()).max(initial=0.0) <= 1e-12 * max(1.0, np.abs(A0).max(initial=0.0))


def test_star_closest_points_on_workload_mesh():
    geo = workloads.star(0.6, 0.15, 5)
    pb = _problem(geo, 64, 2)
    L = dg.Level(oracle_geometry(geo), 2, 64, 2, build_matrix=False)
    assert np.abs(pb.shifts() - L.shifts).max() <= 1e-12


def test_invalid_arguments_rejected():
    geo = workloads.balls([[0.0, 0.0]], [0.7])
    from paper_2506_12899_amd.problem import Problem
    with pytest.raises(native.SbmError):
        Problem(geo, 8, 4, device=-1)
    with pytest.raises(native.SbmError):
        Problem(geo, 0, 1, device=-1)
    # a background mesh beyond int cell indices (n^2 >= 2^31) is refused before any allocation
    with pytest.raises(native.SbmError):
        Problem(geo, 46341, 1, device=-1)
    with pytest.raises(native.SbmError):
        Problem(geo, 8, 1, device=-1, ext=3)
    pb = _problem(geo, 8, 1)
    L = native.lib()
    # device entry points refuse a host-only problem
    assert L.sbm_apply(pb._h, C.c_void_p(1), C.c_void_p(2), 0) == -1
    assert L.sbm_vcycle(pb._h, C.c_void_p(1), C.c_void_p(2), 0) == -1
    assert L.sbm_level_apply(pb._h, 99, C.c_void_p(1), C.c_void_p(2), 0) == -1


def test_callback_level_set_matches_exact_sphere():
    c = np.array([0.03, -0.02, 0.01])

    class CB:
        kind, dim = "callback", 3

        @staticmethod
        def phi(X):
            return np.sum((X - c) ** 2, 1) - 0.75 ** 2

        @staticmethod
        def grad(X):
            return 2 * (X - c)

        @staticmethod
        def hess(X):
            return np.broadcast_to(2 * np.eye(3), (X.shape[0], 3, 3))
    pb_cb = _problem(CB, 8, 1)
    pb_ex = _problem(workloads.balls([c], [0.75]), 8, 1)
    assert np.abs(pb_cb.shifts() - pb_ex.shifts()).max() <= 1e-12


def test_every_declared_symbol_is_exported():
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "sbm.h")).read()
    names = set(re.findall(r"\b(sbm_[a-z0-9_]+)\s*\(", hdr))
    L = C.CDLL(native.LIBPATH)
    for nm in names:
        getattr(L, nm)
    assert {s[0] for s in native.SIGNATURES} >= names


def test_levels_without_active_cells_rejected():
    """Degenerate hierarchies: a domain holding no cell centre, and a small one
    on a mesh coarsened (coarse_dofs = 0) below the point where any coarse
    cell centre lies inside it.  Setup refuses both with a message instead of
    handing empty levels to the device path."""
    from paper_2506_12899_amd.problem import Problem
    small = workloads.balls([[0.0, 0.0]], [0.2])       # centres of the 4^2 mesh lie 0.354 away
    for n, kw in ((4, {}), (32, {"coarse_dofs": 0})):
        with pytest.raises(native.SbmError, match="no active cell"):
            Problem(small, n, 1, device=-1, **kw)
    # the same domain with the default coarsest size stops while levels hold cells
    pb = _problem(small, 32, 1)
    assert all(pb.level_info(l)["n_active"] > 0 for l in range(pb.n_levels))


# the stabilised 3D Q3 form: volume-fraction rule, one penalty degree for the
# hierarchy, singular-value floor of the smoother's block inverses
STAB_CASES = [
    ("sphere", workloads.balls([[0.03, -0.02, 0.01]], [0.8]), 12, 3, dict(workloads.STABILISED_Q3)),
    ("union3_core", workloads.eight_balls(0), 16, 3, dict(workloads.STABILISED_Q3)),
    ("union3", workloads.eight_balls(0), 16, 2, dict(lambda_frac=0.6, penalty_p=2, stab=1.0)),
    ("star", workloads.star(0.6, 0.15, 5), 32, 3, dict(lambda_frac=0.5, stab=1.0)),
    ("disk", workloads.balls([[0.03, -0.02]], [0.7]), 16, 2, dict(lambda_frac=1.0, penalty_p=2)),
]


@pytest.mark.parametrize("name,geo,n,p,kw", STAB_CASES)
def test_stabilised_form_matches_oracle(name, geo, n, p, kw):
    """Active sets by the volume-fraction rule, blocks with the hierarchy's
    penalty degree and the floored inverses agree with the oracle's."""
    pb = _problem(geo, n, p, **kw)
    H = mg.Hierarchy(oracle_geometry(geo), geo.dim, n, p, **kw)
    assert pb.n_levels == len(H.levels)
    floored = 0
    for l, L in enumerate(H.levels):
        assert np.array_equal(pb.active_cells(l), L.cells), l
        assert np.abs(pb.shifts(l) - L.shifts).max(initial=0.0) <= 1e-12
        exact = np.linalg.inv(L.D[L.boundary_cells])
        floored += int(np.sum(np.abs(exact - H.inv[l][L.boundary_cells]).max(axis=(1, 2)) > 0))
        for K in L.boundary_cells:
            D = pb.cell_block(int(K), l)
            assert np.abs(D - L.D[K]).max() <= 1e-12 * np.abs(L.D[K]).max(), (l, K)
            B = pb.cell_block(int(K), l, inverse=True)
            assert np.abs(B - H.inv[l][K]).max() <= 1e-10 * np.abs(H.inv[l][K]).max(), (l, K)
    if kw.get("stab", 0) > 0 and name != "star":
        assert floored > 0      # the floor is exercised


@pytest.mark.parametrize("level", [-1, 0])
def test_set_shifts_rebuilds_blocks_like_oracle(level):
    """Test hook sbm_set_shifts: externally supplied shifts (the computed ones
    perturbed by up to 0.2 h) give the blocks and inverses the oracle builds
    from the same shifts; a wrong count is refused and leaves the problem as
    it was."""
    from paper_2506_12899_amd import native as Nn
    geo = workloads.balls([[0.03, -0.02, 0.01]], [0.75])
    pb = _problem(geo, 8, 2, coarse_dofs=0)
    H = mg.Hierarchy(oracle_geometry(geo), 3, 8, 2, coarse_dofs=0)
    lv = len(H.levels) - 1 if level == -1 else level
    L0 = H.levels[lv]
    sh = L0.shifts + np.random.default_rng(3).uniform(-0.2, 0.2, L0.shifts.shape) * L0.h
    pb.set_shifts(sh, level)
    assert np.array_equal(pb.shifts(level), sh)
    L = dg.Level(oracle_geometry(geo), 3, L0.n, L0.p, shifts=sh)
    inv = mg.cell_inverses(L, L.D, 0.0)
    for K in L.boundary_cells:
        D = pb.cell_block(int(K), lv)
        assert np.abs(D - L.D[K]).max() <= 1e-12 * np.abs(L.D[K]).max()
        B = pb.cell_block(int(K), lv, inverse=True)
        assert np.abs(B - inv[K]).max() <= 1e-10 * np.abs(inv[K]).max()
    if lv == 0:
        A0 = pb.coarse_matrix()
        assert np.abs(A0 - L.A.toarray()).max() <= 1e-12 * np.abs(A0).max()
    with pytest.raises(Nn.SbmError):
        Nn.check(Nn.lib().sbm_set_shifts(pb._h, level, sh.ctypes.data_as(C.POINTER(C.c_double)), sh.size - 1),
                 pb._h)
    assert np.array_equal(pb.shifts(level), sh)


def test_paper_setting_shift_extremes_match_fig3():
    """The library in the paper's setting (paper_mode.problem: box
    [-1.01, 1.01]^2, 4 * 2^k cells, volume-fraction rule) reproduces the
    printed Fig. 3 extremes at levels 1-5 (see the oracle pin of the same
    figure)."""
    from paper_2506_12899_amd import paper_mode
    from paper_2506_12899_amd.problem import Problem
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "fig3_shift_extremes.txt"))
    for lam, lv, plo, phi_ in rows:
        if lv > 5:
            continue
        pr = paper_mode.problem("ball", 2, int(lv), 3, lam)
        pb = Problem(pr.geometry, pr.n, pr.p, device=-1, **pr.opts)
        lo, hi = paper_mode.signed_shift_extremes(pb)
        assert abs(hi - phi_) <= 6e-5, (lam, lv, hi, phi_)
        if lam < 1.0:
            assert abs(lo - plo) <= 6e-5, (lam, lv, lo, plo)


def test_deformed_domain_level_set_derivatives():
    """The deformed domain of Sec. 5.4, phi = (1 - 3/4 sin^2(pi x)) (x^2 + y^2)
    - 1/5, as the callback level set: its gradient and Hessian equal central
    differences, and f = -Lap(phi + 1) equals the differenced Laplacian."""
    from paper_2506_12899_amd import paper_mode
    g = paper_mode.deformed_geometry()
    sol = paper_mode.problem("deformed", 2, 3, 1, 0.5).solution
    X = np.random.default_rng(4).uniform(-1, 1, (20, 2))
    eps = 1e-5
    E = np.eye(2) * eps
    G = np.stack([(g.phi(X + E[c]) - g.phi(X - E[c])) / (2 * eps) for c in range(2)], axis=1)
    assert np.abs(G - g.grad(X)).max() <= 1e-8
    Hs = np.stack([(g.grad(X + E[c]) - g.grad(X - E[c])) / (2 * eps) for c in range(2)], axis=2)
    assert np.abs(Hs - g.hess(X)).max() <= 1e-7
    lap = sum((g.phi(X + E[c]) - 2 * g.phi(X) + g.phi(X - E[c])) / eps ** 2 for c in range(2))
    assert np.abs(sol.f(X) + lap).max() <= 1e-4 * np.abs(lap).max()


def test_deformed_domain_setup_matches_oracle():
    """Sec. 5.4 domain in the paper setting (lambda = 0.5): the library's
    active sets (volume fractions of a general level set) and its closest
    points (Lagrangian Newton, Sec. 4.2) agree with the oracle's independent
    construction on every level; every shift is normal to Gamma at its foot."""
    from paper_2506_12899_amd import paper_mode
    pr = paper_mode.problem("deformed", 2, 3, 2, 0.5)
    pb = _problem(pr.geometry, pr.n, pr.p, **pr.opts)
    og = oracle_geometry(pr.geometry)
    okw = {k: v for k, v in pr.opts.items() if k in ("lo", "hi", "lambda_frac", "c_F", "c_G")}
    for l in range(pb.n_levels):
        info = pb.level_info(l)
        L = dg.Level(og, 2, info["n"], info["p"], build_matrix=False, **okw)
        assert np.array_equal(pb.active_cells(l), L.cells), l
        sh = pb.shifts(l)
        assert np.abs(sh - L.shifts).max() <= 1e-9, l
        foot = (L.face_points + sh).reshape(-1, 2)
        assert np.abs(og.phi(foot)).max() <= 1e-12
        gr = pr.geometry.grad(foot)
        d = sh.reshape(-1, 2)
        cross = d[:, 0] * gr[:, 1] - d[:, 1] * gr[:, 0]
        assert np.abs(cross).max() <= 1e-9 * np.abs(gr).max()
