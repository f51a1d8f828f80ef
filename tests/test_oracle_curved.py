"""Pins of the oracle's curved-element piece (oracle/curved.py): the quadratic geometry map,
the curved mass matrix and its weight-adjusted approximate inverse, the L2 projection, and
the three ways of recovering the field from the mapped variable (section 4)."""
import numpy as np
import pytest

from mtp_inputs import meshes
from oracle import curved
from oracle.maxwell import System
from oracle.simplex import basis, quadrature

REF_NODES = np.array([[0, 0], [1, 0], [0, 1], [0.5, 0], [0.5, 0.5], [0, 0.5]], dtype=float)


def _triangle(eps_disp=0.0, which=1):
    """A non-symmetric triangle; the midpoint of edge `which` (0: (0,1), 1: (1,2), 2: (0,2))
    pushed outward by eps_disp times the edge length."""
    X = np.array([[0.1, -0.2], [1.3, 0.15], [0.35, 0.9]])
    G = np.zeros((6, 2))
    G[:3] = X
    for s, (a, b) in enumerate([(0, 1), (1, 2), (0, 2)]):
        G[3 + s] = 0.5 * (X[a] + X[b])
    a, b = [(0, 1), (1, 2), (0, 2)][which]
    t = X[b] - X[a]
    n = np.array([t[1], -t[0]])
    c = X.mean(axis=0)
    if (G[3 + which] - c) @ n < 0:
        n = -n
    G[3 + which] += eps_disp * n
    return curved.CurvedTriangle(G)


def test_map_interpolates_its_nodes():
    el = _triangle(0.2)
    assert np.allclose(el.map(REF_NODES), el.G, atol=1e-15)
    assert np.allclose(curved.shape_p2(REF_NODES), np.eye(6), atol=1e-15)
    assert np.allclose(curved.shape_p2(np.random.default_rng(0).random((9, 2)) * 0.5).sum(axis=1), 1.0)


def test_straight_midpoints_give_the_affine_jacobian():
    el = _triangle(0.0)
    X = el.G[:3]
    Jaff = np.stack([X[1] - X[0], X[2] - X[0]], axis=1)   # columns d x / d xh_l
    pts = np.random.default_rng(1).random((7, 2)) * 0.5
    assert np.allclose(el.jac(pts), Jaff[None], atol=1e-14)
    assert np.allclose(el.map(pts), X[0] + pts @ Jaff.T, atol=1e-14)


def test_physical_gradients_follow_the_chain_rule():
    """grad_x f at x(xh) equals J^{-T} gradhat (f o x)(xh), the reference gradient taken by
    central differences of the pulled-back function (a transposed J fails)."""
    el = _triangle(0.25, which=2)
    f = lambda x: x[:, 0] ** 2 * x[:, 1] + 3.0 * x[:, 1] - x[:, 0] * x[:, 1] ** 2   # noqa: E731
    gf = lambda x: np.stack([2 * x[:, 0] * x[:, 1] - x[:, 1] ** 2,                    # noqa: E731
                             x[:, 0] ** 2 + 3.0 - 2 * x[:, 0] * x[:, 1]], axis=1)
    pts = np.array([[0.2, 0.3], [0.6, 0.1], [0.1, 0.7], [0.33, 0.33]])
    h = 1e-6
    ghat = np.stack([(f(el.map(pts + h * e)) - f(el.map(pts - h * e))) / (2 * h) for e in np.eye(2)], axis=1)
    Jinv = np.linalg.inv(el.jac(pts))
    gphys = np.einsum("qlr,ql->qr", Jinv, ghat)
    assert np.allclose(gphys, gf(el.map(pts)), rtol=1e-7, atol=1e-7)
    # hat functions: they sum to one, and J^T grad lambda_k = gradhat lambdahat_k
    gl = el.grad_lambda(pts)
    assert np.allclose(gl.sum(axis=1), 0.0, atol=1e-13)
    back = np.einsum("qrl,qkr->qkl", el.jac(pts), gl)
    assert np.allclose(back, np.array([[-1, -1], [1, 0], [0, 1]])[None], atol=1e-13)


def _disk_area(n, curved_edges):
    mm = meshes.disk_tri(n)
    geo = meshes.p2_geometry(mm, on_circle=1.0 if curved_edges else None)
    pts, w = quadrature(2, 4)
    return sum(w @ np.abs(curved.CurvedTriangle(G).detj(pts)) for G in geo)


def test_disk_area_converges_at_fourth_order_with_curved_edges():
    ns = [2, 4, 8, 16]
    err_c = [abs(_disk_area(n, True) - np.pi) for n in ns]
    err_s = [abs(_disk_area(n, False) - np.pi) for n in ns]
    rate_c = np.log2(np.array(err_c[:-1]) / np.array(err_c[1:]))
    rate_s = np.log2(np.array(err_s[:-1]) / np.array(err_s[1:]))
    assert np.all(rate_s > 1.9) and np.all(rate_s < 2.1), rate_s      # inscribed polygon: O(h^2)
    assert np.all(rate_c[1:] > 3.7), rate_c                           # quadratic arcs: O(h^4)
    assert err_c[-1] < 1e-3 * err_s[-1]


@pytest.mark.parametrize("p", [1, 2, 4])
def test_weight_adjusted_inverse_is_exact_on_affine_elements(p):
    el = _triangle(0.0)
    MJ = curved.mass_J(el, p)
    detJ = abs(el.detj(np.array([[0.2, 0.2]]))[0])
    assert np.allclose(MJ, detJ * np.eye(basis(2, p).n), atol=1e-13)
    assert np.allclose(curved.mass_invJ(el, p) @ MJ, np.eye(basis(2, p).n), atol=1e-12)


@pytest.mark.parametrize("p", [1, 3])
def test_weight_adjusted_defect_is_second_order_in_the_curvature(p):
    """||M_{1/J} M_J - I|| = C eps^2 + O(eps^3) for a midpoint pushed out by eps: halving
    eps divides the defect by 4; M_{1/J} stays symmetric positive definite."""
    nb = basis(2, p).n
    defects = []
    for e in (0.04, 0.02, 0.01):
        el = _triangle(e)
        Mi = curved.mass_invJ(el, p)
        assert np.allclose(Mi, Mi.T, atol=1e-15)
        assert np.linalg.eigvalsh(Mi).min() > 0
        defects.append(np.linalg.norm(Mi @ curved.mass_J(el, p) - np.eye(nb), 2))
    r = np.array(defects[:-1]) / np.array(defects[1:])
    assert np.all(r > 3.6) and np.all(r < 4.4), (defects, r)


def test_exact_projection_reproduces_the_space_and_wadg_is_close():
    p = 3
    B = basis(2, p)
    c = np.random.default_rng(5).standard_normal((B.n, 2))
    fun = lambda x: B.eval(x) @ c   # noqa: E731
    errs = []
    for e in (0.04, 0.02):
        el = _triangle(e)
        assert np.allclose(curved.project(el, p, fun, "exact"), c, atol=1e-12)
        errs.append(np.linalg.norm(curved.project(el, p, fun, "wadg") - c))
    assert 3.6 < errs[0] / errs[1] < 4.4
    # a non-polynomial function: both projections are close, the exact one is the
    # best approximation in the |det J|-weighted norm
    g = lambda x: np.sin(3 * x[:, :1]) * np.cos(2 * x[:, 1:])   # noqa: E731
    el = _triangle(0.05)
    Ue, Uw = curved.project(el, p, g, "exact"), curved.project(el, p, g, "wadg")
    pts, w = quadrature(2, p + 8)
    wt = w * np.abs(el.detj(pts))
    res = lambda U: np.sqrt(wt @ ((B.eval(pts) @ U - g(pts)) ** 2).ravel())   # noqa: E731
    assert res(Ue) <= res(Uw) + 1e-15


def test_recoveries_agree_where_K_is_constant():
    """Flat front on a curved element (grad phi = 0, K = diag(eps, eps, mu)): Galerkin and
    the exact projection both give K^{-1} M_J^{-1} Y; on an affine element with a non-zero
    constant grad phi all three give (K(b)^{-1} x M_J^{-1}) Y."""
    sys, p, eps, mu = System(2), 2, 2.25, 1.3
    nb = basis(2, p).n
    Y = np.random.default_rng(7).standard_normal((nb, 3))
    el = _triangle(0.1)
    zero = lambda x: np.zeros((len(x), 2))   # noqa: E731
    want = np.linalg.solve(curved.mass_J(el, p), Y) / sys.g_diag(eps, mu)[None, :]
    assert np.allclose(curved.recover(el, p, sys, Y, zero, eps, mu, "galerkin"), want, atol=1e-12)
    assert np.allclose(curved.recover(el, p, sys, Y, zero, eps, mu, "exact"), want, atol=1e-12)
    el = _triangle(0.0)
    b = np.array([0.3, -0.4])
    const = lambda x: np.tile(b, (len(x), 1))   # noqa: E731
    K = sys.K(b, eps, mu)
    want = np.linalg.solve(curved.mass_J(el, p), Y) @ np.linalg.inv(K).T
    for how in ("galerkin", "exact", "wadg"):
        assert np.allclose(curved.recover(el, p, sys, Y, const, eps, mu, how), want, atol=1e-12), how


def test_wadg_recovery_tracks_the_exact_one_to_second_order():
    """A tent on a curved element (grad phi varying inside it): the weight-adjusted
    recovery differs from the exact-inverse one by O(eps^2) in the curvature amplitude."""
    sys, p, eps, mu = System(2), 3, 1.0, 1.0
    nb = basis(2, p).n
    Y = np.random.default_rng(8).standard_normal((nb, 3))
    diffs = []
    for e in (0.04, 0.02, 0.01):
        el = _triangle(e)
        gphi = curved.front_gradient(el, [0.0, 0.0, 0.0], [0.0, 0.15, 0.0], 0.5)
        Ue = curved.recover(el, p, sys, Y, gphi, eps, mu, "exact")
        Uw = curved.recover(el, p, sys, Y, gphi, eps, mu, "wadg")
        Ug = curved.recover(el, p, sys, Y, gphi, eps, mu, "galerkin")
        assert np.linalg.norm(Ug - Ue) / np.linalg.norm(Ue) < 0.05
        diffs.append(np.linalg.norm(Uw - Ue) / np.linalg.norm(Ue))
    r = np.array(diffs[:-1]) / np.array(diffs[1:])
    assert np.all(r > 3.5) and np.all(r < 4.5), (diffs, r)


# ---------------------------------------------------------------- the curved tent solve
def _disk_solver(n, p, how, curved_edges=True, T=0.2):
    from mtp_inputs import fields
    from oracle.pitch import pitch
    mm = meshes.disk_tri(n)
    geo = meshes.p2_geometry(mm, on_circle=1.0 if curved_edges else None)
    CM = curved.CurvedMesh(mm["coords"], mm["cells"], geo)
    tents = pitch(CM.base, T, 0.5, k_elem=CM.step_bounds(0.5))
    ex = fields.CircularCavityTE()
    S = curved.CurvedSolver(CM, p, p + 1, 2 * p, recovery=how)
    S.set_exact(ex, 0.0)
    S.run(tents)
    e, r = S.l2_error(ex, T)
    return S, tents, CM, e / r


@pytest.mark.parametrize("how", ["galerkin", "exact", "wadg"])
def test_curved_solve_equals_the_affine_oracle_on_straight_elements(how):
    """Straight midpoints: every recovery gives the affine oracle's tent solve (a PEC
    square cavity, P2, q = 3, m = 4, one slab of 0.2)."""
    from mtp_inputs import fields
    from oracle.mesh import Mesh
    from oracle.pitch import pitch
    from oracle.solve import OracleSolver
    mm = meshes.square_tri(3)
    M = Mesh(mm["coords"], mm["cells"])
    tents = pitch(M, 0.2, 0.5)
    ex = fields.CavityTE_PEC()
    A = OracleSolver(M, 2, 3, 4)
    A.set_nodal_u(ex.u(meshes.equispaced_nodes(mm, 2), 0.0))
    C = curved.CurvedSolver(curved.CurvedMesh(mm["coords"], mm["cells"], meshes.p2_geometry(mm)), 2, 3, 4,
                            recovery=how)
    C.cw[:] = A.cw
    A.run(tents)
    C.run(tents)
    assert np.abs(C.cw - A.cw).max() <= 1e-13 * np.abs(A.cw).max()


def test_curved_disk_converges_at_the_optimal_order():
    """Circular PEC cavity, TE mode J_1(k r) cos(theta), P2: with quadratic boundary
    elements the error falls at order >= p + 1 - 0.3 (measured 3.1 from 2 to 3 rings, 3.4
    beyond); the straight-sided disk of the same vertices stalls near order 1.5 (the
    polygonal boundary's geometry error)."""
    errs_c = [_disk_solver(n, 2, "galerkin")[3] for n in (2, 4)]
    errs_s = [_disk_solver(n, 2, "galerkin", curved_edges=False)[3] for n in (2, 4)]
    rate_c = np.log2(errs_c[0] / errs_c[1])
    rate_s = np.log2(errs_s[0] / errs_s[1])
    assert rate_c > 2.7, (errs_c, rate_c)
    assert rate_s < 1.8, (errs_s, rate_s)
    assert errs_c[1] < 0.2 * errs_s[1]


def test_weight_adjusted_scheme_tracks_galerkin_on_the_disk():
    """The weight-adjusted scheme (every curved mass inverse replaced by M_{1/J}) and the
    Galerkin one differ far below their common error against the exact mode."""
    Sg, _, _, eg = _disk_solver(3, 2, "galerkin")
    Sw, _, _, ew = _disk_solver(3, 2, "wadg")
    diff = np.linalg.norm(Sw.cw - Sg.cw) / np.linalg.norm(Sg.cw)
    assert diff < 0.05 * eg, (diff, eg)
    assert abs(ew - eg) < 0.05 * eg


def test_curved_pitcher_keeps_the_causality_bound():
    """Every front met while replaying the disk's tents keeps |grad phi| within the slope
    bound sigma sqrt(eps mu) (sigma = 1/2) on a denser sample than the one the steps use;
    the curved elements are exactly those on the circle, straight ones keep the affine
    rule's step, and some curved ones get a different step from it."""
    from oracle.pitch import pitch
    mm = meshes.disk_tri(4)
    CM = curved.CurvedMesh(mm["coords"], mm["cells"], meshes.p2_geometry(mm, on_circle=1.0))
    k = CM.step_bounds(0.5)
    tents = pitch(CM.base, 0.3, 0.5, k_elem=k)
    assert curved.max_front_slope(CM, tents) <= 0.5 * (1 + 1e-3)
    norms = np.linalg.norm(CM.base.grad_lam, axis=2)
    k_aff = 0.5 / (norms.sum(axis=1, keepdims=True) - norms).min(axis=1)
    assert np.array_equal(CM.curved, np.array([np.any(CM.base.nbr[e] < 0) for e in range(CM.ne)]))
    assert np.array_equal(k[~CM.curved], k_aff[~CM.curved])
    assert np.any(np.abs(k[CM.curved] - k_aff[CM.curved]) > 1e-3 * k_aff[CM.curved])
