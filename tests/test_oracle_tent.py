"""Pins of the oracle's per-tent DG operators and SAT recursion."""
from math import factorial

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.integrate import solve_ivp

from mtp_inputs import meshes
from oracle.mesh import Mesh
from oracle.simplex import basis, reference_nodes
from oracle.tent import TentDG


def _mesh(dim, n, kind=0):
    mm = meshes.cube_kuhn(n) if dim == 3 else meshes.square_tri(n)
    return Mesh(mm["coords"], mm["cells"], face_bc=meshes.uniform_bc(len(mm["cells"]), dim, kind))


def _dense(T, dg, blocks=None):
    ne, N = len(T["es"]), dg.nc * dg.nb
    X = np.zeros((ne * N, ne * N))
    if blocks is None:
        for (a, b), blk in T["A"].items():
            X[a * N:(a + 1) * N, b * N:(b + 1) * N] = blk
    else:
        for a, blk in enumerate(blocks):
            X[a * N:(a + 1) * N, a * N:(a + 1) * N] = blk
    return X


@pytest.mark.parametrize("dim,n,p,kind", [(2, 3, 2, 0), (2, 3, 3, 1), (3, 2, 2, 0), (3, 2, 1, 1)])
def test_energy_identity(dim, n, p, kind):
    """d/dth (1/2 U.MU) = U.AU - 1/2 U.M'U: zero for the central flux (alpha = 0), equal to
    minus the penalty integrals for alpha > 0 (pins every sign of the volume term, the
    tent-map mass derivative and the face terms)."""
    mesh = _mesh(dim, n, kind)
    rng = np.random.default_rng(9)
    tau = rng.uniform(0, 0.01, mesh.nv)
    for alpha in (0.0, 0.5):
        dg = TentDG(mesh, p, alpha=alpha)
        for v in range(mesh.nv):
            T = dg.tent(tau, v, tau[v] + 0.02)
            A = _dense(T, dg)
            Mp = _dense(T, dg, dg.Mprime(T))
            U = rng.standard_normal(A.shape[0])
            val = U @ A @ U - 0.5 * U @ Mp @ U
            scale = np.abs(U) @ np.abs(A) @ np.abs(U)
            if alpha == 0.0:
                assert abs(val) < 1e-13 * scale
            else:
                # penalty: -alpha sum_F int delta |P_t [[u]]|^2 (interior), doubled jump on walls
                pen = 0.0
                for i, (e, k) in enumerate(zip(T["es"], T["ks"])):
                    ue = U[i * dg.nc * dg.nb:(i + 1) * dg.nc * dg.nb].reshape(dg.nc, dg.nb)
                    for f in range(dim + 1):
                        if f == k:
                            continue
                        fc = dg.face(e, f, k)
                        nb = mesh.nbr[e, f]
                        u_in = fc["phi_e"] @ ue.T
                        if nb >= 0:
                            j = [int(x) for x in T["es"]].index(int(nb))
                            un = U[j * dg.nc * dg.nb:(j + 1) * dg.nc * dg.nb].reshape(dg.nc, dg.nb)
                            phi_n = dg.B.eval(mesh.to_ref(nb, fc["xq"]))
                            u_out = phi_n @ un.T
                            wgt = 0.5   # each interior face is visited from both sides
                        else:
                            u_out = u_in @ dg.sys.ghost_matrix(kind).T
                            wgt = 0.5   # u_in.P(u_in - u_out) = |P jump|^2 / 2 on a mirror wall
                        P = dg.sys.A(fc["n"]) @ dg.sys.A(fc["n"])   # tangential projector
                        jump = u_in - u_out
                        pen += wgt * np.sum(fc["w"] * T["H"] * fc["lam"] * np.einsum("qc,cd,qd->q", jump, P, jump))
                assert val <= 1e-13 * scale
                assert abs(val + alpha * pen) < 1e-12 * scale


def _tent_ode(dim, p, seed=10):
    mesh = _mesh(dim, 3)
    dg = TentDG(mesh, p, alpha=0.5)
    rng = np.random.default_rng(seed)
    tau = rng.uniform(0, 0.02, mesh.nv)
    v = int(np.argmin(tau))
    T = dg.tent(tau, v, tau[v] + 0.04)
    return dg, T


@pytest.mark.parametrize("q", [2, 3, 4])
def test_sat_temporal_order(q):
    """SAT(q, m) error against a DOP853 reference of dY/dth = A M(th)^{-1} Y decays as m^-q."""
    dg, T = _tent_ode(2, 2)
    A = _dense(T, dg)
    Mb = lambda th: _dense(T, dg, dg.M_of(T, th))  # noqa: E731
    N = dg.nc * dg.nb
    ne = len(T["es"])
    Y0 = np.random.default_rng(11).standard_normal(ne * N)
    ref = solve_ivp(lambda th, y: A @ np.linalg.solve(Mb(th), y), (0, 1), Y0, method="DOP853",
                    rtol=1e-13, atol=1e-14).y[:, -1]
    errs = []
    for m in (2, 4, 8):
        Y = dg.sat(T, [Y0[i * N:(i + 1) * N] for i in range(ne)], q, m)
        errs.append(np.linalg.norm(np.concatenate(Y) - ref))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > q - 0.35), (errs, rates)
    # with many Taylor terms SAT reproduces the exact tent solution
    Y = dg.sat(T, [Y0[i * N:(i + 1) * N] for i in range(ne)], 20, 2)
    assert np.linalg.norm(np.concatenate(Y) - ref) < 1e-11 * np.linalg.norm(ref)


def test_rk4_variant_is_classical_rk4_on_tent_ode():
    dg, T = _tent_ode(2, 2)
    A = _dense(T, dg)
    N, ne = dg.nc * dg.nb, len(T["es"])
    Y0 = np.random.default_rng(12).standard_normal(ne * N)
    ref = solve_ivp(lambda th, y: A @ np.linalg.solve(_dense(T, dg, dg.M_of(T, th)), y), (0, 1), Y0,
                    method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
    errs = [np.linalg.norm(np.concatenate(dg.rk4(T, [Y0[i * N:(i + 1) * N] for i in range(ne)], m)) - ref)
            for m in (4, 8)]
    assert 3.6 < np.log2(errs[0] / errs[1]) < 4.4


def test_sat_constant_mass_is_taylor_polynomial_of_exp():
    """With M constant (M' = 0) SAT reduces to the classical degree-q Taylor method for
    dY/dth = L Y, L = A M^{-1}: Y(1) = (sum_n (L/m)^n/n!)^m Y0, and to expm(L) for large q."""
    dg, T = _tent_ode(2, 2)
    M0 = dg.M_of(T, 0.0)
    dg_const = TentDG(dg.mesh, dg.p, alpha=0.5)
    dg_const.M_of = lambda T_, th: M0
    dg_const.Mprime = lambda T_: [np.zeros_like(b) for b in M0]
    A = _dense(T, dg)
    L = A @ np.linalg.inv(_dense(T, dg, M0))
    N, ne = dg.nc * dg.nb, len(T["es"])
    Y0 = np.random.default_rng(13).standard_normal(ne * N)
    for q, m in ((3, 4), (4, 3)):
        S = sum(np.linalg.matrix_power(L / m, n) / factorial(n) for n in range(q + 1))
        ref = np.linalg.matrix_power(S, m) @ Y0
        Y = np.concatenate(dg_const.sat(T, [Y0[i * N:(i + 1) * N] for i in range(ne)], q, m))
        assert np.allclose(Y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    Y = np.concatenate(dg_const.sat(T, [Y0[i * N:(i + 1) * N] for i in range(ne)], 24, 2))
    assert np.allclose(Y, sla.expm(L) @ Y0, rtol=1e-11, atol=1e-11 * np.abs(Y).max())


def test_brute_force_integrals_single_triangle():
    """Every integral the oracle assembles, checked on a generic triangle against exact
    sympy integration of polynomials (test function P, trial function Q)."""
    sp = pytest.importorskip("sympy")
    x, y, s, t = sp.symbols("x y s t")
    X = np.array([[0.1, -0.2], [2.0, 0.5], [0.3, 1.7]])
    mesh = Mesh(X, np.array([[0, 1, 2]]))
    p = 2
    dg = TentDG(mesh, p)
    P = 1 + 2 * x - x * y + 0.5 * y ** 2
    Q = 3 - x + 0.25 * x ** 2 + y
    nodes = X[0] + reference_nodes(2, p) @ (X[1:] - X[0])
    V = basis(2, p).eval(reference_nodes(2, p))
    coef = lambda F: np.linalg.solve(V, np.array([float(F.subs({x: a, y: b})) for a, b in nodes]))  # noqa: E731
    cP, cQ = coef(P), coef(Q)
    Xs = [sp.Rational(str(v)) for v in X.ravel()]
    X0, X1, X2 = (Xs[0], Xs[1]), (Xs[2], Xs[3]), (Xs[4], Xs[5])
    xm = X0[0] + s * (X1[0] - X0[0]) + t * (X2[0] - X0[0])
    ym = X0[1] + s * (X1[1] - X0[1]) + t * (X2[1] - X0[1])
    detJ = abs((X1[0] - X0[0]) * (X2[1] - X0[1]) - (X2[0] - X0[0]) * (X1[1] - X0[1]))
    lam = [1 - s - t, s, t]

    def tri_int(F):
        G = F.subs({x: xm, y: ym}, simultaneous=True)
        return float(sp.integrate(sp.integrate(G * detJ, (t, 0, 1 - s)), (s, 0, 1)))

    assert np.isclose(cP @ dg.mass(0) @ cQ, tri_int(P * Q), rtol=1e-12)
    for k in range(3):
        lam_xy = lam[k]  # lambda_k as a function of (s, t)
        D = dg.vol(0, k)
        for j, var in enumerate((x, y)):
            G = (sp.diff(P, var) * Q).subs({x: xm, y: ym}, simultaneous=True) * lam_xy
            exact = float(sp.integrate(sp.integrate(G * detJ, (t, 0, 1 - s)), (s, 0, 1)))
            assert np.isclose(cP @ D[j] @ cQ, exact, rtol=1e-12)
        for f in range(3):
            if f == k:
                continue
            ids = [i for i in range(3) if i != f]
            A0, A1 = X[ids[0]], X[ids[1]]
            xe = A0[0] + s * (A1[0] - A0[0])
            ye = A0[1] + s * (A1[1] - A0[1])
            lam_e = {ids[0]: 1 - s, ids[1]: s}[k]
            L = np.linalg.norm(A1 - A0)
            exact = float(sp.integrate((P * Q).subs({x: xe, y: ye}, simultaneous=True) * lam_e * L, (s, 0, 1)))
            fc = dg.face(0, f, k)
            assert np.isclose(cP @ fc["Fself"] @ cQ, exact, rtol=1e-12)
            # outward normal
            mid = 0.5 * (A0 + A1)
            assert (X[f] - mid) @ fc["n"] < 0 and abs(fc["n"] @ (A1 - A0)) < 1e-14


def test_impedance_flux_fixture_equals_godunov_fixture_for_unit_impedance():
    """The stored oracle runs of the 2D plane wave (eps = mu = 1) with the impedance-matched
    flux and with the alpha = 1/2 flux agree to rounding."""
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    a = np.load(os.path.join(here, "oracle_te_planewave_p2_imp.npz"))
    b = np.load(os.path.join(here, "oracle_te_planewave_p2.npz"))
    assert np.linalg.norm(a["w"] - b["w"]) <= 1e-12 * np.linalg.norm(b["w"])


def test_brute_force_integrals_single_tet_and_shared_face():
    """Every integral the oracle assembles in 3D, checked on a generic tetrahedron (and a
    second one sharing its face 0) against exact sympy integration of polynomials: the
    mass, the lambda_k-weighted derivative terms D_j, the lambda_k-weighted face terms with
    the element's own basis on both sides and with the neighbour's basis as trial
    functions, and the outward unit normals."""
    sp = pytest.importorskip("sympy")
    x, y, z, s, t, r = sp.symbols("x y z s t r")
    X = np.array([[0.1, -0.2, 0.0], [1.3, 0.2, 0.1], [0.2, 1.1, -0.1], [0.3, 0.1, 0.9], [1.2, 1.0, 0.8]])
    cells = np.array([[0, 1, 2, 3], [4, 3, 2, 1]])
    mesh = Mesh(X, cells)
    assert mesh.nbr[0, 0] == 1 and np.all(mesh.detJ > 0)
    p = 2
    dg = TentDG(mesh, p)
    P = 1 + 2 * x - x * y + 0.5 * z ** 2 - y * z
    Q = 3 - x + 0.25 * y ** 2 + z + x * z

    def coef(F, e):
        nodes = X[cells[e, 0]] + reference_nodes(3, p) @ (X[cells[e, 1:]] - X[cells[e, 0]])
        V = basis(3, p).eval(reference_nodes(3, p))
        return np.linalg.solve(V, np.array([float(F.subs({x: a, y: b, z: c})) for a, b, c in nodes]))

    R = lambda v: sp.Rational(str(v))  # noqa: E731
    V0, V1, V2, V3 = [[R(c) for c in X[i]] for i in cells[0]]
    xm = [V0[i] + s * (V1[i] - V0[i]) + t * (V2[i] - V0[i]) + r * (V3[i] - V0[i]) for i in range(3)]
    detJ = abs(sp.Matrix([[V1[i] - V0[i] for i in range(3)], [V2[i] - V0[i] for i in range(3)],
                          [V3[i] - V0[i] for i in range(3)]]).det())
    lam = [1 - s - t - r, s, t, r]

    def tet_int(F):
        G = sp.expand(F.subs({x: xm[0], y: xm[1], z: xm[2]}, simultaneous=True) * detJ)
        return float(sp.integrate(G, (r, 0, 1 - s - t), (t, 0, 1 - s), (s, 0, 1)))

    cP, cQ = coef(P, 0), coef(Q, 0)
    cQn = coef(Q, 1)
    assert np.isclose(cP @ dg.mass(0) @ cQ, tet_int(P * Q), rtol=1e-12)
    for k in range(4):
        D = dg.vol(0, k)
        for j, var in enumerate((x, y, z)):
            assert np.isclose(cP @ D[j] @ cQ, tet_int(sp.diff(P, var) * Q * lam[k]), rtol=1e-12), (k, j)
        for f in range(4):
            if f == k:
                continue
            ids = [i for i in range(4) if i != f]
            A0, A1, A2 = ([R(c) for c in X[cells[0, i]]] for i in ids)
            xf = [A0[i] + s * (A1[i] - A0[i]) + t * (A2[i] - A0[i]) for i in range(3)]
            e1 = sp.Matrix([A1[i] - A0[i] for i in range(3)])
            e2 = sp.Matrix([A2[i] - A0[i] for i in range(3)])
            area2 = sp.sqrt(e1.cross(e2).dot(e1.cross(e2)))
            lam_f = {ids[0]: 1 - s - t, ids[1]: s, ids[2]: t}[k]

            def face_int(F):
                G = sp.expand(F.subs({x: xf[0], y: xf[1], z: xf[2]}, simultaneous=True) * lam_f)
                return float(sp.integrate(G, (t, 0, 1 - s), (s, 0, 1)) * area2)

            fc = dg.face(0, f, k)
            assert np.isclose(cP @ fc["Fself"] @ cQ, face_int(P * Q), rtol=1e-12), (k, f)
            if f == 0:   # the face shared with element 1: neighbour's basis as trial functions
                assert np.isclose(cP @ fc["Fcross"] @ cQn, face_int(P * Q), rtol=1e-12), (k, f)
            nrm = np.array([float(v) for v in e1.cross(e2)])
            nrm /= np.linalg.norm(nrm)
            mid = X[cells[0, ids]].mean(axis=0)
            assert abs(abs(fc["n"] @ nrm) - 1) < 1e-14 and (X[cells[0, f]] - mid) @ fc["n"] < 0
