"""Curved (quadratic) triangles for the oracle: the geometry map, the tent quantities on a
curved element, and the step that turns the mapped variable w into the field u with the
exact or an approximate inverse of the curved mass matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper basis: section 4 (structure-aware Taylor time-stepping), the passage after the
coercivity proof.  Instead of solving the Galerkin system M_i U = Y of the sub-interval
start, the field is recovered pointwise from the mapped variable in closed form and then
projected into the discrete space; on uncurved elements that projection only needs the
(diagonal, in an orthonormal basis) mass inverse, and on the few curved elements the paper
uses an approximation of the exact inverse mass matrix without saying which.

Readings (the paper is silent on all of them):
  * geometry: isoparametric quadratic triangles, x(xh) = sum_i G_i N_i(xh) with the P2
    Lagrange shape functions N_i and nodes G_i (vertices, then the midpoints of the edges
    (0,1), (1,2), (0,2));
  * fronts on a curved element stay P1 in reference coordinates: the hat function of local
    vertex k is lambda_k(x) = lambdahat_k(xh(x)), so grad phi = J^{-T} sum_k tau_k
    gradhat lambdahat_k varies inside the element;
  * the projection is the L2 projection of the physical element (weight |det J|);
  * the approximate inverse: the weight-adjusted one (Chan, Hewett and Warburton,
    "Weight-adjusted discontinuous Galerkin methods: curvilinear meshes", SIAM J. Sci.
    Comput. 2017), M_J^{-1} ~= Mhat^{-1} M_{1/J} Mhat^{-1}, which in the orthonormal
    reference basis (Mhat = I) is M_{1/J}[b, a] = int phi_b phi_a / |det J| dxh.  It is
    exact for affine elements, symmetric positive definite, local, and needs only the
    reference basis and |det J| at quadrature points.

The three ways to get the field U from the tested integrals Y of one element
(Y_b = int_T phi_b (g(u) - f(u) grad phi) dx, component by component):
  galerkin        solve M_i U = Y with M_i[b, a] = int_T phi_b K(b(x)) phi_a dx
  project_exact   w = M_J^{-1} Y;  u(x) = K(b(x))^{-1} w(x) pointwise;  U = M_J^{-1} int phi u
  project_wadg    the same with both M_J^{-1} replaced by M_{1/J}
On an affine element, or wherever K is constant on the element, all three agree.

The curved tent solve (CurvedMesh, CurvedTentDG, CurvedSolver below) runs the tents of
oracle/tent.py with every integral taken with the element map's Jacobian at quadrature
points, and a pitcher step that bounds the hat-function gradients over each curved element.

Pins (tests/test_oracle_curved.py): the map interpolates its nodes and, with straight
midpoints, has the constant affine Jacobian; physical gradients through J^{-T} match the
closed-form gradient of a polynomial pulled back by a curved map; a curved disk's area
converges at fourth order (straight edges: second); M_{1/J} is exact on affine elements,
SPD, and its defect ||M_{1/J} M_J - I|| falls as the square of the curvature amplitude;
the exact projection reproduces the discrete space; the three recoveries agree where K is
constant and the weight-adjusted one tracks the exact one to second order in the
curvature.  The curved tent solve equals the affine oracle (oracle/tent.py) on a
straight-sided mesh for all three recoveries; on the disk with quadratic boundary elements
it converges to a circular-cavity mode (Bessel) at the optimal order p + 1 while the
straight-sided disk stalls near order 1.5; the weight-adjusted scheme tracks the Galerkin
one far below the discretisation error; the curved pitcher keeps every front's slope within
the causality bound on a denser sample.
"""
import numpy as np

from .simplex import basis, quadrature

# barycentric coordinates of the reference triangle and their (constant) gradients
_GL = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
_EDGES = [(0, 1), (1, 2), (0, 2)]


def _bary(xh):
    xh = np.atleast_2d(xh)
    return np.stack([1.0 - xh[:, 0] - xh[:, 1], xh[:, 0], xh[:, 1]], axis=1)


def shape_p2(xh):
    """P2 Lagrange shape functions N_i at reference points -> (npts, 6): vertices
    lambda_v (2 lambda_v - 1), then edge midpoints 4 lambda_a lambda_b."""
    L = _bary(xh)
    out = [L[:, v] * (2.0 * L[:, v] - 1.0) for v in range(3)]
    out += [4.0 * L[:, a] * L[:, b] for a, b in _EDGES]
    return np.stack(out, axis=1)


def shape_p2_grad(xh):
    """Reference gradients dN_i/dxh_l -> (npts, 6, 2)."""
    L = _bary(xh)
    g = [(4.0 * L[:, v] - 1.0)[:, None] * _GL[v][None, :] for v in range(3)]
    g += [4.0 * (L[:, a][:, None] * _GL[b][None, :] + L[:, b][:, None] * _GL[a][None, :]) for a, b in _EDGES]
    return np.stack(g, axis=1)


class CurvedTriangle:
    """One quadratic triangle with geometry nodes G (6, 2)."""

    def __init__(self, G):
        self.G = np.asarray(G, dtype=np.float64)
        assert self.G.shape == (6, 2)

    def map(self, xh):
        """x(xh) = sum_i G_i N_i(xh) -> (npts, 2)."""
        return shape_p2(xh) @ self.G

    def jac(self, xh):
        """J[q, r, l] = d x_r / d xh_l at the points -> (npts, 2, 2)."""
        return np.einsum("qil,ir->qrl", shape_p2_grad(xh), self.G)

    def detj(self, xh):
        return np.linalg.det(self.jac(xh))

    def grad_lambda(self, xh):
        """Physical gradients of the hat functions lambda_k(x) = lambdahat_k(xh(x)) at the
        points: J^{-T} gradhat lambdahat_k -> (npts, 3, 2)."""
        Jinv = np.linalg.inv(self.jac(xh))                 # (q, l, r)
        return np.einsum("qlr,kl->qkr", Jinv, _GL)


def _quad(p, extra):
    return quadrature(2, p + extra)


def mass_weighted(el, p, weight, extra=2):
    """M_w[b, a] = int_That phi_b phi_a weight(xh) dxh for the orthonormal reference basis;
    weight is a function of the reference points."""
    pts, w = _quad(p, extra)
    Phi = basis(2, p).eval(pts)
    return Phi.T @ ((w * weight(pts))[:, None] * Phi)


def mass_J(el, p):
    """The curved element's mass matrix M_J = int phi_b phi_a |det J| dxh (|det J| is a
    quadratic polynomial, so p + 2 points per direction integrate it exactly)."""
    return mass_weighted(el, p, lambda x: np.abs(el.detj(x)), extra=2)


def mass_invJ(el, p, extra=8):
    """M_{1/J} = int phi_b phi_a / |det J| dxh: the weight-adjusted approximation of
    M_J^{-1} in the orthonormal reference basis (1/|det J| is not a polynomial: extra
    points beyond the basis degree)."""
    return mass_weighted(el, p, lambda x: 1.0 / np.abs(el.detj(x)), extra=extra)


def project(el, p, fun, inverse="exact", extra=8):
    """L2 projection onto P_p of the physical element of fun(xh) (values (npts, nc) at
    reference points): U = Minv int phi fun |det J|, Minv = M_J^{-1} ("exact") or M_{1/J}
    ("wadg").  Returns modal coefficients (nb, nc)."""
    pts, w = _quad(p, extra)
    Phi = basis(2, p).eval(pts)
    f = np.atleast_2d(fun(pts))
    if f.shape[0] != len(pts):
        f = f.T
    rhs = Phi.T @ ((w * np.abs(el.detj(pts)))[:, None] * f)
    if inverse == "exact":
        return np.linalg.solve(mass_J(el, p), rhs)
    if inverse == "wadg":
        return mass_invJ(el, p) @ rhs
    raise ValueError(inverse)


def front_gradient(el, tau_b, tau_t, th):
    """grad phi(x, th) at reference points as a function: phi = (1 - th) phi_b + th phi_t,
    phi_b = sum_k tau_b[k] lambda_k (P1 in reference coordinates)."""
    tau = (1.0 - th) * np.asarray(tau_b, dtype=np.float64) + th * np.asarray(tau_t, dtype=np.float64)
    return lambda xh: np.einsum("k,qkr->qr", tau, el.grad_lambda(xh))


def recover(el, p, system, Y, gphi, eps, mu, how, extra=8):
    """The field coefficients U (nb, nc) of one element from its tested integrals Y (nb, nc)
    at a time where grad phi = gphi(xh):
      "galerkin": M_i U = Y, M_i = int phi_b K(b(x)) phi_a dx (componentwise blocks);
      "exact" / "wadg": w = Minv Y, u = K(b)^{-1} w pointwise, U = Minv int phi u dx.
    K(b) = g - f(.) b is the system's mass-form matrix (K(b) u = g(u) - f(u) b)."""
    B = basis(2, p)
    nb, nc = B.n, system.nc
    pts, w = _quad(p, extra)
    Phi = B.eval(pts)
    dJ = np.abs(el.detj(pts))
    bq = gphi(pts)
    Kq = np.stack([system.K(b, eps, mu) for b in bq])          # (q, nc, nc)
    if how == "galerkin":
        # M_i[(c, b), (c', a)] = int phi_b K[c, c'] phi_a |det J|
        Mi = np.einsum("q,qb,qcd,qa->cbda", w * dJ, Phi, Kq, Phi).reshape(nc * nb, nc * nb)
        return np.linalg.solve(Mi, Y.T.reshape(-1)).reshape(nc, nb).T
    if how not in ("exact", "wadg"):
        raise ValueError(how)
    Minv = np.linalg.inv(mass_J(el, p)) if how == "exact" else mass_invJ(el, p, extra)
    W = Minv @ Y                                                 # (nb, nc): coefficients of w
    wq = Phi @ W                                                 # (q, nc)
    uq = np.linalg.solve(Kq, wq[:, :, None])[:, :, 0]
    rhs = Phi.T @ ((w * dJ)[:, None] * uq)
    return Minv @ rhs


# ==================================================================== curved tent solve
# The tent evolution of oracle/tent.py on a mesh whose elements may be quadratic: every
# integral by quadrature with the element map's Jacobian at the points, the tent map's
# grad phi varying inside an element, curved boundary faces with pointwise normals.  The
# recovery of the field from the tested integrals is "galerkin" (solve M_i U = Y: what the
# affine oracle does), "exact" (the paper's pointwise inverse, then the L2 projection with
# the exact curved mass inverse) or "wadg" (the same with the weight-adjusted inverse M_{1/J},
# used then for every mass inverse: the element mass is taken as M_{1/J}^{-1} throughout, so
# the scheme stays consistent and energy-stable).  PEC / PMC walls only (no data faces).

_REF_V = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])


class CurvedMesh:
    """Topology of the straight-sided mesh (neighbours, patches, adjacency from
    oracle.mesh.Mesh) with one quadratic map per element, geo (ne, 6, 2) whose first three
    nodes are the element's vertices in cell order."""

    def __init__(self, coords, cells, geo, eps=None, mu=None, face_bc=None):
        from .mesh import Mesh
        self.base = Mesh(coords, cells, eps, mu, face_bc)
        b = self.base
        self.d, self.ne, self.nv = b.d, b.ne, b.nv
        self.cells, self.nbr, self.v2e, self.adj = b.cells, b.nbr, b.v2e, b.adj
        self.eps, self.mu, self.face_bc = b.eps, b.mu, b.face_bc
        assert self.d == 2
        geo = np.asarray(geo, dtype=np.float64)
        assert np.allclose(geo[:, :3], b.X, atol=1e-14), "geometry vertices must follow the cells"
        self.el = [CurvedTriangle(G) for G in geo]
        # curved: some midpoint node differs from the straight edge midpoint
        mids = 0.5 * (b.X[:, [0, 1, 0]] + b.X[:, [1, 2, 2]])
        scale = np.abs(b.X).max(axis=(1, 2))[:, None, None] + 1.0
        self.curved = np.any(np.abs(geo[:, 3:] - mids) > 1e-14 * scale, axis=(1, 2))

    def step_bounds(self, sigma, n=12):
        """Per-element pitching step.  Straight elements: the affine rule's k_T.  Curved
        elements: sigma sqrt(eps mu) / max over the barycentric lattice (i/n, j/n), i + j <= n,
        of min_i sum_{j != i} |grad lambda_j(x)| (the affine bound taken pointwise)."""
        b = self.base
        norms = np.linalg.norm(b.grad_lam, axis=2)
        k = sigma * np.sqrt(self.eps * self.mu) / (norms.sum(axis=1, keepdims=True) - norms).min(axis=1)
        pts = np.array([(i / n, j / n) for j in range(n + 1) for i in range(n + 1 - j)])
        for e in np.nonzero(self.curved)[0]:
            nrm = np.linalg.norm(self.el[e].grad_lambda(pts), axis=2)   # (q, 3)
            s = (nrm.sum(axis=1, keepdims=True) - nrm).min(axis=1)      # min_i sum_{j!=i}
            k[e] = sigma * np.sqrt(self.eps[e] * self.mu[e]) / s.max()
        return k

    def to_ref(self, e, x, xh0=None):
        """Reference points of physical points x in element e (Newton on the map)."""
        el = self.el[e]
        xh = self.base.to_ref(e, x) if xh0 is None else np.array(xh0, dtype=np.float64)
        for _ in range(30):
            r = el.map(xh) - x
            if np.max(np.abs(r)) < 1e-15 * (1.0 + np.max(np.abs(x))):
                break
            xh = xh - np.einsum("qlr,qr->ql", np.linalg.inv(el.jac(xh)), r)
        return xh


REF_NODES6 = np.array([[0, 0], [1, 0], [0, 1], [0.5, 0], [0.5, 0.5], [0, 0.5]], dtype=np.float64)


class CurvedTentDG:
    def __init__(self, mesh, p, alpha=0.5, recovery="galerkin", extra=4):
        from .maxwell import System
        self.mesh, self.p, self.alpha, self.recovery = mesh, p, alpha, recovery
        self.sys = System(2)
        self.nc = 3
        self.B = basis(2, p)
        self.nb = self.B.n
        self.qv_pts, self.qv_w = quadrature(2, p + extra)
        self.Phi_v = self.B.eval(self.qv_pts)
        self.Grad_v = self.B.grad(self.qv_pts)
        self.qf_s, self.qf_w = quadrature(1, p + extra)
        self.lam_v = _bary(self.qv_pts)                       # lambdahat_k at the points
        self._geo, self._mass, self._minv, self._vol, self._face = {}, {}, {}, {}, {}

    # ---------------------------------------------------------------- element data
    def geo(self, e):
        """|det J|, physical basis gradients (q, b, x) and hat-function gradients (q, k, x)
        at the volume quadrature points of element e."""
        if e not in self._geo:
            el = self.mesh.el[e]
            J = el.jac(self.qv_pts)
            Jinv = np.linalg.inv(J)                               # (q, l, r)
            dj = np.abs(np.linalg.det(J))
            gphys = np.einsum("qbl,qlr->qbr", self.Grad_v, Jinv)
            self._geo[e] = (dj, gphys, el.grad_lambda(self.qv_pts))
        return self._geo[e]

    def mass(self, e):
        """The element's scalar mass: M_J, or M_{1/J}^{-1} for the weight-adjusted scheme."""
        if e not in self._mass:
            el = self.mesh.el[e]
            if self.recovery == "wadg":
                self._mass[e] = np.linalg.inv(mass_invJ(el, self.p))
            else:
                self._mass[e] = mass_J(el, self.p)
        return self._mass[e]

    def minv(self, e):
        if e not in self._minv:
            el = self.mesh.el[e]
            self._minv[e] = mass_invJ(el, self.p) if self.recovery == "wadg" else np.linalg.inv(mass_J(el, self.p))
        return self._minv[e]

    def vol(self, e, k):
        """D[j][b, a] = int_T lambda_k d_j phi_b phi_a (physical derivative j)."""
        key = (e, k)
        if key not in self._vol:
            dj, gphys, _ = self.geo(e)
            w = self.qv_w * dj * self.lam_v[:, k]
            self._vol[key] = np.einsum("q,qbj,qa->jba", w, gphys, self.Phi_v)
        return self._vol[key]

    def face(self, e, f, k):
        """Quadrature data of local face f of element e (opposite local vertex f): points,
        weights times the surface measure, outward unit normals, lambda_k, the element's
        basis, and the neighbour's basis at the same physical points."""
        key = (e, f, k)
        if key in self._face:
            return self._face[key]
        m = self.mesh
        el = m.el[e]
        a, b = [i for i in range(3) if i != f]
        s = self.qf_s[:, 0]
        xh = _REF_V[a][None, :] + s[:, None] * (_REF_V[b] - _REF_V[a])[None, :]
        x = el.map(xh)
        tang = np.einsum("qrl,l->qr", el.jac(xh), _REF_V[b] - _REF_V[a])
        meas = np.linalg.norm(tang, axis=1)
        n = np.stack([tang[:, 1], -tang[:, 0]], axis=1) / meas[:, None]
        inward = el.map(np.array([[1.0 / 3.0, 1.0 / 3.0]]))[0] - x
        sign = np.where(np.einsum("qr,qr->q", n, inward) > 0, -1.0, 1.0)
        n = n * sign[:, None]
        out = {"n": n, "w": self.qf_w * meas, "lam": _bary(xh)[:, k], "phi_e": self.B.eval(xh)}
        nb = m.nbr[e, f]
        if nb >= 0:
            out["phi_n"] = self.B.eval(m.to_ref(nb, x))
        self._face[key] = out
        return out

    # ---------------------------------------------------------------- tent operators
    def tent(self, tau, v, t_top):
        m, sys, nc = self.mesh, self.sys, self.nc
        es = m.v2e[v]
        ks = [int(np.where(m.cells[e] == v)[0][0]) for e in es]
        pos = {int(e): i for i, e in enumerate(es)}
        H = t_top - tau[v]
        tau_t = tau.copy()
        tau_t[v] = t_top
        T = {"es": es, "ks": ks, "H": H, "A": {}, "gphi_b": [], "gphi_t": [], "mass": [], "eps": [], "mu": []}
        I = np.eye(nc)
        for i, (e, k) in enumerate(zip(es, ks)):
            _, _, gl = self.geo(e)
            T["gphi_b"].append(np.einsum("k,qkr->qr", tau[m.cells[e]], gl))
            T["gphi_t"].append(np.einsum("k,qkr->qr", tau_t[m.cells[e]], gl))
            T["mass"].append(np.kron(I, self.mass(e)))
            T["eps"].append(m.eps[e])
            T["mu"].append(m.mu[e])
            D = self.vol(e, k)
            Aee = sum(np.kron(sys.Aj[j], H * D[j]) for j in range(2))
            for f in range(3):
                if f == k:
                    continue   # the face opposite V lies on the patch boundary: delta = 0
                fc = self.face(e, f, k)
                nb = m.nbr[e, f]
                wl = H * fc["w"] * fc["lam"]
                kind = int(m.face_bc[e, f])
                if nb < 0 and kind not in (0, 1):
                    raise ValueError("curved oracle: walls only")
                cross = np.zeros((nc * self.nb, nc * self.nb))
                for q in range(len(wl)):
                    Bi, Bo = sys.flux_matrices(fc["n"][q], self.alpha, None)
                    Fs = wl[q] * np.outer(fc["phi_e"][q], fc["phi_e"][q])
                    if nb >= 0:
                        Aee = Aee - np.kron(Bi, Fs)
                        cross -= np.kron(Bo, wl[q] * np.outer(fc["phi_e"][q], fc["phi_n"][q]))
                    else:
                        R = sys.ghost_matrix(kind)
                        Aee = Aee - np.kron(Bi + Bo @ R, Fs)
                if nb >= 0:
                    j = pos[int(nb)]
                    T["A"][(i, j)] = T["A"].get((i, j), 0.0) + cross
            T["A"][(i, i)] = T["A"].get((i, i), 0.0) + Aee
        return T

    def _Kq(self, T, i, th):
        b = (1.0 - th) * T["gphi_b"][i] + th * T["gphi_t"][i]
        return np.stack([self.sys.K(bq, T["eps"][i], T["mu"][i]) for bq in b])

    def M_of(self, T, th):
        """M(th) per element: int phi_b K(b(x, th))_{cd} phi_a, block (c, b), (d, a)."""
        out = []
        for i, e in enumerate(T["es"]):
            dj, _, _ = self.geo(e)
            Kq = self._Kq(T, i, th)
            M = np.einsum("q,qb,qcd,qa->cbda", self.qv_w * dj, self.Phi_v, Kq, self.Phi_v)
            out.append(M.reshape(self.nc * self.nb, self.nc * self.nb))
        return out

    def Mprime(self, T):
        """dM/dth: int phi_b (-A(grad phi_t - grad phi_b)) phi_a."""
        out = []
        for i, e in enumerate(T["es"]):
            dj, _, _ = self.geo(e)
            bp = T["gphi_t"][i] - T["gphi_b"][i]
            Aq = np.stack([-self.sys.A(x) for x in bp])
            M = np.einsum("q,qb,qcd,qa->cbda", self.qv_w * dj, self.Phi_v, Aq, self.Phi_v)
            out.append(M.reshape(self.nc * self.nb, self.nc * self.nb))
        return out

    def recover(self, T, i, th, Mi, Yv):
        """U from the tested integrals Yv (component-major) of patch element i at th."""
        if self.recovery == "galerkin":
            return np.linalg.solve(Mi, Yv)
        e = T["es"][i]
        nb, nc = self.nb, self.nc
        dj, _, _ = self.geo(e)
        Minv = self.minv(e)
        W = Minv @ Yv.reshape(nc, nb).T                 # (nb, nc): coefficients of w
        wq = self.Phi_v @ W
        Kq = self._Kq(T, i, th)
        uq = np.linalg.solve(Kq, wq[:, :, None])[:, :, 0]     # K(b(x_q))^{-1} w(x_q)
        U = Minv @ (self.Phi_v.T @ ((self.qv_w * dj)[:, None] * uq))
        return U.T.reshape(-1)

    def apply_A(self, T, U):
        out = [np.zeros(self.nc * self.nb) for _ in T["es"]]
        for (i, j), blk in T["A"].items():
            out[i] += blk @ U[j]
        return out

    def sat(self, T, Y, q, m):
        """q-stage SAT on m sub-intervals, the sub-interval start and the correction
        recovered by self.recovery."""
        from math import factorial
        Mp = self.Mprime(T)
        ne = len(T["es"])
        for i in range(m):
            th = i / m
            Mi = self.M_of(T, th)
            U = [self.recover(T, e, th, Mi[e], Y[e]) for e in range(ne)]
            Ys = [Y]
            for n in range(1, q + 1):
                Yn = self.apply_A(T, U)
                Ys.append(Yn)
                if n <= q - 1:
                    U = [self.recover(T, e, th, Mi[e], Yn[e] - n * (Mp[e] @ U[e])) for e in range(ne)]
            Y = [sum(Ys[n][e] / (m ** n * factorial(n)) for n in range(q + 1)) for e in range(ne)]
        return Y


class CurvedSolver:
    """Tents layer by layer on a curved mesh (the state per element: modal coefficients of
    w in the basis orthonormal on the reference element)."""

    def __init__(self, mesh, p, q, m, alpha=0.5, recovery="galerkin"):
        self.mesh, self.p, self.q, self.m = mesh, p, q, m
        self.dg = CurvedTentDG(mesh, p, alpha=alpha, recovery=recovery)
        self.nc, self.nb = 3, self.dg.nb
        self.tau = np.zeros(mesh.nv)
        self.cw = np.zeros((mesh.ne, self.nc * self.nb))

    def set_exact(self, exact, t0=0.0):
        """w = g(u) of the exact fields on the flat front t0, projected element by element
        (exact projection; the weight-adjusted inverse for the "wadg" scheme)."""
        self.tau[:] = t0
        dg = self.dg
        for e in range(self.mesh.ne):
            el = self.mesh.el[e]
            g = dg.sys.g_diag(self.mesh.eps[e], self.mesh.mu[e])
            fun = lambda xh: exact.u(el.map(xh), t0) * g[None, :]   # noqa: E731
            U = project(el, self.p, fun, "wadg" if dg.recovery == "wadg" else "exact")
            self.cw[e] = U.T.reshape(-1)

    def set_nodal_u(self, u_nodal, t0=0.0):
        """Fields u on a flat front as nodal values (ne, Np, nc) at the documented equispaced
        nodes mapped through each element's map: w = g(u) interpolated there."""
        from .simplex import reference_nodes
        self.tau[:] = t0
        V = self.dg.B.eval(reference_nodes(2, self.p))
        Vinv = np.linalg.inv(V)
        for e in range(self.mesh.ne):
            g = self.dg.sys.g_diag(self.mesh.eps[e], self.mesh.mu[e])
            w = np.asarray(u_nodal[e], dtype=np.float64) * g[None, :]
            self.cw[e] = (Vinv @ w).T.reshape(-1)

    def nodal_w(self):
        from .simplex import reference_nodes
        V = self.dg.B.eval(reference_nodes(2, self.p))
        c = self.cw.reshape(self.mesh.ne, self.nc, self.nb)
        return np.einsum("ab,ecb->eac", V, c)

    def run_tent(self, v, t_top):
        dg = self.dg
        T = dg.tent(self.tau, v, t_top)
        Y = [T["mass"][i] @ self.cw[e] for i, e in enumerate(T["es"])]
        Y = dg.sat(T, Y, self.q, self.m)
        for i, e in enumerate(T["es"]):
            self.cw[e] = np.linalg.solve(T["mass"][i], Y[i])
        self.tau[v] = t_top

    def run(self, tents):
        for i in np.argsort(tents["layer"], kind="stable"):
            self.run_tent(int(tents["vertex"][i]), float(tents["t_top"][i]))

    def l2_error(self, exact, t):
        """Spatial L2 error of all components on a flat front at t (u = w / g there)."""
        dg = self.dg
        pts, w = quadrature(2, self.p + 5)
        Phi = dg.B.eval(pts)
        err2 = ref2 = 0.0
        for e in range(self.mesh.ne):
            el = self.mesh.el[e]
            g = dg.sys.g_diag(self.mesh.eps[e], self.mesh.mu[e])
            uq = (Phi @ self.cw[e].reshape(self.nc, self.nb).T) / g[None, :]
            ue = exact.u(el.map(pts), t)
            ww = w * np.abs(el.detj(pts))
            err2 += np.sum(ww[:, None] * (uq - ue) ** 2)
            ref2 += np.sum(ww[:, None] * ue ** 2)
        return np.sqrt(err2), np.sqrt(ref2)


def max_front_slope(mesh, tents, n=12):
    """Replay a tent list on a curved mesh and return the largest ratio
    |grad phi(x)| / sqrt(eps mu) over every front met and the points of a degree-n rule
    (a denser sample than the one step_bounds uses) of every element of the moved patch."""
    pts = quadrature(2, n)[0]
    gl = [el.grad_lambda(pts) for el in mesh.el]
    tau = np.zeros(mesh.nv)
    worst = 0.0
    for i in np.argsort(tents["layer"], kind="stable"):
        v = int(tents["vertex"][i])
        tau[v] = tents["t_top"][i]
        for e in mesh.v2e[v]:
            g = np.einsum("k,qkr->qr", tau[mesh.cells[e]], gl[e])
            worst = max(worst, np.linalg.norm(g, axis=1).max() / np.sqrt(mesh.eps[e] * mesh.mu[e]))
    return worst
