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

Pins (tests/test_oracle_curved.py): the map interpolates its nodes and, with straight
midpoints, has the constant affine Jacobian; physical gradients through J^{-T} match the
closed-form gradient of a polynomial pulled back by a curved map; a curved disk's area
converges at fourth order (straight edges: second); M_{1/J} is exact on affine elements,
SPD, and its defect ||M_{1/J} M_J - I|| falls as the square of the curvature amplitude;
the exact projection reproduces the discrete space; the three recoveries agree where K is
constant and the weight-adjusted one tracks the exact one to second order in the
curvature.
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
    uq = np.stack([np.linalg.solve(Kq[i], wq[i]) for i in range(len(pts))])
    rhs = Phi.T @ ((w * dJ)[:, None] * uq)
    return Minv @ rhs
