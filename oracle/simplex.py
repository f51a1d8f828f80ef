"""Reference simplex for the oracle: quadrature, an orthonormal modal basis and the
documented equispaced interchange nodes.

Reference d-simplex: {xhat_l >= 0, sum_l xhat_l <= 1}, vertices 0, e_1, ..., e_d.
Pins (tests/test_oracle_simplex.py): quadrature is exact on monomials against the
closed form  int xhat^a yhat^b zhat^c = a! b! c! / (a+b+c+d)!;  the basis is orthonormal
and spans all polynomials of degree <= p; gradients match the exact derivative of the
Legendre expansion checked by central differences.
"""
from functools import lru_cache
from math import comb

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import roots_jacobi


def _jacobi01(n, alpha):
    """n-point Gauss-Jacobi rule on [0,1] for the weight (1-u)^alpha."""
    x, w = roots_jacobi(n, alpha, 0.0)
    return (x + 1.0) / 2.0, w / 2.0 ** (alpha + 1)


@lru_cache(maxsize=None)
def quadrature(d, n):
    """Collapsed-coordinate (Duffy) rule on the reference d-simplex with n points per
    direction; exact for polynomials of total degree <= 2n-1.

    d=1: x = u;  d=2: x = u, y = (1-u) v;  d=3: x = u, y = (1-u) v, z = (1-u)(1-v) w,
    with the Jacobian (1-u)^(d-1) (1-v)^(d-2) absorbed into Gauss-Jacobi weights.
    Returns (points (nq, d), weights (nq,)) summing to 1/d!."""
    if d == 1:
        u, wu = _jacobi01(n, 0.0)
        return u[:, None], wu
    if d == 2:
        u, wu = _jacobi01(n, 1.0)
        v, wv = _jacobi01(n, 0.0)
        U, V = np.meshgrid(u, v, indexing="ij")
        W = np.outer(wu, wv)
        pts = np.stack([U.ravel(), ((1 - U) * V).ravel()], axis=1)
        return pts, W.ravel()
    if d == 3:
        u, wu = _jacobi01(n, 2.0)
        v, wv = _jacobi01(n, 1.0)
        w, ww = _jacobi01(n, 0.0)
        U, V, Wc = np.meshgrid(u, v, w, indexing="ij")
        Wt = wu[:, None, None] * wv[None, :, None] * ww[None, None, :]
        pts = np.stack([U.ravel(), ((1 - U) * V).ravel(), ((1 - U) * (1 - V) * Wc).ravel()], axis=1)
        return pts, Wt.ravel()
    raise ValueError("d must be 1, 2 or 3")


def exponents(d, p):
    """Multi-indices (a_1..a_d) with total degree <= p, in a fixed order."""
    out = []
    if d == 1:
        out = [(a,) for a in range(p + 1)]
    elif d == 2:
        out = [(a, b) for s in range(p + 1) for b in range(s + 1) for a in [s - b]]
    else:
        out = [(a, b, c) for s in range(p + 1) for c in range(s + 1) for b in range(s - c + 1) for a in [s - b - c]]
    assert len(out) == comb(p + d, d)
    return out


def _leg(x, n, der=0):
    """Legendre polynomial P_n(2x-1) (or its derivative w.r.t. x) at points x."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    if der:
        c = npleg.legder(c) * 2.0
    return npleg.legval(2.0 * x - 1.0, c)


class ModalBasis:
    """Orthonormal modal basis of P_p on the reference d-simplex.

    Raw functions psi_k(x) = prod_l P_{a_l}(2 xhat_l - 1) (Legendre products of total
    degree <= p, a basis of P_p); phi = L^{-1} psi with G = L L^T the Gram matrix of psi
    computed with an exact quadrature rule, so that (phi_a, phi_b) = delta_ab."""

    def __init__(self, d, p):
        self.d, self.p = d, p
        self.exps = exponents(d, p)
        self.n = len(self.exps)
        pts, w = quadrature(d, p + 2)
        Psi = self._raw(pts)
        # Cholesky orthonormalisation, applied twice (the second pass removes the
        # rounding left by the first on the ill-conditioned raw Gram matrix)
        self.Linv = np.eye(self.n)
        for _ in range(2):
            Phi = Psi @ self.Linv.T
            G = Phi.T @ (w[:, None] * Phi)
            L = np.linalg.cholesky(G)
            self.Linv = np.linalg.solve(L, self.Linv)

    def _raw(self, x):
        x = np.atleast_2d(x)
        out = np.ones((x.shape[0], self.n))
        for k, e in enumerate(self.exps):
            for l in range(self.d):
                out[:, k] *= _leg(x[:, l], e[l])
        return out

    def _raw_grad(self, x):
        x = np.atleast_2d(x)
        out = np.ones((x.shape[0], self.n, self.d))
        for k, e in enumerate(self.exps):
            for g in range(self.d):
                for l in range(self.d):
                    out[:, k, g] *= _leg(x[:, l], e[l], der=int(l == g))
        return out

    def eval(self, x):
        """phi_a(x) for reference points x (npts, d) -> (npts, n)."""
        return self._raw(x) @ self.Linv.T

    def grad(self, x):
        """Reference gradient d phi_a / d xhat_g -> (npts, n, d)."""
        return np.einsum("ab,qbg->qag", self.Linv, self._raw_grad(x))


@lru_cache(maxsize=None)
def basis(d, p):
    return ModalBasis(d, p)


def reference_nodes(d, p):
    """The documented equispaced interchange nodes in reference coordinates:
    (i/p, j/p[, k/p]), i fastest, then j, then k, with i+j(+k) <= p."""
    pts = []
    if d == 1:
        pts = [(i / p,) for i in range(p + 1)]
    elif d == 2:
        for j in range(p + 1):
            for i in range(p + 1 - j):
                pts.append((i / p, j / p))
    else:
        for k in range(p + 1):
            for j in range(p + 1 - k):
                for i in range(p + 1 - j - k):
                    pts.append((i / p, j / p, k / p))
    return np.asarray(pts, dtype=np.float64)
