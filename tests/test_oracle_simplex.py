"""Pins of the oracle's reference-simplex pieces against closed forms."""
from math import comb, factorial

import numpy as np
import pytest

from mtp_inputs import meshes
from oracle.simplex import basis, exponents, quadrature, reference_nodes


@pytest.mark.parametrize("d", [1, 2, 3])
def test_quadrature_exact_on_monomials(d):
    # int over the unit simplex of x^a y^b z^c = a! b! c! / (a+b+c+d)!
    n = 5
    pts, w = quadrature(d, n)
    for e in exponents(d, 2 * n - 1):
        exact = np.prod([factorial(a) for a in e]) / factorial(sum(e) + d)
        approx = np.sum(w * np.prod(pts ** np.array(e), axis=1))
        assert abs(approx - exact) <= 1e-15 + 1e-13 * exact


@pytest.mark.parametrize("d,p", [(1, 3), (2, 1), (2, 3), (2, 5), (3, 1), (3, 3), (3, 5)])
def test_basis_orthonormal_and_complete(d, p):
    B = basis(d, p)
    assert B.n == comb(p + d, d)
    pts, w = quadrature(d, p + 3)
    Phi = B.eval(pts)
    G = Phi.T @ (w[:, None] * Phi)
    assert np.max(np.abs(G - np.eye(B.n))) < 1e-12
    # spans P_p: interpolation at the equispaced nodes (a unisolvent set) is invertible
    V = B.eval(reference_nodes(d, p))
    assert np.linalg.cond(V) < 1e6
    # each basis function is a polynomial of degree <= p: reproduced exactly by its
    # degree-p interpolant at random points
    xr = np.random.default_rng(1).dirichlet(np.ones(d + 1), size=20)[:, 1:]
    interp = B.eval(xr) @ np.linalg.solve(V, V)
    assert np.max(np.abs(interp - B.eval(xr))) < 1e-10


@pytest.mark.parametrize("d,p", [(2, 3), (3, 4)])
def test_basis_gradient_matches_central_differences(d, p):
    B = basis(d, p)
    x = np.random.default_rng(2).dirichlet(np.ones(d + 1), size=7)[:, 1:] * 0.9 + 0.02
    G = B.grad(x)
    h = 1e-6
    for g in range(d):
        dx = np.zeros(d)
        dx[g] = h
        fd = (B.eval(x + dx) - B.eval(x - dx)) / (2 * h)
        assert np.max(np.abs(fd - G[:, :, g])) < 1e-6 * max(1.0, np.max(np.abs(G)))


def test_reference_nodes_match_interchange_format():
    # the oracle's own node construction agrees with the documented format used for inputs
    for d, mk in [(2, lambda: meshes.square_tri(2)), (3, lambda: meshes.cube_kuhn(1))]:
        mesh = mk()
        for p in [1, 2, 4]:
            ref = reference_nodes(d, p)
            assert len(ref) == comb(p + d, d)
            X = mesh["coords"][mesh["cells"]]
            mine = X[:, :1, :] + np.einsum("nl,eld->end", ref, X[:, 1:, :] - X[:, :1, :])
            assert np.allclose(mine, meshes.equispaced_nodes(mesh, p), atol=1e-15)
