"""Pins of the oracle's mesh topology and affine geometry (the conforming simplicial mesh
and vertex patches of section 2): face matching, Euler characteristic, patch sizes,
volumes, barycentric gradients and outward face normals."""
from math import factorial

import numpy as np
import pytest

from mtp_inputs import meshes
from oracle.mesh import Mesh


def _mesh(kind, n):
    if kind == "square":
        return Mesh(**{k: v for k, v in meshes.square_tri(n).items()})
    if kind == "kuhn":
        return Mesh(**{k: v for k, v in meshes.cube_kuhn(n).items()})
    if kind == "graded":
        return Mesh(**{k: v for k, v in meshes.cube_kuhn(n, axis_map=lambda g: 0.25 * g + 0.75 * g * g).items()})
    if kind == "fan":
        return Mesh(**{k: v for k, v in meshes.fan_disk(n).items()})
    return Mesh(**{k: v for k, v in meshes.graded_delaunay_cube(n=n, a=1.0, jitter=0.3, seed=3).items()})


def _faces(m):
    """Every (d-1)-face as a sorted vertex tuple -> number of elements holding it."""
    cnt = {}
    for c in m.cells:
        for j in range(m.d + 1):
            key = tuple(sorted(int(v) for k, v in enumerate(c) if k != j))
            cnt[key] = cnt.get(key, 0) + 1
    return cnt


CASES = [("square", 4), ("kuhn", 3), ("graded", 3), ("fan", 12), ("delaunay", 3)]


@pytest.mark.parametrize("kind,n", CASES)
def test_faces_shared_by_at_most_two_and_neighbours_symmetric(kind, n):
    m = _mesh(kind, n)
    cnt = _faces(m)
    assert set(cnt.values()) <= {1, 2}
    n_interior = sum(1 for c in cnt.values() if c == 2)
    assert (m.nbr >= 0).sum() == 2 * n_interior        # each interior face seen from both sides
    for e in range(m.ne):
        for j in range(m.d + 1):
            e2 = m.nbr[e, j]
            if e2 >= 0:
                assert e in m.nbr[e2]
                shared = set(m.cells[e]) - {m.cells[e, j]}
                assert shared <= set(m.cells[e2])


@pytest.mark.parametrize("kind,n", CASES)
def test_euler_characteristic_of_a_ball(kind, n):
    """V - E + F (- T) = 1 for a triangulated disk / ball."""
    m = _mesh(kind, n)
    edges = {tuple(sorted((int(a), int(b)))) for c in m.cells for a in c for b in c if a < b}
    if m.d == 2:
        chi = m.nv - len(edges) + m.ne
    else:
        faces = _faces(m)
        chi = m.nv - len(edges) + len(faces) - m.ne
    assert chi == 1


def test_patch_sizes_of_structured_meshes():
    sq = _mesh("square", 4)
    sizes = np.array([len(p) for p in sq.v2e])
    interior = [v for v in range(sq.nv) if 0 < sq.coords[v, 0] < 1 and 0 < sq.coords[v, 1] < 1]
    assert np.all(sizes[interior] == 6) and sizes.sum() == 3 * sq.ne
    cube = _mesh("kuhn", 3)
    sizes = np.array([len(p) for p in cube.v2e])
    x = cube.coords
    interior = np.all((x > 0) & (x < 1), axis=1)
    assert np.all(sizes[interior] == 24) and sizes.sum() == 4 * cube.ne
    # the 6 Kuhn tets of a cube are the 6 monotone lattice paths from (0,0,0) to (1,1,1):
    # the diagonal's ends lie on all 6, every other corner of the cube on 2
    corner = np.all((x == 0) | (x == 1), axis=1)
    on_diag = np.all(x == 0, axis=1) | np.all(x == 1, axis=1)
    assert np.all(sizes[corner & on_diag] == 6) and np.all(sizes[corner & ~on_diag] == 2)
    fan = _mesh("fan", 12)
    assert len(fan.v2e[0]) == 12


@pytest.mark.parametrize("kind,n,total", [("square", 4, 1.0), ("kuhn", 3, 1.0), ("graded", 3, 1.0),
                                          ("delaunay", 3, 1.0), ("fan", 12, 3.0)])
def test_volumes_positive_and_sum_to_the_domain(kind, n, total):
    m = _mesh(kind, n)
    v = m.volume()
    assert np.all(m.detJ > 0) and np.all(v > 0)
    assert abs(v.sum() - total) < 1e-12
    # volume from the vertices directly (independent of detJ's sign convention)
    X = m.coords[m.cells]
    direct = np.abs(np.linalg.det(X[:, 1:] - X[:, :1])) / factorial(m.d)
    assert np.allclose(v, direct, rtol=1e-14)


@pytest.mark.parametrize("kind,n", CASES)
def test_barycentric_gradients(kind, n):
    """grad lambda_k . (x_j - x_0) = delta_kj - delta_k0, and the gradients sum to zero."""
    m = _mesh(kind, n)
    X = m.coords[m.cells]
    dX = X - X[:, :1]                                    # (ne, d+1, d)
    G = np.einsum("ekx,ejx->ekj", m.grad_lam, dX)
    want = np.eye(m.d + 1)                               # row k, column j
    want[0, :] -= 1.0
    assert np.allclose(G, want[None], atol=1e-12)
    assert np.allclose(m.grad_lam.sum(axis=1), 0.0, atol=1e-10 * np.abs(m.grad_lam).max())
    # barycentric coordinates of the vertices are the unit vectors
    for e in (0, m.ne // 2, m.ne - 1):
        assert np.allclose(m.barycentric(e, X[e]), np.eye(m.d + 1), atol=1e-12)
