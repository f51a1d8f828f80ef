"""Pins of the oracle's tent pitcher against the pitching rule's definitions."""
import numpy as np
import pytest

from mtp_inputs import meshes
from oracle.mesh import Mesh
from oracle.pitch import QUANTUM, SAFETY, pitch, validate


@pytest.mark.parametrize("dim,n,sigma,T", [(2, 4, 0.5, 0.5), (2, 8, 0.5, 0.5), (3, 2, 0.125, 0.3), (3, 3, 0.125, 0.2)])
def test_structured_meshes_validate(dim, n, sigma, T):
    mm = meshes.cube_kuhn(n) if dim == 3 else meshes.square_tri(n)
    mesh = Mesh(mm["coords"], mm["cells"])
    tents = pitch(mesh, T, sigma=sigma)
    assert validate(mesh, tents, T, sigma=sigma)
    # all times are multiples of the quantum (or the end time)
    tt = tents["t_top"]
    on_grid = np.isclose(tt / QUANTUM, np.round(tt / QUANTUM), rtol=0, atol=1e-6)
    assert np.all(on_grid | (tt == T))
    # every vertex reaches the end time; its tents chain bottom-to-top
    for v in range(mesh.nv):
        sel = tents["vertex"] == v
        assert tents["t_bot"][sel][0] == 0.0 and tents["t_top"][sel][-1] == T
        assert np.all(tents["t_bot"][sel][1:] == tents["t_top"][sel][:-1])


def test_first_tents_by_hand():
    """Single right triangle (0,0),(1,0),(0,1), eps = mu = 1, sigma = 1/2.
    |grad lambda| = (sqrt2, 1, 1); the smallest sum over two of them is 2, so every edge
    step is k = 1/4.  Vertex 0 (smallest id on the flat front) rises to q(1/4), vertex 1
    to q(min(q(1/4), 0) + 1/4) = q(1/4), vertex 2 to q(q(1/4) + 1/4), with q the
    quantiser; the three tents share one element, so they sit in layers 0, 1, 2."""
    mesh = Mesh(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 1, 2]]))
    tents = pitch(mesh, 10.0, sigma=0.5)
    q = lambda t: QUANTUM * np.floor(t / QUANTUM - SAFETY)  # noqa: E731
    t0 = q(0.25)
    assert t0 == 0.25 - QUANTUM
    assert list(tents["vertex"][:4]) == [0, 1, 2, 0]
    assert list(tents["t_top"][:4]) == [t0, q(0.25), q(t0 + 0.25), q(t0 + 0.25)]
    assert list(tents["layer"][:4]) == [0, 1, 2, 3]


def test_layers_are_independent_sets():
    mm = meshes.square_tri(6)
    mesh = Mesh(mm["coords"], mm["cells"])
    tents = pitch(mesh, 0.4)
    for lay in np.unique(tents["layer"]):
        vs = tents["vertex"][tents["layer"] == lay]
        for a in vs:
            assert not np.isin(mesh.adj[int(a)], vs).any()


def test_jittered_mesh_terminates():
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(1)
    pts = np.concatenate([rng.uniform(0, 1, (60, 2)), np.array([[0, 0], [1, 0], [0, 1], [1, 1.0]])])
    cells = Delaunay(pts).simplices
    mm = {"coords": pts, "cells": meshes._orient(pts, cells.astype(np.int32))}
    mesh = Mesh(mm["coords"], mm["cells"])
    tents = pitch(mesh, 0.3, sigma=0.5)
    assert validate(mesh, tents, 0.3, sigma=0.5)
