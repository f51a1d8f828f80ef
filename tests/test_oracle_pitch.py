"""Pins of the oracle's tent pitcher against the pitching rule's definitions."""
import numpy as np
import pytest

from mtp_inputs import meshes
from oracle.mesh import Mesh
from oracle.pitch import QUANTUM, SAFETY, greedy_colouring, pitch, validate


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


def _valid(mm, T=0.3):
    mesh = Mesh(mm["coords"], mm["cells"])
    tents = pitch(mesh, T, sigma=0.5)
    assert validate(mesh, tents, T)
    return mesh, {k: v.copy() for k, v in tents.items()}, T


def _last_tent_of(tents, v):
    return int(np.where(tents["vertex"] == v)[0][-1])


def test_validate_rejects_over_tall_tent():
    """A tent raised to 2.5x its height breaks the slope bound (the vertex's later tents
    shifted with it, so only the slope can fail)."""
    mesh, t, T = _valid(meshes.square_tri(4))
    v = 12                                        # an interior vertex
    i = int(np.where(t["vertex"] == v)[0][0])     # its first tent
    dh = 1.5 * (t["t_top"][i] - t["t_bot"][i])
    later = np.where((t["vertex"] == v) & (np.arange(len(t["vertex"])) > i))[0]
    t["t_top"][i] += dh
    t["t_bot"][later[0]] += dh
    with pytest.raises(AssertionError, match="slope bound"):
        validate(mesh, t, T)


def test_validate_rejects_overlapping_patches_in_a_layer():
    """Two neighbouring vertices' tents put in one layer: their patches share elements."""
    mesh, t, T = _valid(meshes.square_tri(4))
    a = int(np.where(t["vertex"] == 12)[0][0])
    b = int(np.where(t["vertex"] == 13)[0][0])
    assert 13 in mesh.adj[12]
    t["layer"][b] = t["layer"][a]
    with pytest.raises(AssertionError):
        validate(mesh, t, T)


def test_validate_rejects_wrong_layer_order():
    """A tent moved to a layer before one it depends on (its own vertex's previous tent)."""
    mesh, t, T = _valid(meshes.square_tri(4))
    idx = np.where(t["vertex"] == 12)[0]
    t["layer"][idx[1]] = t["layer"][idx[0]] - 1
    with pytest.raises(AssertionError):
        validate(mesh, t, T)


def test_validate_rejects_non_flat_final_front():
    """The last tent of one vertex dropped: the final front is not flat at T."""
    mesh, t, T = _valid(meshes.square_tri(4))
    keep = np.ones(len(t["vertex"]), bool)
    keep[_last_tent_of(t, 5)] = False
    t = {k: v[keep] for k, v in t.items()}
    with pytest.raises(AssertionError, match="flat"):
        validate(mesh, t, T)


def test_validate_rejects_non_positive_height_and_bottom_mismatch():
    mesh, t, T = _valid(meshes.square_tri(4))
    i = int(np.where(t["vertex"] == 7)[0][0])
    bad = {k: v.copy() for k, v in t.items()}
    bad["t_top"][i] = bad["t_bot"][i]
    with pytest.raises(AssertionError, match="height"):
        validate(mesh, bad, T)
    bad = {k: v.copy() for k, v in t.items()}
    bad["t_bot"][i] += 1e-3
    with pytest.raises(AssertionError, match="bottom"):
        validate(mesh, bad, T)


def test_validate_rejects_steep_front_on_a_graded_two_material_mesh():
    """The slope bound is sigma sqrt(eps mu) (slope 1/(2c)): a table pitched for eps = 16
    on half of a graded mesh (waves 4x slower, fronts 4x steeper allowed there) is valid for
    that mesh and fails the slope bound when validated against eps = 1 everywhere.  (The
    edge rule stays well inside the bound, so a factor 2.25 would not show.)"""
    mm = meshes.cube_kuhn(3, axis_map=lambda g: 0.3 * g + 0.7 * g * g)
    eps, mu = meshes.materials_split(mm, eps_right=16.0)
    slow = Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    unit = Mesh(mm["coords"], mm["cells"])
    t = pitch(slow, 0.2, sigma=0.5)
    assert validate(slow, t, 0.2)
    with pytest.raises(AssertionError, match="slope bound"):
        validate(unit, t, 0.2)


# ---- the colour rule ------------------------------------------------------------------

def _colour_meshes():
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(1)
    pts = np.concatenate([rng.uniform(0, 1, (60, 2)), np.array([[0, 0], [1, 0], [0, 1], [1, 1.0]])])
    jit = {"coords": pts, "cells": meshes._orient(pts, Delaunay(pts).simplices.astype(np.int32))}
    graded = meshes.cube_kuhn(3, axis_map=lambda g: 0.3 * g + 0.7 * g * g)
    return {"square6": (meshes.square_tri(6), None), "disk6": (meshes.disk_tri(6), None),
            "fan12": (meshes.fan_disk(12), None), "jittered": (jit, None), "kuhn3": (meshes.cube_kuhn(3), None),
            "graded3_eps": (graded, meshes.materials_split(graded))}


@pytest.mark.parametrize("name", ["square6", "disk6", "fan12", "jittered", "kuhn3", "graded3_eps"])
def test_colour_rule_validates(name):
    mm, mat = _colour_meshes()[name]
    eps, mu = mat if mat else (None, None)
    mesh = Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    T = 0.3
    tents = pitch(mesh, T, sigma=0.5, rule="colour")
    assert validate(mesh, tents, T, sigma=0.5)
    for v in range(mesh.nv):
        sel = tents["vertex"] == v
        assert tents["t_bot"][sel][0] == 0.0 and tents["t_top"][sel][-1] == T


def test_greedy_colouring_is_proper_and_greedy():
    """Adjacent vertices differ; a vertex of colour c sees every colour below c on an
    earlier neighbour (what the greedy rule in id order produces, and nothing else)."""
    for mm in (meshes.disk_tri(5), meshes.cube_kuhn(3), meshes.fan_disk(9)):
        mesh = Mesh(mm["coords"], mm["cells"])
        col = greedy_colouring(mesh)
        for v in range(mesh.nv):
            nb = np.asarray(mesh.adj[v])
            assert np.all(col[nb] != col[v])
            earlier = set(col[nb[nb < v]].tolist())
            assert set(range(col[v])) <= earlier
        # the greedy bound: at most one colour more than the largest vertex degree
        assert col.max() + 1 <= max(len(a) for a in mesh.adj) + 1


@pytest.mark.parametrize("rule", ["min_vertex", "colour"])
def test_tent_tops_are_tight_against_an_edge(rule):
    """Every move goes as far as the constraints allow, up to the quantiser: a tent top is
    either t_end or within 2Q of the tightest of tau_w + k_vw over the neighbours w at that
    moment and, for the colour rule, the pole cap tau_v + 1.5 min_w k_vw (the fronts replayed
    in emission order; the constraints read from the element steps)."""
    mm = meshes.disk_tri(4)
    mesh = Mesh(mm["coords"], mm["cells"])
    T = 0.2
    tents = pitch(mesh, T, sigma=0.5, rule=rule)
    norms = np.linalg.norm(mesh.grad_lam, axis=2)
    k_T = 0.5 / (norms.sum(axis=1, keepdims=True) - norms).min(axis=1)
    tau = np.zeros(mesh.nv)
    capped = 0
    for v, tb, tt in zip(tents["vertex"], tents["t_bot"], tents["t_top"]):
        assert tau[v] == tb
        k_vw = [min(k_T[e] for e in mesh.v2e[v] if w in mesh.cells[e]) for w in mesh.adj[v]]
        if rule == "colour":
            assert tt - tb <= 1.5 * min(k_vw) * (1 + 1e-12)
        if tt != T:
            lim = min(tau[w] + k for w, k in zip(mesh.adj[v], k_vw))
            if rule == "colour" and tb + 1.5 * min(k_vw) < lim:
                lim = tb + 1.5 * min(k_vw)
                capped += 1
            assert tt <= lim and tt + 2 * QUANTUM > lim
        tau[v] = tt
    if rule == "colour":
        assert capped > 0      # the cap is active on this mesh


def test_colour_rule_by_hand():
    """Unit square split along (1,0)-(0,1): triangles [0,1,2], [1,3,2], every edge step 1/4
    (right isosceles, legs 1), pole cap 3/8.  Greedy colours 0,1,2,0: vertices 0 and 3 share
    colour 0 and rise together to q(1/4) in layer 0, where the minimum-vertex rule serialises
    0, 1, 2, 3; vertex 1 follows to q(1/4); vertex 2, with every neighbour at q(1/4), would
    reach q(q(1/4) + 1/4) but the cap holds it at q(3/8); then 0 and 3 rise to q(q(1/4) + 1/4)
    (the edge to vertex 1, below q(3/8) + 1/4 and the cap q(1/4) + 3/8)."""
    X = np.array([[0, 0], [1, 0], [0, 1], [1, 1.0]])
    mesh = Mesh(X, np.array([[0, 1, 2], [1, 3, 2]]))
    q = lambda t: QUANTUM * np.floor(t / QUANTUM - SAFETY)  # noqa: E731
    t0 = q(0.25)
    assert list(greedy_colouring(mesh)) == [0, 1, 2, 0]
    c = pitch(mesh, 10.0, sigma=0.5, rule="colour")
    assert list(c["vertex"][:6]) == [0, 3, 1, 2, 0, 3]
    assert list(c["t_top"][:6]) == [t0, t0, t0, q(0.375), q(t0 + 0.25), q(t0 + 0.25)]
    assert list(c["layer"][:6]) == [0, 0, 1, 2, 3, 3]
    m = pitch(mesh, 10.0, sigma=0.5)
    assert list(m["vertex"][:4]) == [0, 1, 2, 3] and list(m["layer"][:4]) == [0, 1, 2, 3]


def test_colour_rule_widens_layers_on_the_disk():
    """The minimum-vertex order serialises an irregular disk; the colour turns give layers a
    colour class wide, with fewer tents (each move spans more of the causal step)."""
    mm = meshes.disk_tri(8)
    mesh = Mesh(mm["coords"], mm["cells"])
    a = pitch(mesh, 0.2)
    b = pitch(mesh, 0.2, rule="colour")
    assert validate(mesh, b, 0.2)
    assert b["layer"].max() + 1 < (a["layer"].max() + 1) / 5
    assert len(b["vertex"]) < len(a["vertex"])


def test_unknown_rule_refused():
    mm = meshes.square_tri(2)
    with pytest.raises(ValueError):
        pitch(Mesh(mm["coords"], mm["cells"]), 0.1, rule="random")


@pytest.mark.parametrize("name,expected", [("disk6", "colour"), ("graded3_eps", "min_vertex"), ("square6", "colour")])
def test_auto_rule_picks_the_table_with_less_work(name, expected):
    """rule="auto": both orderings, and the table whose tents' patch sizes sum to less; the
    work is recounted here from the patch sizes (the disk and square favour the colour order,
    the graded two-media cube the minimum vertex)."""
    mm, mat = _colour_meshes()[name]
    eps, mu = mat if mat else (None, None)
    mesh = Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    T = 0.3
    t = pitch(mesh, T, sigma=0.5, rule="auto")
    a = pitch(mesh, T, sigma=0.5)
    b = pitch(mesh, T, sigma=0.5, rule="colour")
    sizes = np.bincount(np.asarray(mm["cells"]).ravel(), minlength=mesh.nv)
    wa, wb = sizes[a["vertex"]].sum(), sizes[b["vertex"]].sum()
    assert t["rule"] == expected == ("colour" if wb < wa else "min_vertex")
    ref = b if expected == "colour" else a
    for k in ("vertex", "t_bot", "t_top", "layer"):
        assert np.array_equal(t[k], ref[k]), k
    assert validate(mesh, t, T)
