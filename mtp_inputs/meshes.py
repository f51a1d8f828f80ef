"""Synthetic simplicial meshes (seeded, deterministic).

Every generator returns a dict with
  coords : float64 (nv, d)   vertex coordinates
  cells  : int32  (ne, d+1)  vertex ids of each simplex, positively oriented
Boundary-condition kinds are given per (element, local face); local face j is the face
opposite local vertex j.  The kind is only read for faces on the domain boundary.
"""
import itertools

import numpy as np

# boundary-condition kinds (same values as the C interface)
PEC, PMC, DATA = 0, 1, 2


def _orient(coords, cells):
    """Swap two vertices of negatively oriented simplices so every det J > 0."""
    X = coords[cells]
    J = X[:, 1:, :] - X[:, :1, :]
    det = np.linalg.det(J)
    bad = det < 0
    cells = cells.copy()
    cells[bad, 0], cells[bad, 1] = cells[bad, 1].copy(), cells[bad, 0].copy()
    return cells


def square_tri(n, length=1.0, origin=(0.0, 0.0)):
    """n x n squares on [ox, ox+L]^2, each split along its (0,0)-(1,1) diagonal."""
    h = length / n
    xs = origin[0] + h * np.arange(n + 1)
    ys = origin[1] + h * np.arange(n + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    coords = np.stack([X.ravel(), Y.ravel()], axis=1)
    vid = lambda i, j: j * (n + 1) + i  # noqa: E731
    cells = []
    for j in range(n):
        for i in range(n):
            v00, v10, v01, v11 = vid(i, j), vid(i + 1, j), vid(i, j + 1), vid(i + 1, j + 1)
            cells.append((v00, v10, v11))
            cells.append((v00, v11, v01))
    cells = np.asarray(cells, dtype=np.int32)
    return {"coords": coords, "cells": _orient(coords, cells)}


def cube_kuhn(n, length=1.0, axis_map=None):
    """n^3 cubes on [0,L]^3, each split into the 6 Kuhn (Freudenthal) tetrahedra that
    share the cube's main diagonal; conforming across cubes.

    axis_map, if given, maps the uniform lattice coordinate in [0, L] to a graded one
    (applied to each axis)."""
    g = np.linspace(0.0, length, n + 1)
    if axis_map is not None:
        g = axis_map(g)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def vid(i, j, k):
        return (i * (n + 1) + j) * (n + 1) + k

    steps = np.eye(3, dtype=np.int64)
    cells = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for perm in itertools.permutations(range(3)):
                    c = np.array([i, j, k])
                    tet = [vid(*c)]
                    for ax in perm:
                        c = c + steps[ax]
                        tet.append(vid(*c))
                    cells.append(tet)
    cells = np.asarray(cells, dtype=np.int32)
    return {"coords": coords, "cells": _orient(coords, cells)}


def graded_delaunay_cube(n=32, a=2.0 / 9.0, jitter=0.15, seed=11029):
    """(n+1)^3 lattice on the unit cube graded toward the corner 0 by x -> a x + (1-a) x^2
    per axis (h_max/h_min = (2-a)/a), interior points jittered by jitter*h_local
    (tangential only on faces, none on edges/corners), Delaunay-triangulated.
    Zero-volume simplices are dropped."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    u = np.linspace(0.0, 1.0, n + 1)
    g = a * u + (1.0 - a) * u * u
    hloc = np.gradient(g)
    I, J, K = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    idx = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    coords = g[idx]
    h = np.min(hloc[idx], axis=1)
    on_bnd = (idx == 0) | (idx == n)  # per axis: fixed coordinate
    delta = rng.uniform(-1.0, 1.0, size=coords.shape) * jitter * h[:, None]
    delta[on_bnd] = 0.0
    coords = coords + delta
    tri = Delaunay(coords, qhull_options="Qbb Qc Qz Q12")
    cells = tri.simplices.astype(np.int32)
    X = coords[cells]
    vol = np.abs(np.linalg.det(X[:, 1:, :] - X[:, :1, :])) / 6.0
    hmin = g[1] - g[0]
    cells = cells[vol > 1e-9 * hmin ** 3]
    return {"coords": coords, "cells": _orient(coords, cells)}


def uniform_bc(ne, dim, kind):
    """Per (element, local face) boundary kind array, all faces of one kind."""
    return np.full((ne, dim + 1), kind, dtype=np.int32)


def element_centroids(mesh):
    return mesh["coords"][mesh["cells"]].mean(axis=1)


def materials_split(mesh, eps_right=2.25, x_split=0.5):
    """eps = eps_right where the element centroid has x > x_split, else 1; mu = 1."""
    c = element_centroids(mesh)
    eps = np.where(c[:, 0] > x_split, eps_right, 1.0)
    mu = np.ones(len(eps))
    return eps, mu


def equispaced_nodes(mesh, p):
    """Physical coordinates of the documented equispaced nodes, shape (ne, Np, d).

    Node order (the interchange format of nodal fields): reference coordinates
    (i/p, j/p[, k/p]) with i fastest, then j, then k, restricted to i+j(+k) <= p;
    x = v0 + sum_l xhat_l (v_l - v0) with v the element's vertices in cell order."""
    d = mesh["coords"].shape[1]
    pts = []
    if d == 2:
        for j in range(p + 1):
            for i in range(p + 1 - j):
                pts.append((i / p, j / p))
    else:
        for k in range(p + 1):
            for j in range(p + 1 - k):
                for i in range(p + 1 - j - k):
                    pts.append((i / p, j / p, k / p))
    ref = np.asarray(pts)
    X = mesh["coords"][mesh["cells"]]  # (ne, d+1, d)
    J = X[:, 1:, :] - X[:, :1, :]      # rows = v_l - v0
    return X[:, :1, :] + np.einsum("nl,eld->end", ref, J)


def fan_disk(nfan, radius=1.0, rings=2):
    """Disk of the given radius around a centre vertex of valence nfan: `rings` rings of
    nfan vertices (ring r at radius r/rings, every other ring rotated by half a sector),
    the centre joined to the first ring, neighbouring rings joined by strips of 2 nfan
    triangles.  The centre's patch holds nfan triangles."""
    coords = [(0.0, 0.0)]
    for r in range(1, rings + 1):
        off = 0.5 * (r % 2 == 0)
        for i in range(nfan):
            a = 2.0 * np.pi * (i + off) / nfan
            coords.append((radius * r / rings * np.cos(a), radius * r / rings * np.sin(a)))
    coords = np.asarray(coords)
    vid = lambda r, i: 1 + (r - 1) * nfan + (i % nfan)  # noqa: E731
    cells = [(0, vid(1, i), vid(1, i + 1)) for i in range(nfan)]
    for r in range(1, rings):
        for i in range(nfan):
            if r % 2 == 1:   # outer ring r+1 is rotated forward by half a sector
                cells.append((vid(r, i), vid(r + 1, i), vid(r, i + 1)))
                cells.append((vid(r, i + 1), vid(r + 1, i), vid(r + 1, i + 1)))
            else:            # outer ring r+1 is aligned with ring r - 1, behind ring r
                cells.append((vid(r, i), vid(r + 1, i + 1), vid(r, i + 1)))
                cells.append((vid(r, i), vid(r + 1, i), vid(r + 1, i + 1)))
    cells = np.asarray(cells, dtype=np.int32)
    return {"coords": coords, "cells": _orient(coords, cells)}


def disk_tri(n, radius=1.0):
    """Disk of the given radius: the centre and n rings, ring k (k = 1..n) holding 6k vertices
    at radius k/n * radius (angles 2 pi j / (6k)); consecutive rings are joined by walking
    both by angle and closing, at every step, the triangle whose new vertex comes first.
    6 n^2 triangles, 3 n (n + 1) + 1 vertices; boundary = ring n."""
    coords = [(0.0, 0.0)]
    start = [0]
    for k in range(1, n + 1):
        start.append(len(coords))
        for j in range(6 * k):
            a = 2.0 * np.pi * j / (6 * k)
            coords.append((radius * k / n * np.cos(a), radius * k / n * np.sin(a)))
    coords = np.asarray(coords)
    cells = []
    # centre fan
    for j in range(6):
        cells.append((0, start[1] + j, start[1] + (j + 1) % 6))
    for k in range(1, n):
        ni, no = 6 * k, 6 * (k + 1)
        i = o = 0
        while i < ni or o < no:
            ai = (i + 1) / ni   # angle (in turns) of the next inner vertex
            ao = (o + 1) / no
            vi, vo = start[k] + i % ni, start[k + 1] + o % no
            if o < no and (i >= ni or ao <= ai):
                cells.append((vi, vo, start[k + 1] + (o + 1) % no))
                o += 1
            else:
                cells.append((vi, vo, start[k] + (i + 1) % ni))
                i += 1
    cells = np.asarray(cells, dtype=np.int32)
    return {"coords": coords, "cells": _orient(coords, cells)}


def p2_geometry(mesh, on_circle=None):
    """Quadratic (P2) geometry nodes per triangle, shape (ne, 6, 2): the three vertices in
    cell order, then the midpoints of edges (0,1), (1,2), (0,2).  With on_circle = R, the
    midpoint of every edge whose two vertices lie on the circle |x| = R is moved onto the
    circle (at the mean angle of its ends), which curves the elements along the boundary;
    every other midpoint stays straight.  Without it, every element is affine."""
    X = mesh["coords"][mesh["cells"]]
    mids = [(0, 1), (1, 2), (0, 2)]
    geo = np.zeros((len(X), 6, 2))
    geo[:, :3] = X
    for s, (a, b) in enumerate(mids):
        m = 0.5 * (X[:, a] + X[:, b])
        if on_circle is not None:
            ra = np.linalg.norm(X[:, a], axis=1)
            rb = np.linalg.norm(X[:, b], axis=1)
            bnd = (np.abs(ra - on_circle) < 1e-12 * on_circle) & (np.abs(rb - on_circle) < 1e-12 * on_circle)
            m[bnd] = on_circle * m[bnd] / np.linalg.norm(m[bnd], axis=1)[:, None]
        geo[:, 3 + s] = m
    return geo


def equispaced_nodes_p2(geo, p):
    """Physical coordinates of the documented equispaced nodes on quadratic triangles
    (geo from p2_geometry), shape (ne, Np, 2): the reference nodes (i/p, j/p), i fastest,
    mapped by x = sum_i G_i N_i with the P2 Lagrange shape functions (vertices
    l_v (2 l_v - 1), edge midpoints 4 l_a l_b, l the barycentric coordinates)."""
    pts = np.array([(i / p, j / p) for j in range(p + 1) for i in range(p + 1 - j)])
    L = np.stack([1.0 - pts[:, 0] - pts[:, 1], pts[:, 0], pts[:, 1]], axis=1)
    N = np.stack([L[:, 0] * (2 * L[:, 0] - 1), L[:, 1] * (2 * L[:, 1] - 1), L[:, 2] * (2 * L[:, 2] - 1),
                  4 * L[:, 0] * L[:, 1], 4 * L[:, 1] * L[:, 2], 4 * L[:, 0] * L[:, 2]], axis=1)
    return np.einsum("ni,eix->enx", N, np.asarray(geo, dtype=np.float64))
