"""Mesh topology and affine element geometry for the oracle (section "Mesh generation
by tent pitching": conforming simplicial mesh, vertex patches omega_V).

Pins: tests/test_oracle_mesh.py (every interior face has exactly two elements, Euler
characteristic of the structured meshes, patch sizes, volumes sum to the domain's).
"""
from collections import defaultdict

import numpy as np


class Mesh:
    def __init__(self, coords, cells, eps=None, mu=None, face_bc=None):
        self.coords = np.asarray(coords, dtype=np.float64)
        self.cells = np.asarray(cells, dtype=np.int64)
        self.ne, nvert = self.cells.shape
        self.d = nvert - 1
        self.nv = self.coords.shape[0]
        self.eps = np.ones(self.ne) if eps is None else np.asarray(eps, dtype=np.float64)
        self.mu = np.ones(self.ne) if mu is None else np.asarray(mu, dtype=np.float64)
        self.face_bc = (np.zeros((self.ne, self.d + 1), dtype=np.int64) if face_bc is None
                        else np.asarray(face_bc, dtype=np.int64))
        d = self.d
        X = self.coords[self.cells]                       # (ne, d+1, d)
        self.X = X
        self.J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))   # columns v_l - v_0
        self.detJ = np.linalg.det(self.J)
        self.Jinv = np.linalg.inv(self.J)                 # rows = grad lambda_l, l>=1
        gl = np.empty((self.ne, d + 1, d))
        gl[:, 1:, :] = self.Jinv
        gl[:, 0, :] = -self.Jinv.sum(axis=1)
        self.grad_lam = gl                                 # grad of barycentric coords

        # neighbours across local faces (face j is opposite local vertex j)
        key_to = {}
        self.nbr = -np.ones((self.ne, d + 1), dtype=np.int64)
        for e in range(self.ne):
            for j in range(d + 1):
                key = tuple(sorted(int(v) for k, v in enumerate(self.cells[e]) if k != j))
                if key in key_to:
                    e2, j2 = key_to.pop(key)
                    self.nbr[e, j] = e2
                    self.nbr[e2, j2] = e
                else:
                    key_to[key] = (e, j)

        self.v2e = defaultdict(list)                       # vertex patch omega_V
        for e in range(self.ne):
            for v in self.cells[e]:
                self.v2e[int(v)].append(e)
        self.v2e = [np.asarray(self.v2e[v], dtype=np.int64) for v in range(self.nv)]
        adj = [set() for _ in range(self.nv)]
        for c in self.cells:
            for a in c:
                for b in c:
                    if a != b:
                        adj[int(a)].add(int(b))
        self.adj = [np.asarray(sorted(s), dtype=np.int64) for s in adj]

    def volume(self):
        from math import factorial
        return np.abs(self.detJ) / factorial(self.d)

    def barycentric(self, e, x):
        """Barycentric coordinates of physical points x (npts, d) in element e."""
        xh = (x - self.X[e, 0]) @ self.Jinv[e].T
        return np.concatenate([1.0 - xh.sum(axis=1, keepdims=True), xh], axis=1)

    def to_ref(self, e, x):
        return (x - self.X[e, 0]) @ self.Jinv[e].T

    def to_phys(self, e, xh):
        return self.X[e, 0] + xh @ self.J[e].T
