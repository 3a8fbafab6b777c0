"""Structured meshes of the unit square/cube (test infrastructure).

n^d cells, each the image of the reference cell [0,1]^d under the standard
multilinear map T_K of its 2^d vertices (Sec. 2.2).  Vertices may be displaced
by x_i += amp * prod_j sin(2 pi x_j) for every coordinate i (reading G16);
boundary vertices do not move.  Numbering is lexicographic with direction 0
(x) fastest for cells, vertices and the global Gauss-Lobatto velocity nodes.
"""
from itertools import product

import numpy as np


class Mesh:
    def __init__(self, d, n, amp=0.0):
        self.d, self.n, self.amp = d, n, float(amp)
        g = np.linspace(0.0, 1.0, n + 1)
        pts = np.array(list(product(*([g] * d))))[:, ::-1]  # x fastest
        if amp != 0.0:
            s = np.prod(np.sin(2.0 * np.pi * pts), axis=1)
            pts = pts + amp * s[:, None]
        self.vertices = pts  # ((n+1)^d, d)
        self.n_cells = n ** d

    def cell_coords(self, c):
        """Integer coordinates (c_0, ..., c_{d-1}) of cell index c."""
        return [(c // self.n ** j) % self.n for j in range(self.d)]

    def cell_vertices(self, c):
        """(2^d, d) vertex coordinates of cell c, local vertex v = sum v_j 2^j."""
        cc = self.cell_coords(c)
        out = np.zeros((2 ** self.d, self.d))
        for v in range(2 ** self.d):
            idx = sum((cc[j] + ((v >> j) & 1)) * (self.n + 1) ** j for j in range(self.d))
            out[v] = self.vertices[idx]
        return out

    def map(self, c, xi):
        """Physical points x(xi) and Jacobians J[p, i, j] = dx_i/dxi_j."""
        X = self.cell_vertices(c)
        xi = np.atleast_2d(xi)
        npnt, d = xi.shape[0], self.d
        x = np.zeros((npnt, d))
        J = np.zeros((npnt, d, d))
        for v in range(2 ** d):
            bits = [(v >> j) & 1 for j in range(d)]
            N = np.ones(npnt)
            dN = np.ones((npnt, d))
            for j in range(d):
                f = xi[:, j] if bits[j] else 1.0 - xi[:, j]
                df = 1.0 if bits[j] else -1.0
                N = N * f
                for g in range(d):
                    dN[:, g] *= df if g == j else f
            x += N[:, None] * X[v][None, :]
            J += X[v][None, :, None] * dN[:, None, :]
        return x, J


class VelocityDofs:
    """Global continuous Q_{r+1} node grid: nn = n (r+1) + 1 nodes per
    direction, node index sum g_j nn^j; cell c, local node i -> global node."""

    def __init__(self, mesh, r):
        self.mesh, self.r = mesh, r
        self.Q = r + 2
        self.q = r + 1
        self.nn = mesh.n * self.q + 1
        self.n_nodes = self.nn ** mesh.d
        d, Q = mesh.d, self.Q
        self.cell_nodes = np.zeros((mesh.n_cells, Q ** d), dtype=np.int64)
        for c in range(mesh.n_cells):
            cc = mesh.cell_coords(c)
            for i in range(Q ** d):
                ii = [(i // Q ** j) % Q for j in range(d)]
                self.cell_nodes[c, i] = sum((cc[j] * self.q + ii[j]) * self.nn ** j for j in range(d))
        gidx = np.array([[(m // self.nn ** j) % self.nn for j in range(d)] for m in range(self.n_nodes)])
        self.boundary = np.any((gidx == 0) | (gidx == self.nn - 1), axis=1)
        self.valence = np.bincount(self.cell_nodes.ravel(), minlength=self.n_nodes)
