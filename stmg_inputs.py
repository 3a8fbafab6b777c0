"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's
callers.  This module holds problem data only (right-hand sides, viscosity
fields, a manufactured solution) and none of the solver's arithmetic.

Vector layout (the library's ABI, Eq. (DefX) of the paper):
X = (V_1, P_1, ..., V_N, P_N); V_n = (V_n^1..V_n^{k+1}); V_n^a is
component-major over the global Gauss-Lobatto velocity nodes
(nn = n (r+1) + 1 per direction, x fastest); P_n^a is cell-major
(cells x fastest) over the C(r+d, d) Legendre modes of each cell.
"""
from math import comb

import numpy as np


def layout(d, n, r, k, N):
    nn = n * (r + 1) + 1
    nodes = nn ** d
    Mv = d * nodes
    Mp = n ** d * comb(r + d, d)
    slab = (k + 1) * (Mv + Mp)
    return dict(nn=nn, nodes=nodes, Mv=Mv, Mp=Mp, slab=slab, ndofs=N * slab)


def boundary_nodes(d, n, r):
    """Boolean per velocity node: True on the boundary of the unit cube."""
    nn = n * (r + 1) + 1
    g = np.arange(nn)
    onb = (g == 0) | (g == nn - 1)
    out = np.zeros([nn] * d, dtype=bool)          # axis order (x_{d-1}, ..., x_0)
    for j in range(d):
        shape = [1] * d
        shape[d - 1 - j] = nn
        out = out | onb.reshape(shape)
    return out.ravel()


def random_rhs(d, n, r, k, N, seed):
    """B = (F, 0): velocity entries i.i.d. U[-1,1] on interior velocity nodes,
    zero on Dirichlet nodes and on every pressure row (PCG64 stream)."""
    lay = layout(d, n, r, k, N)
    rng = np.random.Generator(np.random.PCG64(seed))
    b = np.zeros(lay["ndofs"])
    free = np.tile(~boundary_nodes(d, n, r), d)
    for s in range(N):
        for a in range(k + 1):
            o = s * lay["slab"] + a * lay["Mv"]
            vals = rng.uniform(-1.0, 1.0, lay["Mv"])
            b[o:o + lay["Mv"]] = np.where(free, vals, 0.0)
    return b


# ------------------------------------------------------------------ viscosity
class FourierViscosity:
    """nu(x) = exp(0.5 g(x)), g a random smooth Fourier series on [0,1]^3:
    g = sum_{m in {0..7}^3 \\ 0} (a_m cos 2 pi m.x + b_m sin 2 pi m.x) (1+|m|^2)^{-3/2},
    a, b ~ N(0,1) from the seed, rescaled so that max |g| = 1 over a 48^3 grid
    of the unit cube (so nu lies in about [e^-0.5, e^0.5]).  Evaluated as
    Re sum_m (a_m - i b_m) e^{2 pi i m.x}, contracted one axis at a time."""

    def __init__(self, seed, modes=8):
        rng = np.random.Generator(np.random.PCG64(seed))
        m = np.array([(i, j, l) for i in range(modes) for j in range(modes) for l in range(modes)
                      if (i, j, l) != (0, 0, 0)], dtype=int)
        self.modes = modes
        damp = (1.0 + np.sum(m * m, axis=1)) ** -1.5
        a = rng.standard_normal(len(m)) * damp
        b = rng.standard_normal(len(m)) * damp
        self.C = np.zeros((modes, modes, modes), dtype=complex)
        self.C[m[:, 0], m[:, 1], m[:, 2]] = a - 1j * b
        self.scale = 1.0
        g = np.linspace(0.0, 1.0, 48)
        pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
        self.scale = 1.0 / np.max(np.abs(self._g(pts)))

    def _g(self, x):
        x = np.asarray(x, float)
        out = np.empty(len(x))
        k = np.arange(self.modes)
        M = self.modes
        C0 = self.C.reshape(M, M * M)
        for s in range(0, len(x), 1 << 16):
            xs = x[s:s + (1 << 16)]
            E = [np.exp(2j * np.pi * xs[:, d])[:, None] ** k for d in range(3)]   # (P, M)
            t = (E[0] @ C0).reshape(-1, M, M)                                     # sum over m1
            t = np.einsum("pj,pjk->pk", E[1], t)                                  # sum over m2
            out[s:s + (1 << 16)] = self.scale * np.einsum("pk,pk->p", E[2], t).real
        return out

    def __call__(self, x):
        return np.exp(0.5 * self._g(x))


# --------------------------------------------------- manufactured solution
class Manufactured2D:
    """u = curl psi, psi = sin^2(pi x) sin^2(pi y) sin t; curl = (d_y, -d_x);
    p = sin t sin(pi x) cos(pi x) sin(pi y) cos(pi y); f = u_t - nu Lap u + grad p.
    The forcing is written out by hand below."""

    def __init__(self, nu=1.0):
        self.nu = nu

    def v(self, x, t):
        X, Y = np.pi * x[:, 0], np.pi * x[:, 1]
        u1 = np.pi * np.sin(X) ** 2 * np.sin(2 * Y) * np.sin(t)
        u2 = -np.pi * np.sin(2 * X) * np.sin(Y) ** 2 * np.sin(t)
        return np.stack([u1, u2], axis=1)

    def gradv(self, x, t):
        X, Y = np.pi * x[:, 0], np.pi * x[:, 1]
        st, pi = np.sin(t), np.pi
        g = np.zeros((len(X), 2, 2))
        g[:, 0, 0] = pi ** 2 * st * np.sin(2 * X) * np.sin(2 * Y)
        g[:, 0, 1] = 2 * pi ** 2 * st * np.sin(X) ** 2 * np.cos(2 * Y)
        g[:, 1, 0] = -2 * pi ** 2 * st * np.cos(2 * X) * np.sin(Y) ** 2
        g[:, 1, 1] = -pi ** 2 * st * np.sin(2 * X) * np.sin(2 * Y)
        return g

    def p(self, x, t):
        X, Y = np.pi * x[:, 0], np.pi * x[:, 1]
        return np.sin(t) * 0.25 * np.sin(2 * X) * np.sin(2 * Y)

    def f(self, x, t):
        X, Y = np.pi * x[:, 0], np.pi * x[:, 1]
        pi, nu = np.pi, self.nu
        st, ct = np.sin(t), np.cos(t)
        f1 = (ct * pi * np.sin(X) ** 2 * np.sin(2 * Y)
              - nu * 2 * pi ** 3 * st * np.sin(2 * Y) * (2 * np.cos(2 * X) - 1)
              + st * 0.5 * pi * np.cos(2 * X) * np.sin(2 * Y))
        f2 = (-ct * pi * np.sin(2 * X) * np.sin(Y) ** 2
              + nu * 2 * pi ** 3 * st * np.sin(2 * X) * (2 * np.cos(2 * Y) - 1)
              + st * 0.5 * pi * np.sin(2 * X) * np.cos(2 * Y))
        return np.stack([f1, f2], axis=1)


# ------------------------------------------------------------ lid-driven cavity
def lid_dirichlet(d, n, r, k, N, tau, t0, t_hat):
    """Dirichlet values of the lid-driven cavity for one slab (layout above):
    on the lid (the face x_{d-1} = 1, its edges included) the first velocity
    component is sin(pi t / 4), every other Dirichlet value is 0 (no-slip
    walls); free entries and pressure are 0.  Temporal dof a of subinterval
    s sits at t0 + tau (s + (t_hat[a] + 1) / 2), t_hat the DG(k) nodes on
    (-1, 1] (the caller supplies them)."""
    lay = layout(d, n, r, k, N)
    nn = lay["nn"]
    lid = np.zeros(lay["nodes"], dtype=bool)
    lid.reshape([nn] * d)[nn - 1] = True          # first axis is x_{d-1}
    g = np.zeros(lay["ndofs"])
    for s in range(N):
        for a in range(k + 1):
            t = t0 + tau * (s + 0.5 * (t_hat[a] + 1.0))
            o = s * lay["slab"] + a * lay["Mv"]
            g[o:o + lay["nodes"]] = np.where(lid, np.sin(np.pi * t / 4.0), 0.0)
    return g
