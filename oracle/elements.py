"""Reference-element data (test infrastructure; see oracle/__init__.py).

Space: velocity Q_{r+1} with Lagrange basis at the r+2 Gauss-Lobatto points of
[0,1] in each direction (basis choice not stated in the paper; reading G18),
pressure P_r^disc spanned by products of shifted Legendre polynomials of total
degree <= r on the reference cell [0,1]^d (Sec. 2.2, Eq. (Def:VKQK); the
"mapped" variant, reading G5).

Time: DG(k) with Lagrange basis at the right-sided (k+1)-point Gauss-Radau
points of [-1,1] (Sec. 3.1, Eq. (GF), (BasYk)); temporal matrices from
Eq. (DefKMC).
"""
from itertools import product
from math import comb

import numpy as np
from numpy.polynomial import legendre as npleg


# ----------------------------------------------------------------- 1D rules
def gauss_01(n):
    """n-point Gauss-Legendre rule mapped to [0,1] (points, weights)."""
    x, w = npleg.leggauss(n)
    return (x + 1.0) / 2.0, w / 2.0


def gauss_m11(n):
    """n-point Gauss-Legendre rule on [-1,1]."""
    return npleg.leggauss(n)


def gauss_lobatto_01(n):
    """n >= 2 Gauss-Lobatto points on [0,1]: the end points and the roots of
    P'_{n-1} (textbook definition)."""
    if n < 2:
        raise ValueError("Gauss-Lobatto needs at least two points")
    c = np.zeros(n)
    c[n - 1] = 1.0
    inner = npleg.legroots(npleg.legder(c)) if n > 2 else np.array([])
    x = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    return (x + 1.0) / 2.0


def radau_right(k):
    """Right-sided (k+1)-point Gauss-Radau rule on [-1,1], Eq. (GF).

    The points are the roots of P_k - P_{k+1} (they include t=+1); the weights
    are fixed by exactness on the monomials 1, t, ..., t^k (moment equations).
    """
    n = k + 1
    c = np.zeros(n + 1)
    c[k] += 1.0
    c[k + 1] -= 1.0
    t = np.sort(np.real(npleg.legroots(c)))
    t[-1] = 1.0
    V = np.vander(t, n, increasing=True).T           # V[j, i] = t_i^j
    mom = np.array([(1.0 - (-1.0) ** (j + 1)) / (j + 1) for j in range(n)])
    w = np.linalg.solve(V, mom)
    return t, w


# ------------------------------------------------------- Lagrange 1D bases
def lagrange_values(nodes, pts):
    """L[p, i] = ell_i(pts[p]) for the Lagrange basis on `nodes`."""
    nodes = np.asarray(nodes, float)
    pts = np.atleast_1d(np.asarray(pts, float))
    n = len(nodes)
    L = np.ones((len(pts), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                L[:, i] *= (pts - nodes[j]) / (nodes[i] - nodes[j])
    return L


def lagrange_derivs(nodes, pts):
    """D[p, i] = ell_i'(pts[p]) (product rule, term by term)."""
    nodes = np.asarray(nodes, float)
    pts = np.atleast_1d(np.asarray(pts, float))
    n = len(nodes)
    D = np.zeros((len(pts), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(pts), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (pts - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += term
    return D


# ------------------------------------------------------ pressure P_r basis
def pressure_modes(d, r):
    """Multi-indices alpha with |alpha| <= r: ordered by total degree, and
    inside one degree lexicographically with alpha_0 (the x exponent) largest
    first.  Mode 0 is the constant (reading G5)."""
    modes = []
    for t in range(r + 1):
        deg = [a for a in product(range(t + 1), repeat=d) if sum(a) == t]
        deg.sort(key=lambda a: tuple(-x for x in a))
        modes.extend(deg)
    assert len(modes) == comb(r + d, d)
    return modes


def shifted_legendre(m, x):
    """P_m(2x-1) on [0,1] with the classical normalisation P_m(1)=1."""
    c = np.zeros(m + 1)
    c[m] = 1.0
    return npleg.legval(2.0 * np.asarray(x, float) - 1.0, c)


def shifted_legendre_deriv(m, x):
    c = np.zeros(m + 1)
    c[m] = 1.0
    return 2.0 * npleg.legval(2.0 * np.asarray(x, float) - 1.0, npleg.legder(c))


def pressure_values(d, r, pts):
    """psi[p, l] for reference points pts[p, :] (shape (np, d))."""
    pts = np.atleast_2d(pts)
    modes = pressure_modes(d, r)
    out = np.ones((pts.shape[0], len(modes)))
    for l, a in enumerate(modes):
        for j in range(d):
            out[:, l] *= shifted_legendre(a[j], pts[:, j])
    return out


# ------------------------------------------------------ tensor-product data
def tensor_points(x1d, d):
    """All points of the tensor grid, x (direction 0) fastest: shape (n^d, d)."""
    grids = np.meshgrid(*([x1d] * d), indexing="ij")  # grids[j][i0, i1, ...]
    # lexicographic with direction 0 fastest -> iterate reversed axes
    pts = np.stack([g.transpose(tuple(range(d))[::-1]).ravel() for g in grids], axis=1)
    return pts


def tensor_weights(w1d, d):
    w = np.ones(1)
    for _ in range(d):
        w = np.kron(w1d, w)  # direction 0 fastest
    return w


def velocity_basis(d, r, pts):
    """Values phi[p, i] and reference gradients dphi[p, i, j] of the Q_{r+1}
    Gauss-Lobatto Lagrange basis at reference points pts (n_p, d).  Local node
    index i = i_0 + Q i_1 + Q^2 i_2 (x fastest), Q = r + 2."""
    Q = r + 2
    nodes = gauss_lobatto_01(Q)
    pts = np.atleast_2d(pts)
    vals = [lagrange_values(nodes, pts[:, j]) for j in range(d)]
    ders = [lagrange_derivs(nodes, pts[:, j]) for j in range(d)]
    nloc = Q ** d
    phi = np.ones((pts.shape[0], nloc))
    dphi = np.ones((pts.shape[0], nloc, d))
    for i in range(nloc):
        idx = [(i // Q ** j) % Q for j in range(d)]
        for j in range(d):
            phi[:, i] *= vals[j][:, idx[j]]
            for g in range(d):
                dphi[:, i, g] *= (ders[j] if g == j else vals[j])[:, idx[j]]
    return phi, dphi


# ---------------------------------------------------------- time matrices
def temporal_data(k):
    """Reference temporal data of DG(k) on [-1,1] (Eq. (DefKMC)).

    Returns dict with
      t, w   : Radau points/weights
      K      : K_ab = int phi_b' phi_a dt + phi_b(-1) phi_a(-1)   (tau-free)
      M      : M_ab = int phi_b phi_a dt on [-1,1]; M^tau_n = (tau/2) M
      phim1  : phi_a(-1); C^tau_n = phim1 e_{k+1}^T, Eq. (DefKMC) for n > 1
    All integrals use a Gauss rule with k+2 points (exact for degree 2k+1).
    """
    t, w = radau_right(k)
    xg, wg = gauss_m11(k + 2)
    V = lagrange_values(t, xg)
    Dv = lagrange_derivs(t, xg)
    K = np.einsum("q,qa,qb->ab", wg, V, Dv)
    phim1 = lagrange_values(t, [-1.0])[0]
    K += np.outer(phim1, phim1)
    M = np.einsum("q,qa,qb->ab", wg, V, V)
    return {"t": t, "w": w, "K": K, "M": M, "phim1": phim1}


def n_pressure(d, r):
    return comb(r + d, d)


def vanka_block_size(d, r, k):
    """(k+1)(d (r+2)^d + dim P_r): the cell-patch size of Sec. 4.2 with the
    total-degree pressure dimension (reading G4)."""
    return (k + 1) * (d * (r + 2) ** d + n_pressure(d, r))
