"""Pins of the oracle's smoother, transfers, V-cycle and learned correction
against what the mathematics fixes, with no second copy of their formulas:

* P7 (whole-domain patch): on a one-cell mesh with one subinterval the cell
  Vanka patch is the whole space, so one sweep with omega = 1 is the exact
  (mean-zero) solve, and a V-cycle on such a level is exact whichever of its
  smoothing steps runs last.
* Valence weighting: D^{-1} sum_T R_T^T R_T is the identity on free dofs
  (the weights of the patch-construction remark of Sec. 4.2 form a partition
  of unity), and a 2x2 mesh built by hand with hand-counted valences.
* App. A: the composite space-time prolongation reproduces space-time
  polynomials of the coarse space at the fine nodes and Radau points, and on
  undeformed meshes with constant viscosity (nested spaces, exact quadrature)
  rediscretisation equals the Galerkin product P^T S_f P.
* Coarse-grid correction: with Galerkin levels, a V-cycle without smoothing
  returns P e_c exactly for the right-hand side S_f P e_c.
* P8: flipping the sign of the continuity rows (reading G1) or changing the
  pressure basis cell by cell by an orthogonal map (reading G5) leaves the
  FGMRES iteration counts and residual histories unchanged.
* Learned correction (reading G15): sum_T R_T^T s_T head(net(R_T r / s_T))
  against a per-cell loop with hand-computed indices and valences.

The check functions return the error they measure, so that
tests/test_oracle_mutations.py can plant mistakes in the oracle and show
that these pins catch them.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import elements as el
from oracle import learned as ln
from oracle.assembly import SpatialLevel
from oracle.coarse import CoarseSolver
from oracle.fgmres import fgmres
from oracle.mg import Multigrid
from oracle.spacetime import SpaceTimeLevel
from oracle.transfer import prolongation
from oracle.vanka import Vanka
from stmg_inputs import random_rhs

TAU = 0.05


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def level(d, n, r, k, N, amp=0.0, nu=1.0, T=None):
    """Space-time level on [0, T] with N subintervals (T = N tau by default)."""
    T = N * TAU if T is None else T
    return SpaceTimeLevel(SpatialLevel(d, n, r, amp, nu), k, N, T / N)


def free_rhs(L, seed):
    """Random velocity entries on free dofs, zero pressure rows (consistent)."""
    rng = np.random.default_rng(seed)
    b = np.zeros(L.ndofs)
    for n in range(L.N):
        for a in range(L.nt):
            sl = L.v_index(n, a)
            b[sl] = rng.uniform(-1, 1, L.Mv) * L.free_v
    return b


# ---------------------------------------------------------------- P7: Vanka
def check_whole_domain_vanka(d, r, k, seed=0):
    """One omega = 1 sweep from zero on a one-cell, one-subinterval level
    versus the bordered direct solve of the level (reading G6)."""
    L = level(d, 1, r, k, 1, amp=0.0)
    b = free_rhs(L, seed)
    x = Vanka(L, 1.0, literal=True).smooth(b, np.zeros(L.ndofs), 1, L.apply)
    return rel(x, CoarseSolver(L).solve(b))


@pytest.mark.parametrize("d,r,k", [(2, 1, 1), (2, 2, 0), (2, 2, 2), (3, 1, 1), (3, 2, 1)])
def test_vanka_whole_domain_patch_is_exact_solve(d, r, k):
    """P7: on one cell the Vanka patch (bordered pressure) is the exact solve."""
    assert check_whole_domain_vanka(d, r, k) < 1e-12


def check_vcycle_whole_domain(d, nu_pre, nu_post, seed=1):
    """A two-level V-cycle whose fine level is one cell and one subinterval
    (so one omega = 1 Vanka sweep there is exact) returns the exact solution
    if at least one smoothing step runs and every step keeps it exact."""
    mg = Multigrid(d, 1, 2, 1, 1, TAU, n_coarse=1, omega=1.0, nu_pre=nu_pre, nu_post=nu_post)
    L = mg.levels[0]
    assert len(mg.levels) == 2 and L.sp.mesh.n_cells == 1
    b = free_rhs(L, seed)
    return rel(mg.vcycle(b), CoarseSolver(L).solve(b))


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("nu_pre,nu_post", [(1, 0), (0, 1), (1, 1)])
def test_vcycle_exact_when_the_patch_is_the_domain(d, nu_pre, nu_post):
    """Alg. 1: presmoothing, coarse correction and postsmoothing in order; an
    exact sweep before the correction leaves a zero residual (nothing to
    correct), an exact sweep after it overrides the correction."""
    assert check_vcycle_whole_domain(d, nu_pre, nu_post) < 1e-12


# --------------------------------------------------------- valence weights
def check_partition_of_unity(d, n, r, k, N, seed=2):
    """With every local inverse replaced by the identity the smoother's
    correction is D^{-1} sum_T R_T^T R_T r, which must be r on free dofs
    (valence = number of cells holding the dof) and 0 on Dirichlet dofs."""
    L = level(d, n, r, k, N, amp=0.03)
    sm = Vanka(L, 0.8, literal=True)
    sm.inv = np.broadcast_to(np.eye(sm.inv.shape[1]), sm.inv.shape).copy()
    r_ = np.random.default_rng(seed).standard_normal(L.ndofs)
    want = np.where(L.dirichlet_mask(), 0.0, r_)
    return rel(sm.correction(r_), want)


@pytest.mark.parametrize("d,n,r,k,N", [(2, 3, 1, 1, 2), (2, 2, 2, 0, 1), (3, 2, 1, 1, 2)])
def test_vanka_valence_is_partition_of_unity(d, n, r, k, N):
    assert check_partition_of_unity(d, n, r, k, N) < 1e-15


def hand_built_vanka_2x2(r_vec, S, k, N):
    """Eq. (vanka0) on the 2D 2x2 mesh with Q2/P1 x DG(k), written out with
    explicit index arithmetic: nn = 5 nodes per direction, node (gx, gy) has
    index gx + 5 gy, cell (cx, cy) holds nodes 2 cx .. 2 cx + 2 along x;
    valence of a node = (2 if gx == 2 else 1) * (2 if gy == 2 else 1)."""
    nt, nn, q, C, ncell = k + 1, 5, 2, 3, 4
    Mv, Mp = 2 * nn * nn, ncell * C
    slab = nt * (Mv + Mp)
    u = np.zeros_like(r_vec)
    for n in range(N):
        for cy in range(2):
            for cx in range(2):
                idx = []
                for a in range(nt):
                    for comp in range(2):
                        for iy in range(3):
                            for ix in range(3):
                                g = (q * cx + ix) + nn * (q * cy + iy)
                                idx.append(n * slab + a * Mv + comp * nn * nn + g)
                for a in range(nt):
                    for l in range(C):
                        idx.append(n * slab + nt * Mv + a * Mp + (cx + 2 * cy) * C + l)
                idx = np.array(idx)
                A = S[idx][:, idx].toarray()
                u[idx] += np.linalg.solve(A, r_vec[idx])
    for n in range(N):
        for a in range(nt):
            for comp in range(2):
                for gy in range(nn):
                    for gx in range(nn):
                        i = n * slab + a * Mv + comp * nn * nn + gx + nn * gy
                        if gx in (0, nn - 1) or gy in (0, nn - 1):
                            u[i] = 0.0
                        else:
                            u[i] /= (2 if gx == 2 else 1) * (2 if gy == 2 else 1)
    return u


@pytest.mark.parametrize("k,N", [(1, 2), (0, 1)])
def test_vanka_correction_against_hand_built_2x2(k, N):
    L = level(2, 2, 1, k, N, amp=0.03)
    r_ = np.random.default_rng(3).standard_normal(L.ndofs)
    got = Vanka(L, 0.8, literal=True).correction(r_)
    assert rel(got, hand_built_vanka_2x2(r_, L.csr(), k, N)) < 1e-12


# --------------------------------------------------------------- transfers
def ref_node_positions(s):
    """Undeformed positions of the global velocity nodes, from the node grid:
    node (g_0, .., g_{d-1}) sits at (c + x_i) / n with c = min(g // q, n - 1)."""
    q, n, nn = s.r + 1, s.n, s.vdofs.nn
    gll = el.gauss_lobatto_01(q + 1)
    one = np.array([(min(g // q, n - 1) + gll[g - min(g // q, n - 1) * q]) / n for g in range(nn)])
    m = np.arange(s.n_nodes)
    return np.stack([one[(m // nn ** j) % nn] for j in range(s.d)], axis=1)


def st_coefficients(L, T, vel, pres):
    """Coefficient vector of the space-time function (velocity vel(X, t) ->
    (npts, d), pressure pres(X, t) -> (npts,)), both in the level's space:
    nodal values at the Gauss-Lobatto nodes and Radau points; per cell the
    pressure coefficients fitted to samples (exact, the function lies in
    P_r on every cell)."""
    s = L.sp
    X = ref_node_positions(s)
    tr = el.radau_right(L.k)[0]
    rng = np.random.default_rng(0)
    xi = rng.random((3 * s.C, s.d))
    psi = el.pressure_values(s.d, s.r, xi)
    out = np.zeros(L.ndofs)
    for n in range(L.N):
        for a in range(L.nt):
            t = (n + (tr[a] + 1.0) / 2.0) * T / L.N
            out[L.v_index(n, a)] = vel(X, t).T.ravel()
            pc = np.zeros(s.Mp)
            for c in range(s.mesh.n_cells):
                Xc = (np.array(s.mesh.cell_coords(c))[None, :] + xi) / s.n
                pc[c * s.C:(c + 1) * s.C] = np.linalg.lstsq(psi, pres(Xc, t), rcond=None)[0]
            out[L.p_index(n, a)] = pc
    return out


def check_composite_prolongation(pair):
    (d, nf, rf, kf, Nf), (_, nc, rc, kc, Nc) = pair
    T = 0.2
    Lf, Lc = level(d, nf, rf, kf, Nf, amp=0.03, T=T), level(d, nc, rc, kc, Nc, amp=0.03, T=T)
    P = prolongation(Lf, Lc)

    def g(t, c=0):  # degree kc in time
        return sum((j + 1.0 + c) * t ** j for j in range(kc + 1))

    def vel(X, t):  # Q_{rc+1} in space, zero on the boundary, one factor per component
        bub = np.prod(X * (1 - X), axis=1)
        lin = (1.0 + 0.4 * X[:, 0] - 0.3 * X[:, -1]) if rc >= 2 else 1.0
        return np.stack([(c + 1.0) * bub * lin * g(t, c) for c in range(d)], axis=1)

    def pres(X, t):  # total degree rc in space
        p = 0.5 + X[:, 0] - 2.0 * X[:, 1] + (0.7 * X[:, 2] if d == 3 else 0.0)
        if rc >= 2:
            p = p + X[:, 0] * X[:, 1] - 0.3 * X[:, 1] ** 2
        return p * g(t)

    return rel(P @ st_coefficients(Lc, T, vel, pres), st_coefficients(Lf, T, vel, pres))


PAIRS = [
    ((2, 2, 2, 2, 2), (2, 2, 1, 1, 2)),   # p in space and time
    ((2, 4, 1, 1, 2), (2, 2, 1, 1, 1)),   # h in space and time
    ((2, 4, 2, 1, 2), (2, 2, 1, 0, 1)),   # h and p in space and time at once
    ((3, 2, 2, 2, 2), (3, 1, 1, 1, 1)),   # 3D, all four
]


@pytest.mark.parametrize("pair", PAIRS)
def test_composite_prolongation_reproduces_space_time_polynomials(pair):
    """App. A, Eq. (DefTlspr), (DefoTsl): P is the embedding of the coarse
    space-time space, velocity and pressure together."""
    assert check_composite_prolongation(pair) < 1e-12


def check_galerkin(pair):
    (d, nf, rf, kf, Nf), (_, nc, rc, kc, Nc) = pair
    T = 0.2
    Lf, Lc = level(d, nf, rf, kf, Nf, T=T), level(d, nc, rc, kc, Nc, T=T)
    P = prolongation(Lf, Lc)
    G = (P.T @ Lf.csr() @ P).toarray()
    Sc = Lc.csr().toarray()
    fr = ~Lc.dirichlet_mask()
    return rel(G[np.ix_(fr, fr)], Sc[np.ix_(fr, fr)])


@pytest.mark.parametrize("pair", PAIRS)
def test_rediscretisation_equals_galerkin_on_nested_spaces(pair):
    """Undeformed meshes, constant nu: the level spaces are nested and every
    integral of Eq. (DefMAB), (DefKMC) is exact, so S_c = P^T S_f P."""
    assert check_galerkin(pair) < 1e-12


def check_coarse_correction(seed=4):
    """V-cycle with no smoothing on Galerkin levels: the right-hand side
    S_f P e_c is solved exactly (to P e_c, mean-zero pressure)."""
    mg = Multigrid(2, 4, 1, 1, 2, TAU, n_coarse=2, omega=0.8, nu_pre=0, nu_post=0)
    assert len(mg.levels) == 2
    Lf, Lc = mg.levels
    ec = Lc.project_pressure(free_rhs(Lc, seed) + 0.1 * np.random.default_rng(seed).standard_normal(Lc.ndofs)
                             * ~Lc.dirichlet_mask())
    ef = mg.P[0] @ ec
    return rel(mg.vcycle(Lf.apply(ef)), ef)


def test_vcycle_coarse_correction_is_exact_on_coarse_errors():
    assert check_coarse_correction() < 1e-12


# ----------------------------------------------------------------------- P8
class Transformed:
    """The level's system G_l S G_r with the same dof layout."""

    def __init__(self, L, Gl, Gr):
        self._L, self._Gr = L, Gr
        self._S = (Gl @ L.csr() @ Gr).tocsr()

    def __getattr__(self, name):
        return getattr(self._L, name)

    def csr(self):
        return self._S

    def apply(self, x):
        return self._S @ x

    def constraint_vectors(self):
        return (self._Gr.T @ self._L.constraint_vectors().T).T


def slab_blockdiag(L, vel_block, pres_block):
    blocks = []
    for n in range(L.N):
        blocks += [vel_block] * L.nt + [pres_block] * L.nt
    return sp.block_diag(blocks, format="csr")


def transformed_mg(kind, seed=5):
    """The oracle's multigrid on the transformed levels: continuity rows
    negated (kind "sign"), or the pressure basis of every cell rotated by a
    random orthogonal matrix (kind "basis")."""
    mg = Multigrid(2, 4, 1, 1, 2, TAU, amp=0.03, n_coarse=1, omega=0.8)
    rng = np.random.default_rng(seed)
    G = []
    for L in mg.levels:
        s = L.sp
        Iv = sp.identity(L.Mv, format="csr")
        if kind == "sign":
            G.append((slab_blockdiag(L, Iv, -sp.identity(L.Mp)), sp.identity(L.ndofs, format="csr")))
        else:
            Ts = [np.linalg.qr(rng.standard_normal((s.C, s.C)))[0] for _ in range(s.mesh.n_cells)]
            Gr = slab_blockdiag(L, Iv, sp.block_diag(Ts, format="csr"))
            G.append((Gr.T.tocsr(), Gr))
    levels = [Transformed(L, Gl, Gr) for L, (Gl, Gr) in zip(mg.levels, G)]
    mg2 = Multigrid.__new__(Multigrid)
    mg2.spec, mg2.nu_pre, mg2.nu_post = mg.spec, mg.nu_pre, mg.nu_post
    mg2.levels = levels
    mg2.P = [(G[i][1].T @ mg.P[i] @ G[i + 1][1]).tocsr() for i in range(len(mg.P))]
    mg2.smoothers = [Vanka(L, 0.8, literal=True) for L in levels[:-1]]
    mg2.coarse = CoarseSolver(levels[-1])
    return mg, mg2, G[0][0]


@pytest.mark.parametrize("kind", ["sign", "basis"])
def test_fgmres_invariant_under_sign_and_basis_change(kind):
    """P8 (readings G1, G5)."""
    mg, mg2, Gl = transformed_mg(kind)
    L, L2 = mg.levels[0], mg2.levels[0]
    b = random_rhs(2, 4, 1, 1, 2, 9)
    x, it, h = fgmres(L.apply, mg.vcycle, b, rtol=1e-10, max_it=60)
    x2, it2, h2 = fgmres(L2.apply, mg2.vcycle, Gl @ b, rtol=1e-10, max_it=60)
    assert it == it2, (it, it2)
    assert np.allclose(h, h2, rtol=1e-6, atol=1e-14)


# -------------------------------------------------------- learned correction
def hand_built_learned(r_vec, Ws, n, N):
    """Reading G15 per space-time cell of a 3D Q2/P1 x DG(1) level on n^3
    cells, with the vector layout of Eq. (DefX) written out by hand."""
    q, nn, C, nt, d = 2, 2 * n + 1, 4, 2, 3
    Mv, Mp = d * nn ** 3, n ** 3 * C
    slab = nt * (Mv + Mp)

    def vel_index(s, a, comp, g):
        return s * slab + a * Mv + comp * nn ** 3 + g[0] + nn * g[1] + nn * nn * g[2]

    def valence(g):
        v = 1
        for x in g:
            v *= 2 if (x % q == 0 and 0 < x < nn - 1) else 1
        return v

    def boundary(g):
        return any(x in (0, nn - 1) for x in g)

    u = np.zeros_like(r_vec)
    for s in range(N):
        for cz in range(n):
            for cy in range(n):
                for cx in range(n):
                    cell = cx + n * (cy + n * cz)
                    X = np.zeros((15, 27))
                    nodes = [(q * cx + i % 3, q * cy + (i // 3) % 3, q * cz + i // 9) for i in range(27)]
                    for i, g in enumerate(nodes):
                        X[14, i] = 1.0 if boundary(g) else 0.0
                        for a in range(nt):
                            for comp in range(d):
                                if not boundary(g):
                                    X[comp * 2 + a, i] = r_vec[vel_index(s, a, comp, g)]
                    for a in range(nt):
                        for l in range(C):
                            X[6 + 4 * a + l, :] = r_vec[s * slab + nt * Mv + a * Mp + cell * C + l]
                    sT = np.sqrt(np.sum(X[:6] ** 2) + np.sum(X[6:14, 0] ** 2))
                    if sT == 0.0:
                        continue
                    X[:14] /= sT
                    y = ln.forward(Ws, X[None])[0]
                    for i, g in enumerate(nodes):
                        if boundary(g):
                            continue
                        for a in range(nt):
                            for comp in range(d):
                                u[vel_index(s, a, comp, g)] += sT * y[comp * 2 + a, i] / valence(g)
                    for a in range(nt):
                        for l in range(C):
                            u[s * slab + nt * Mv + a * Mp + cell * C + l] += sT * np.mean(y[6 + 4 * a + l, :])
    return u


def test_learned_correction_against_per_cell_loop():
    L = level(3, 2, 1, 1, 2, amp=0.03)
    Ws = ln.init_weights(6)
    r_ = np.random.default_rng(7).standard_normal(L.ndofs)
    r_[L.dirichlet_mask()] = 0.0
    got = ln.correction(L, Ws, r_)
    assert rel(got, hand_built_learned(r_, Ws, 2, 2)) < 1e-12
