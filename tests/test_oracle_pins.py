"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of these tests re-types the
oracle's own formula: they compare against printed values, closed forms,
textbook identities, invariants or brute force.
"""
import json
import os
from math import comb, factorial

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import elements as el
from oracle.assembly import SpatialLevel
from oracle.hierarchy import build_levels, paper_levels, smoother_entries, space_time_dofs
from oracle.spacetime import SpaceTimeLevel

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------ time (Sec. 3.1)
def test_radau_closed_forms():
    """Eq. (GF): right Radau rule; closed forms for k = 0, 1, 2."""
    t, w = el.radau_right(0)
    assert np.allclose(t, [1.0]) and np.allclose(w, [2.0])
    t, w = el.radau_right(1)
    assert np.allclose(t, [-1 / 3, 1.0], atol=1e-15) and np.allclose(w, [1.5, 0.5], atol=1e-15)
    t, w = el.radau_right(2)
    s6 = np.sqrt(6.0)
    assert np.allclose(t, [(-1 - s6) / 5, (-1 + s6) / 5, 1.0], atol=1e-14)
    assert np.allclose(w, [(16 - s6) / 18, (16 + s6) / 18, 2 / 9], atol=1e-14)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_radau_exact_degree_2k(k):
    """Eq. (GF) is exact for P_{2k} (and not for degree 2k+1)."""
    t, w = el.radau_right(k)
    for deg in range(2 * k + 1):
        exact = (1 - (-1) ** (deg + 1)) / (deg + 1)
        assert abs(w @ t ** deg - exact) < 1e-13
    deg = 2 * k + 1
    exact = (1 - (-1) ** (deg + 1)) / (deg + 1)
    assert abs(w @ t ** deg - exact) > 1e-6


def test_temporal_matrices_k1_k2():
    """Eq. (DefKMC), values worked out by hand for k=1 and numerically for k=2."""
    td = el.temporal_data(1)
    assert np.allclose(td["K"], [[9 / 8, 3 / 8], [-9 / 8, 5 / 8]], atol=1e-15)
    assert np.allclose(td["M"], np.diag([1.5, 0.5]), atol=1e-15)
    assert np.allclose(td["phim1"], [1.5, -0.5], atol=1e-15)
    td = el.temporal_data(2)
    K = [[1.213804, 0.439579, -0.095304], [-1.828467, 0.397307, 0.539749], [0.614664, -0.836886, 0.555556]]
    assert np.allclose(td["K"], K, atol=2e-6)
    assert np.allclose(td["phim1"], [1.558078, -0.891412, 1 / 3], atol=2e-6)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_mass_diagonal_and_constants(k):
    """Radau exactness makes M^tau diagonal with the Radau weights; K 1 = phi(-1),
    i.e. (K - C) 1 = 0: a constant-in-time function has no time derivative part."""
    td = el.temporal_data(k)
    assert np.allclose(td["M"], np.diag(td["w"]), atol=1e-14)
    assert np.allclose(td["K"] @ np.ones(k + 1), td["phim1"], atol=1e-13)


def pade_exp(m, n, z):
    num = sum(factorial(m + n - j) * factorial(m) / (factorial(m + n) * factorial(j) * factorial(m - j)) * z ** j
              for j in range(m + 1))
    den = sum(factorial(m + n - j) * factorial(n) / (factorial(m + n) * factorial(j) * factorial(n - j)) * (-z) ** j
              for j in range(n + 1))
    return num / den


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_dg_is_radau_iia_pade(k):
    """DG(k) on y' = lambda y reproduces the (k, k+1) Pade approximant of e^z
    (textbook equivalence of DG in time with Radau IIA)."""
    td = el.temporal_data(k)
    for z in [-0.5, -3.0, 0.7, -20.0]:
        Y = np.linalg.solve(td["K"] - 0.5 * z * td["M"], td["phim1"])
        assert abs(Y[-1] - pade_exp(k, k + 1, z)) < 1e-12 * max(1.0, abs(pade_exp(k, k + 1, z)))


# ------------------------------------------------------- space (Sec. 2.2, 3.1)
def test_gauss_lobatto_and_lagrange():
    x = el.gauss_lobatto_01(4)
    assert np.allclose(x, [0, (1 - 1 / np.sqrt(5)) / 2, (1 + 1 / np.sqrt(5)) / 2, 1], atol=1e-15)
    L = el.lagrange_values(x, x)
    assert np.allclose(L, np.eye(4), atol=1e-14)
    # derivative of the interpolant of a cubic equals the cubic's derivative
    pts = np.linspace(0, 1, 7)
    D = el.lagrange_derivs(x, pts)
    assert np.allclose(D @ (x ** 3 - 2 * x), 3 * pts ** 2 - 2, atol=1e-12)


@pytest.mark.parametrize("d,r", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_pressure_basis_dimension_and_orthogonality(d, r):
    """P_r^disc has dim C(r+d,d) (reading G4); shifted Legendre products are
    L2-orthogonal on [0,1]^d and mode 0 is the constant."""
    modes = el.pressure_modes(d, r)
    assert len(modes) == comb(r + d, d) and modes[0] == (0,) * d
    x1, w1 = el.gauss_01(r + 2)
    pts, w = el.tensor_points(x1, d), el.tensor_weights(w1, d)
    psi = el.pressure_values(d, r, pts)
    G = np.einsum("p,pa,pb->ab", w, psi, psi)
    expect = np.array([np.prod([1.0 / (2 * a + 1) for a in m]) for m in modes])
    assert np.allclose(G, np.diag(expect), atol=1e-14)


@pytest.mark.parametrize("d,n,r,amp", [(2, 3, 1, 0.0), (2, 4, 2, 0.03), (3, 2, 1, 0.03), (3, 2, 2, 0.03)])
def test_spatial_invariants(d, n, r, amp):
    """Eq. (DefMAB) invariants: 1^T M 1 = |Omega| = 1 even on deformed cells (the
    cells tile the unit cube and the Gauss rule is exact for det J); A 1 = 0
    (unconstrained); sum of pressure moments of mode 0 = 1; B^T c_1 = 0 on
    interior velocity rows (int div v = 0 for v in H^1_0)."""
    s = SpatialLevel(d, n, r, amp, 1.0)
    one = np.ones(s.n_nodes)
    assert abs(one @ (s.Ms @ one) - 1.0) < 1e-13
    assert np.abs(s.As @ one).max() < 1e-12
    assert abs(s.moments[:, 0].sum() - 1.0) < 1e-13
    c1 = np.zeros(s.Mp)
    c1[:: s.C] = 1.0
    btc = s.B.T @ c1
    assert np.abs(btc[~s.vel_boundary]).max() < 1e-13


def test_laplacian_energy_of_linear_field():
    """A brute-force check of A_h: for u = a.x (a linear function, in the
    finite element space), u^T A u = |a|^2 |Omega| and u^T M u = int (a.x)^2."""
    s = SpatialLevel(2, 3, 1, 0.03, 1.0)
    # node coordinates: physical positions of the Gauss-Lobatto nodes
    pos = np.zeros((s.n_nodes, 2))
    xg = el.gauss_lobatto_01(3)
    pts = el.tensor_points(xg, 2)
    for c in range(s.mesh.n_cells):
        x, _ = s.mesh.map(c, pts)
        pos[s.vdofs.cell_nodes[c]] = x
    a = np.array([0.3, -1.2])
    u = pos @ a
    # deformed cells are non-affine, so a.x is not in the space: check on the
    # undeformed mesh instead
    s0 = SpatialLevel(2, 3, 1, 0.0, 1.0)
    pos0 = np.zeros((s0.n_nodes, 2))
    for c in range(s0.mesh.n_cells):
        x, _ = s0.mesh.map(c, pts)
        pos0[s0.vdofs.cell_nodes[c]] = x
    u0 = pos0 @ a
    assert abs(u0 @ (s0.As @ u0) - a @ a) < 1e-12
    exact = a[0] ** 2 / 3 + a[1] ** 2 / 3 + 2 * a[0] * a[1] / 4
    assert abs(u0 @ (s0.Ms @ u0) - exact) < 1e-12
    assert np.isfinite(u @ (s.As @ u))


# ------------------------------------------------------------- counts (Sec. 5)
def test_table2b_cell_patch_sizes():
    """Table 2(b): all 72 printed N_sm^el values (hp: paper-table2 hierarchy
    mode of reading G12; h-MG: every spatial level keeps r and k)."""
    g = load("table2b_cell_patch_sizes.json")
    for L in range(2, 8):
        for c in range(1, 7):
            hp = smoother_entries(paper_levels(2 ** c, L - 1, L - 1, "table2"), 2)
            assert hp == g["hp"][str(L)][c - 1], (L, c)
            hm = sum(4 ** j * el.vanka_block_size(2, L - 1, L - 1) ** 2 for j in range(c + 1))
            assert hm == g["hmg"][str(L)][c - 1], (L, c)


def test_appendix_c_hierarchy():
    """App. C: Alg. 2 + Alg. 3 with fine-end padding."""
    g = load("appendix_c_hierarchy.json")
    lv = paper_levels(4, 2, 2, "appendix")
    got = [dict(level=i, h_factor=4 // n, r=r, tau_factor=1, k=k) for i, (n, r, k) in enumerate(lv)]
    assert got == g["levels_coarsest_first"]


def test_lid_driven_dof_counts():
    """Sec. 5.2 and Table 4 dof counts (Dirichlet dofs included)."""
    g = load("lid_driven_dof_counts.json")
    for r in (2, 3):
        n = 2 ** 7
        spatial = 3 * ((r + 1) * n + 1) ** 3 + n ** 3 * comb(r + 3, 3)
        assert spatial == g["c7_spatial_dofs"][str(r)]
        assert (r + 1) * spatial == g["c7_local_system_unknowns"][str(r)]
        assert space_time_dofs(3, n, r, r, 16 * n) == g["c7_space_time_dofs"][str(r)]
        for c in range(4, 8):
            assert space_time_dofs(3, 2 ** c, r, r, 16 * 2 ** c) == g["table4_N_dof"][str(r)][str(c)]
    for c in range(4, 8):
        assert (2 ** c) ** 3 * 16 * 2 ** c == g["table3_st_cells"][str(c)]


def test_config_level_lists():
    """Level placement on the benchmark configurations: Alg. 2 + Alg. 3
    (temporal coarsening padded at the fine end, App. C) and the alternative
    that halves r and k together first (reading G12)."""
    def rows(levels):
        return [tuple(l.values()) for l in levels]
    assert rows(build_levels(4, 1, 1, 2, 1)) == [(4, 1, 1, 2), (2, 1, 1, 2), (1, 1, 1, 2)]
    assert rows(build_levels(4, 1, 1, 2, 1, time_h=True)) == [(4, 1, 1, 2), (2, 1, 1, 2), (1, 1, 1, 1)]
    assert rows(build_levels(16, 2, 2, 4, 2, 1, 0)) == [(16, 2, 2, 4), (16, 1, 2, 4), (8, 1, 2, 4), (4, 1, 1, 4),
                                                        (2, 1, 0, 4)]
    assert rows(build_levels(16, 2, 2, 4, 2, 1, 2)) == [(16, 2, 2, 4), (16, 1, 2, 4), (8, 1, 2, 4), (4, 1, 2, 4),
                                                        (2, 1, 2, 4)]
    c2 = build_levels(16, 2, 2, 4, 2, 1, 0, time_h=True, placement="top")
    assert rows(c2) == [(16, 2, 2, 4), (16, 1, 1, 4), (16, 1, 0, 4), (8, 1, 0, 4), (4, 1, 0, 2), (2, 1, 0, 1)]
    assert space_time_dofs(2, 4, 1, 1, 2) == 840
    assert space_time_dofs(3, 16, 2, 2, 4) == 4726884
    assert space_time_dofs(3, 32, 2, 1, 4) == 24525592
    assert space_time_dofs(3, 32, 2, 1, 8) == 49051184


# ------------------------------------------------------ operator (Sec. 3.2)
@pytest.mark.parametrize("d,n,r,k,N,amp", [(2, 2, 1, 1, 2, 0.0), (2, 3, 2, 2, 3, 0.03), (3, 2, 1, 1, 2, 0.03)])
def test_factored_apply_equals_literal_csr(d, n, r, k, N, amp):
    s = SpatialLevel(d, n, r, amp, 1.0)
    L = SpaceTimeLevel(s, k, N, 0.05)
    x = np.random.default_rng(0).standard_normal(L.ndofs)
    assert np.allclose(L.apply(x), L.csr() @ x, rtol=0, atol=1e-13 * np.abs(x).max())


def test_operator_kernel_is_constant_pressure():
    """The singular directions of S are one constant pressure per slice
    (Eq. (DefRsSs)); the matrix is consistent for B = (F, 0)."""
    s = SpatialLevel(2, 3, 1, 0.03, 1.0)
    L = SpaceTimeLevel(s, 1, 2, 0.05)
    S = L.csr()
    for z in L.kernel_vectors():
        assert np.abs(S @ z).max() < 1e-14
        assert np.abs(S.T @ z).max() < 1e-14
    sv = np.linalg.svd(S.toarray(), compute_uv=False)
    assert np.sum(sv < 1e-12 * sv[0]) == L.N * L.nt


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_temporal_eigenvalues_are_the_pade_poles(k):
    """The temporal decoupling of the cell patches diagonalises
    diag(c)^{-1} K (c = (tau/2) w); tau times its eigenvalues are those of
    2 M^{-1} K (M = diag(w)), the poles of the DG(k) stability function,
    i.e. the roots of the denominator of the (k, k+1) Pade approximant of
    e^z: Q(z) = sum_j (2k+1-j)! (k+1)! / ((2k+1)! j! (k+1-j)!) (-z)^j.
    For k = 1 these are 2 +- i sqrt(2): one conjugate pair, no real root."""
    td = el.temporal_data(k)
    ev = np.linalg.eigvals(2.0 * np.linalg.solve(td["M"], td["K"]))
    m, n = k, k + 1
    q = [factorial(m + n - j) * factorial(n) / (factorial(m + n) * factorial(j) * factorial(n - j)) * (-1) ** j
         for j in range(n + 1)]
    roots = np.roots(q[::-1])
    key = lambda z: (round(z.real, 8), round(z.imag, 8))
    assert np.allclose(sorted(ev, key=key), sorted(roots, key=key), atol=1e-10 * max(1.0, np.abs(roots).max()))
    if k == 1:
        assert np.allclose(sorted(ev, key=key), [2 - 1j * np.sqrt(2), 2 + 1j * np.sqrt(2)], atol=1e-12)
