"""Pins of the oracle's time marching over slabs with inhomogeneous Dirichlet
data (oracle/marching.py; Eq. (AlgSysTMS) of Sec. 3.2), against what the
mathematics fixes:

  * a constant flow u = c, p = 0 with boundary data c and initial value c
    solves the Stokes system with f = 0, and the discrete scheme reproduces
    it exactly (constants are in every space; K 1 = phi(-1) so the time
    derivative and the jump cancel; A_h annihilates constants);
  * a flow linear in time, u = t c, p = 0, with forcing c is reproduced
    exactly by DG(k >= 1) (the Radau rule integrates the test functions
    exactly, so the slab equation holds for the interpolant);
  * marching slab after slab is block forward substitution of the global
    system of Eq. (GloSys): two slabs of N subintervals equal one slab of 2N;
  * the lid-driven cavity's lifted data keep the slab system consistent
    (the constant pressure of every slice sees a zero right-hand side, since
    the lid velocity is tangential and the edge contributions cancel).
A planted sign error in the C^1 V_0 term, or a dropped Dirichlet column in
the lifting, fails the last three."""
import numpy as np
import pytest

from oracle import elements as el
from oracle import marching as mr
from oracle.assembly import SpatialLevel
from oracle.coarse import CoarseSolver
from oracle.errors import load_vector
from oracle.spacetime import SpaceTimeLevel
from stmg_inputs import lid_dirichlet

CASES = [dict(d=2, n=4, r=1, k=1, N=2, amp=0.0), dict(d=3, n=2, r=1, k=2, N=1, amp=0.03),
         dict(d=2, n=3, r=2, k=2, N=2, amp=0.05)]


def level(c, N=None, nu=1.0, tau=0.05):
    sp = SpatialLevel(c["d"], c["n"], c["r"], c["amp"], nu)
    return SpaceTimeLevel(sp, c["k"], c["N"] if N is None else N, tau)


def velocity_const(L, cvec):
    x = np.zeros(L.ndofs)
    for n in range(L.N):
        for a in range(L.nt):
            x[L.v_index(n, a)] = np.repeat(cvec, L.sp.n_nodes)
    return x


def times(L, t0):
    return [[t0 + L.tau * (n + 0.5 * (L.td["t"][a] + 1.0)) for a in range(L.nt)] for n in range(L.N)]


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"{c['d']}d_r{c['r']}_k{c['k']}")
def test_constant_flow_is_reproduced(c):
    L = level(c)
    cvec = np.array([0.7, -0.3, 0.2][: c["d"]])
    u = velocity_const(L, cvec)
    v0 = np.repeat(cvec, L.sp.n_nodes)
    x = mr.solve_slab(L, CoarseSolver(L).solve, None, v0, u)
    assert np.max(np.abs(x - u)) <= 1e-10 * np.max(np.abs(cvec))


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"{c['d']}d_r{c['r']}_k{c['k']}")
def test_linear_in_time_flow_is_reproduced(c):
    if c["k"] < 1:
        pytest.skip("DG(0) does not reproduce linear functions of time")
    L = level(c)
    t0 = 0.3
    cvec = np.array([0.4, 0.9, -0.5][: c["d"]])
    u = np.zeros(L.ndofs)
    for n, row in enumerate(times(L, t0)):
        for a, t in enumerate(row):
            u[L.v_index(n, a)] = np.repeat(t * cvec, L.sp.n_nodes)
    f = load_vector(L, lambda x, t: np.tile(cvec, (len(x), 1)), t0=t0)
    v0 = np.repeat(t0 * cvec, L.sp.n_nodes)
    x = mr.solve_slab(L, CoarseSolver(L).solve, f, v0, u)
    assert np.max(np.abs(x - u)) <= 1e-10 * np.max(np.abs(u))


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"{c['d']}d_r{c['r']}_k{c['k']}")
def test_two_slabs_equal_one_slab_of_twice_the_length(c):
    L1, L2 = level(c), level(c, N=2 * c["N"])
    rng = np.random.default_rng(5)
    f2 = rng.standard_normal(L2.ndofs)
    f2[L2.dirichlet_mask()] = 0.0
    t_hat = L1.td["t"]
    g2 = lid_dirichlet(c["d"], c["n"], c["r"], c["k"], 2 * c["N"], L1.tau, 0.1, t_hat)
    v0 = rng.standard_normal(L1.Mv)
    x2 = mr.solve_slab(L2, CoarseSolver(L2).solve, f2, v0, g2)
    xs = mr.march(L1, CoarseSolver(L1).solve, 2, f2.reshape(2, -1), g2.reshape(2, -1), v0)
    assert np.max(np.abs(xs.ravel() - x2)) <= 1e-10 * np.max(np.abs(x2))


def test_lid_data_keep_the_slab_system_consistent():
    c = dict(d=3, n=2, r=2, k=2, N=2, amp=0.0)
    L = level(c, nu=0.1)
    g = lid_dirichlet(3, 2, 2, 2, 2, L.tau, 0.0, L.td["t"])
    assert np.max(np.abs(g)) > 0.01
    b = mr.slab_rhs(L, None, None, g)
    assert np.max(np.abs(b)) > 1e-6
    for n in range(L.N):
        for a in range(L.nt):
            p = b[L.p_index(n, a)].reshape(L.sp.mesh.n_cells, L.sp.C)
            assert abs(p[:, 0].sum()) <= 1e-13 * np.max(np.abs(b))


def test_time_nodes_pin():
    """The temporal dofs sit at the right Radau points (end point 1), so the
    last dof is the end value the next slab couples to."""
    for k in range(4):
        t = el.temporal_data(k)["t"]
        assert abs(t[-1] - 1.0) < 1e-15
