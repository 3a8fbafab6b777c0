"""Pins of the oracle's transfers, smoother, V-cycle and FGMRES, and of the
discretisation's convergence orders (Table 1's optimal orders)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import elements as el
from oracle.assembly import SpatialLevel
from oracle.coarse import CoarseSolver
from oracle.errors import errors, load_vector
from oracle.fgmres import fgmres
from oracle.mg import Multigrid
from oracle.spacetime import SpaceTimeLevel
from oracle.transfer import pressure_prolongation, prolongation, time_prolongation, velocity_prolongation
from oracle.vanka import local_matrices_factored, local_matrices_literal
from stmg_inputs import Manufactured2D, random_rhs


def node_positions_ref(s):
    """Undeformed positions of the global velocity nodes (brute force)."""
    xg = el.gauss_lobatto_01(s.r + 2)
    pos = np.zeros((s.n_nodes, s.d))
    for c in range(s.mesh.n_cells):
        cc = s.mesh.cell_coords(c)
        pts = el.tensor_points(xg, s.d)
        pos[s.vdofs.cell_nodes[c]] = (np.array(cc)[None, :] + pts) / s.n
    return pos


@pytest.mark.parametrize("d,nf,rf,nc,rc", [(2, 4, 2, 4, 1), (2, 4, 1, 2, 1), (3, 2, 2, 2, 1), (3, 4, 1, 2, 1)])
def test_velocity_prolongation_reproduces_polynomials(d, nf, rf, nc, rc):
    """App. A, Eq. (DefPrRe)/(DefPrRer): the prolongation is the embedding, so a
    polynomial of the coarse space (times a bubble vanishing on the boundary)
    is reproduced exactly at the fine nodes."""
    sf, sc = SpatialLevel(d, nf, rf, 0.03), SpatialLevel(d, nc, rc, 0.03)
    P = velocity_prolongation(sf, sc)
    deg = rc + 1  # Q_{rc+1} per direction on each coarse cell -> use a global polynomial of that degree
    def f(X):
        # vanishes on the boundary, degree <= 2 per direction, times a linear factor
        v = np.ones(len(X))
        for j in range(d):
            v *= X[:, j] * (1 - X[:, j])
        return v * (1 + 0.5 * X[:, 0]) if deg >= 3 else v
    uc = f(node_positions_ref(sc))
    uf = f(node_positions_ref(sf))
    assert np.abs(P @ uc - uf).max() < 1e-13


@pytest.mark.parametrize("d,nf,rf,nc,rc", [(2, 4, 2, 4, 1), (2, 4, 2, 2, 2), (3, 2, 2, 1, 2), (3, 2, 2, 2, 1)])
def test_pressure_prolongation_is_embedding(d, nf, rf, nc, rc):
    """Coarse cell polynomials evaluated at fine-cell points equal the
    prolongated fine representation (brute-force point evaluation)."""
    sf, sc = SpatialLevel(d, nf, rf), SpatialLevel(d, nc, rc)
    P = pressure_prolongation(sf, sc).toarray()
    rng = np.random.default_rng(1)
    pc = rng.standard_normal(sc.Mp)
    pf = P @ pc
    ratio = nf // nc
    xi = rng.random((5, d))
    for cf in range(sf.mesh.n_cells):
        ccf = sf.mesh.cell_coords(cf)
        par = sum((ccf[j] // ratio) * nc ** j for j in range(d))
        Xc = (np.array([x % ratio for x in ccf])[None, :] + xi) / ratio
        vf = el.pressure_values(d, rf, xi) @ pf[cf * sf.C:(cf + 1) * sf.C]
        vc = el.pressure_values(d, rc, Xc) @ pc[par * sc.C:(par + 1) * sc.C]
        assert np.allclose(vf, vc, atol=1e-13)


@pytest.mark.parametrize("kf,Nf,kc,Nc", [(2, 2, 1, 2), (1, 2, 0, 2), (1, 4, 1, 2), (0, 2, 0, 1), (2, 1, 2, 1)])
def test_time_prolongation_reproduces_polynomials(kf, Nf, kc, Nc):
    """Eq. (DeftPrRe)/(DefPrRek): a polynomial of degree kc on each coarse
    subinterval is reproduced at the fine Radau points."""
    P = time_prolongation(kf, Nf, kc, Nc)
    tc, tf = el.radau_right(kc)[0], el.radau_right(kf)[0]
    T = 1.0
    def g(t):
        return np.polyval(np.arange(1, kc + 2, dtype=float), t)  # degree kc
    # coarse subinterval i covers [i, i+1] * T/Nc; a global polynomial of degree kc
    cvals = np.concatenate([g((i + (tc + 1) / 2) * T / Nc) for i in range(Nc)])
    fvals = np.concatenate([g((i + (tf + 1) / 2) * T / Nf) for i in range(Nf)])
    assert np.allclose(P @ cvals, fvals, atol=1e-12)


def test_restriction_preserves_consistency():
    """The restricted residual of a consistent system stays orthogonal to the
    constant pressures of the coarse level (transfers preserve constants)."""
    mg = Multigrid(3, 2, 2, 2, 2, 0.05, amp=0.03, n_coarse=2, k_min=0, omega=0.8)
    for i, P in enumerate(mg.P):
        Lc = mg.levels[i + 1]
        Lf = mg.levels[i]
        for z in Lc.kernel_vectors():
            zf = P @ z
            # the prolongation of a coarse constant pressure is a fine kernel vector
            assert np.abs(Lf.apply(zf)).max() < 1e-12


def test_local_blocks_literal_equal_factored():
    """Reading G7: the Kronecker construction of A_T equals S[idx_T, idx_T]."""
    s = SpatialLevel(3, 2, 1, 0.03)
    L = SpaceTimeLevel(s, 1, 2, 0.05)
    assert np.allclose(local_matrices_literal(L), local_matrices_factored(L), atol=1e-14)


def test_fgmres_against_direct_solve():
    rng = np.random.default_rng(3)
    A = np.eye(60) * 4 + rng.standard_normal((60, 60))
    b = rng.standard_normal(60)
    x, it, _ = fgmres(lambda v: A @ v, lambda v: v, b, rtol=1e-12, max_it=60)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-10 * np.linalg.norm(x)
    Ainv = np.linalg.inv(A)
    x, it, _ = fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, rtol=1e-12)
    assert it == 1


def test_manufactured_forcing_matches_finite_differences():
    """The hand-derived forcing f = u_t - nu Lap u + grad p and div u = 0
    (reading G17), checked by central differences."""
    ms = Manufactured2D(1.0)
    rng = np.random.default_rng(4)
    x = rng.random((20, 2))
    t, h = 0.37, 1e-4
    ut = (ms.v(x, t + h) - ms.v(x, t - h)) / (2 * h)
    lap = np.zeros_like(ut)
    gp = np.zeros_like(ut)
    div = np.zeros(len(x))
    for j in range(2):
        e = np.zeros(2); e[j] = h
        lap += (ms.v(x + e, t) - 2 * ms.v(x, t) + ms.v(x - e, t)) / h ** 2
        gp[:, j] = (ms.p(x + e, t) - ms.p(x - e, t)) / (2 * h)
        div += (ms.v(x + e, t)[:, j] - ms.v(x - e, t)[:, j]) / (2 * h)
    assert np.allclose(ms.f(x, t), ut - lap + gp, atol=2e-5)
    assert np.abs(div).max() < 1e-6
    g = ms.gradv(x, t)
    for j in range(2):
        e = np.zeros(2); e[j] = h
        assert np.allclose(g[:, :, j], (ms.v(x + e, t) - ms.v(x - e, t)) / (2 * h), atol=1e-6)


def direct_solution(L, b):
    return CoarseSolver(L).solve(b)


def test_c1_mg_fgmres_equals_direct_solve():
    """P6: the MG-preconditioned FGMRES solution of configuration C1 equals the
    bordered direct solve (after the per-slice pressure projection)."""
    mg = Multigrid(2, 4, 1, 1, 2, 0.05, nu=1.0, omega=0.8)
    L = mg.levels[0]
    assert L.ndofs == 840
    b = load_vector(L, Manufactured2D(1.0).f)
    x, it, hist = fgmres(L.apply, mg.vcycle, b, rtol=1e-13)
    xd = direct_solution(L, b)
    rel = np.linalg.norm(L.project_pressure(x) - xd) / np.linalg.norm(xd)
    assert rel < 1e-10
    x, it, hist = fgmres(L.apply, mg.vcycle, b, rtol=1e-10)
    assert 5 <= it <= 51          # loose band of Table 2(a)
    assert hist[-1] <= 1e-10


@pytest.mark.parametrize("n,r,k,N,kmin", [(4, 1, 1, 2, 1), (2, 2, 2, 2, 0)])
def test_3d_mg_fgmres_equals_direct_solve(n, r, k, N, kmin):
    mg = Multigrid(3, n, r, k, N, 0.05, amp=0.03, n_coarse=2, k_min=kmin, omega=0.8)
    L = mg.levels[0]
    b = random_rhs(3, n, r, k, N, 7)
    x, it, _ = fgmres(L.apply, mg.vcycle, b, rtol=1e-12)
    S = L.csr()
    Z = L.constraint_vectors().T
    A = sp.bmat([[S, sp.csr_matrix(Z)], [sp.csr_matrix(Z.T), None]], format="csc")
    xd = spla.spsolve(A, np.concatenate([b, np.zeros(Z.shape[1])]))[: L.ndofs]
    rel = np.linalg.norm(L.project_pressure(x) - xd) / np.linalg.norm(xd)
    assert rel < 1e-10


def manufactured_errors(n, r, k, N, tau):
    s = SpatialLevel(2, n, r, 0.0, 1.0)
    L = SpaceTimeLevel(s, k, N, tau)
    ms = Manufactured2D(1.0)
    b = load_vector(L, ms.f)
    S = L.csr()
    Z = L.constraint_vectors().T
    A = sp.bmat([[S, sp.csr_matrix(Z)], [sp.csr_matrix(Z.T), None]], format="csc")
    X = spla.spsolve(A, np.concatenate([b, np.zeros(Z.shape[1])]))[: L.ndofs]
    return errors(L, X, ms.v, ms.gradv, ms.p)


@pytest.mark.slow
def test_spatial_convergence_orders():
    """Table 1 / Sec. 5.1: optimal orders r+2 (velocity L2), r+1 (velocity H1
    seminorm, pressure L2) in space; time kept accurate (k=3, small slab).
    A dropped term or a wrong sign in the operator or the load vector
    destroys these rates."""
    r = 1
    errs = [manufactured_errors(n, r, 3, 2, 0.01) for n in (4, 8, 16)]
    e = np.array(errs)
    eoc = np.log2(e[:-1] / e[1:])
    assert abs(eoc[-1, 0] - (r + 2)) < 0.3, eoc
    assert abs(eoc[-1, 1] - (r + 1)) < 0.3, eoc
    # pressure: at least the optimal order r+1 (pre-asymptotically the
    # uniform-mesh pressure converges faster: ~2.9 at h=1/16 for r=1)
    assert eoc[-1, 2] > (r + 1) - 0.3, eoc


@pytest.mark.slow
def test_temporal_convergence_order():
    """DG(k) in time: L2(L2) error ~ tau^{k+1} (space resolved with r=3)."""
    k = 1
    T = 0.8
    errs = [manufactured_errors(4, 3, k, N, T / N) for N in (2, 4, 8)]
    e = np.array(errs)
    eoc = np.log2(e[:-1, 0] / e[1:, 0])
    assert abs(eoc[-1] - (k + 1)) < 0.3, eoc
