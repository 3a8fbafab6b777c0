"""GPU parity: every step of the hot path, called through the C ABI, against
the CPU oracle on the same seeded inputs.  FP64 tolerance 1e-12 relative
(max-norm) for the operator, smoother, transfers and coarse solve; identical
FGMRES iteration counts; solutions within 1e-10 after the per-slice pressure
projection."""
import numpy as np
import pytest
import torch

from paper_2502_09159_amd.stmg import RESTART
from gpu_common import CONFIGS, announce, dev, host, make_solver, oracle_mg, rel, rhs

pytestmark = pytest.mark.gpu

NAMES = list(CONFIGS)
_solvers = {}


def solver(name, **over):
    key = (name, tuple(sorted(over.items())))
    if key not in _solvers:
        announce(f"setup {name} {over}")
        _solvers[key] = make_solver(CONFIGS[name], **over)
    return _solvers[key]


@pytest.fixture(scope="module", autouse=True)
def _cleanup():
    yield
    for s in _solvers.values():
        s.close()
    _solvers.clear()


@pytest.mark.parametrize("name", NAMES)
def test_level_sizes_match(name):
    g, o = solver(name), oracle_mg(name)
    assert g.n_levels == len(o.levels)
    for l, L in enumerate(o.levels):
        nd, nv, npr, _ = g.sizes(l)
        assert (nd, nv, npr) == (L.ndofs, L.Mv, L.Mp)


@pytest.mark.parametrize("name", NAMES)
def test_apply_every_level(name):
    """Eq. (GloSys): matrix-free apply = assembled mat-vec, <= 1e-12."""
    g, o = solver(name), oracle_mg(name)
    rng = np.random.default_rng(11)
    for l, L in enumerate(o.levels):
        announce(f"apply {name} level {l}")
        x = rng.standard_normal(L.ndofs)
        y = torch.empty(L.ndofs, dtype=torch.float64, device="cuda")
        g.apply(dev(x), y, level=l)
        ref = L.csr() @ x
        assert rel(host(y), ref) < 1e-12, (l, rel(host(y), ref))
        b = rng.standard_normal(L.ndofs)
        r = torch.empty_like(y)
        g.residual(dev(b), dev(x), r, level=l)
        assert rel(host(r), b - ref) < 1e-12


@pytest.mark.parametrize("name", NAMES)
def test_smoother_every_level(name):
    """Eq. (vanka): one and two cell-Vanka sweeps, <= 1e-12."""
    g, o = solver(name), oracle_mg(name)
    rng = np.random.default_rng(12)
    for l, L in enumerate(o.levels[:-1]):
        announce(f"smooth {name} level {l}")
        dm = L.dirichlet_mask()
        b = rng.standard_normal(L.ndofs); b[dm] = 0
        x0 = rng.standard_normal(L.ndofs); x0[dm] = 0
        for steps in (1, 2):
            xg = dev(x0)
            g.smooth(dev(b), xg, steps=steps, level=l)
            ref = o.smoothers[l].smooth(b, x0.copy(), steps, L.apply)
            assert rel(host(xg), ref) < 1e-12, (l, steps, rel(host(xg), ref))


@pytest.mark.parametrize("name", NAMES)
def test_fp32_smoother_every_level(name):
    """Eq. (vanka) in the mixed precision's FP32 hierarchy: two sweeps, whose
    second residual comes from the FP32 operator, against the FP64 oracle.
    Bound 1e-5 relative (measured at most 2.4e-7): FP32 rounding (unit
    roundoff 6e-8) of the operator, the stored local factors and the solves,
    amplified by the conditioning of the cell systems."""
    g, o = solver(name, precision=1), oracle_mg(name)
    rng = np.random.default_rng(14)
    for l, L in enumerate(o.levels[:-1]):
        dm = L.dirichlet_mask()
        b = rng.standard_normal(L.ndofs); b[dm] = 0
        x0 = rng.standard_normal(L.ndofs); x0[dm] = 0
        for steps in (1, 2):
            xg = dev(x0)
            g.smooth(dev(b), xg, steps=steps, level=l)
            ref = o.smoothers[l].smooth(b, x0.copy(), steps, L.apply)
            err = rel(host(xg), ref)
            announce(f"fp32 smooth {name} level {l} steps {steps}: {err:.2e}")
            assert err < 1e-5, (l, steps, err)


def test_vanka_forms_agree():
    """The stored forms of the same local inverse give the same sweep: the
    default (per level), decoupled in time, Schur-factored space-time block,
    dense."""
    name = "c2_small"
    gs = [solver(name), solver(name, vanka_mode=2), solver(name, vanka_mode=0), solver(name, vanka_mode=1)]
    o = oracle_mg(name)
    rng = np.random.default_rng(13)
    for l, L in enumerate(o.levels[:-1]):
        dm = L.dirichlet_mask()
        b = rng.standard_normal(L.ndofs); b[dm] = 0
        xs = [dev(np.zeros(L.ndofs)) for _ in gs]
        for g, x in zip(gs, xs):
            g.smooth(dev(b), x, 1, level=l)
        for x in xs[1:]:
            assert rel(host(x), host(xs[0])) < 1e-12


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("mode", [0, 2], ids=["coupled", "decoupled"])
def test_vanka_form_every_level(name, precision, mode):
    """Each factored form on every level, whatever the default picks there:
    the Schur-factored space-time block (vanka_mode 0) and the decoupled
    spatial blocks (vanka_mode 2) against the oracle, one and two sweeps,
    1e-12 in FP64 and 1e-5 in the FP32 hierarchy."""
    g, o = solver(name, vanka_mode=mode, precision=precision), oracle_mg(name)
    rng = np.random.default_rng(16)
    for l, L in enumerate(o.levels[:-1]):
        dm = L.dirichlet_mask()
        b = rng.standard_normal(L.ndofs); b[dm] = 0
        x0 = rng.standard_normal(L.ndofs); x0[dm] = 0
        for steps in (1, 2):
            xg = dev(x0)
            g.smooth(dev(b), xg, steps=steps, level=l)
            err = rel(host(xg), o.smoothers[l].smooth(b, x0.copy(), steps, L.apply))
            assert err < (1e-12 if precision == 0 else 1e-5), (l, steps, err)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_diagonal_vanka_every_level(name, precision):
    """The diagonal Vanka (local_solver 1; reading G22: spatial mass and
    stiffness blocks of the patch replaced by their diagonals, temporal
    coupling and divergence exact) against the oracle's dense inverse of that
    patch matrix: one and two sweeps, 1e-12 in FP64, 1e-5 in FP32."""
    g, o = solver(name, local_solver=1, precision=precision), oracle_mg(name, "diagonal")
    rng = np.random.default_rng(17)
    for l, L in enumerate(o.levels[:-1]):
        dm = L.dirichlet_mask()
        b = rng.standard_normal(L.ndofs); b[dm] = 0
        x0 = rng.standard_normal(L.ndofs); x0[dm] = 0
        for steps in (1, 2):
            xg = dev(x0)
            g.smooth(dev(b), xg, steps=steps, level=l)
            err = rel(host(xg), o.smoothers[l].smooth(b, x0.copy(), steps, L.apply))
            assert err < (1e-12 if precision == 0 else 1e-5), (l, steps, err)


@pytest.mark.parametrize("name", ["c5_small", "r1k1_n8", "c2_small"])
def test_diagonal_vanka_solve_iterations(name):
    """FGMRES with the V-cycle on the diagonal Vanka: identical iteration
    counts, solution within 1e-10 at 1e-10."""
    from oracle.fgmres import fgmres
    g, o = solver(name, local_solver=1), oracle_mg(name, "diagonal")
    L = o.levels[0]
    b = rhs(CONFIGS[name], 24)
    x = torch.empty(len(b), dtype=torch.float64, device="cuda")
    info = g.solve(dev(b), x, rtol=1e-10, max_it=100)
    xo, it, _ = fgmres(L.apply, o.vcycle, b, rtol=1e-10, max_it=100, restart=RESTART)
    announce(f"diagonal Vanka solve {name}: gpu {info['iterations']} oracle {it}")
    assert info["iterations"] == it
    xo = L.project_pressure(xo)
    assert np.linalg.norm(host(x) - xo) / np.linalg.norm(xo) < 1e-10


@pytest.mark.parametrize("name", NAMES)
def test_transfers_every_pair(name):
    """App. A: prolongation P and restriction P^T, <= 1e-12."""
    g, o = solver(name), oracle_mg(name)
    rng = np.random.default_rng(14)
    for l, P in enumerate(o.P):
        announce(f"transfer {name} pair {l}")
        xc = rng.standard_normal(P.shape[1])
        xf = torch.empty(P.shape[0], dtype=torch.float64, device="cuda")
        g.prolongate(dev(xc), xf, level=l)
        assert rel(host(xf), P @ xc) < 1e-12
        rf = rng.standard_normal(P.shape[0])
        bc = torch.empty(P.shape[1], dtype=torch.float64, device="cuda")
        g.restrict(dev(rf), bc, level=l)
        assert rel(host(bc), P.T @ rf) < 1e-12


SPLIT_NAMES = [n for n in NAMES if CONFIGS[n]["n_sub"] > 1]


@pytest.mark.parametrize("name", SPLIT_NAMES)
@pytest.mark.parametrize("order", [1, 2], ids=["components_outer", "components_inner"])
def test_apply_subinterval_split(name, order):
    """The operator's cell kernel with every split of the slab among waves:
    one subinterval per wave (the jump term of Eq. (InAlg) read from the
    previous subinterval's nodes) up to all N subintervals walked by one wave
    (the jump term carried in registers), in FP64 (1e-12) and in the FP32
    V-cycle precision (1e-5 of the largest row; unit roundoff 6e-8), with
    either loop order of the FP32 3D cell kernel."""
    g64, g32, o = solver(name), solver(name, precision=1), oracle_mg(name)
    rng = np.random.default_rng(12)
    try:
        g32.set_option(3, order)
        for l, L in enumerate(o.levels):
            x = rng.standard_normal(L.ndofs)
            ref = L.csr() @ x
            N = L.N
            for nper in sorted({1, 2, N} & set(range(1, N + 1))):
                y = torch.empty(L.ndofs, dtype=torch.float64, device="cuda")
                g64.set_option(1, nper)
                g64.apply(dev(x), y, level=l)
                e64 = rel(host(y), ref)
                g32.set_option(1, nper)
                g32.apply_vcycle_precision(dev(x), y, level=l)
                e32 = rel(host(y), ref)
                announce(f"split {name} level {l} N={N} nper={nper} order {order}: fp64 {e64:.2e} fp32 {e32:.2e}")
                assert e64 < 1e-12
                assert e32 < 1e-5
    finally:
        g64.set_option(1, 0)
        g32.set_option(1, 0)
        g32.set_option(3, 0)


@pytest.mark.parametrize("name", NAMES)
def test_coarse_solve(name):
    """Alg. 1 step 3: bordered direct solve, mean-zero pressure."""
    g, o = solver(name), oracle_mg(name)
    L = o.levels[-1]
    rng = np.random.default_rng(15)
    b = rng.standard_normal(L.ndofs)
    x = torch.empty(L.ndofs, dtype=torch.float64, device="cuda")
    g.coarse_solve(dev(b), x)
    err = rel(host(x), o.coarse.solve(b))
    announce(f"coarse {name}: {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("name", NAMES)
def test_vcycle(name):
    """Alg. 1: one V-cycle from zero."""
    g, o = solver(name), oracle_mg(name)
    b = rhs(CONFIGS[name], 21)
    x = torch.empty(len(b), dtype=torch.float64, device="cuda")
    g.vcycle(dev(b), x)
    err = rel(host(x), o.vcycle(b))
    announce(f"vcycle {name}: {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("name", NAMES)
def test_solve_iterations_and_solution(name):
    """FGMRES + V-cycle: identical iteration counts, solution within 1e-10."""
    from oracle.fgmres import fgmres
    g, o = solver(name), oracle_mg(name)
    L = o.levels[0]
    b = rhs(CONFIGS[name], 22)
    for rtol in (1e-8, 1e-10):
        x = torch.empty(len(b), dtype=torch.float64, device="cuda")
        info = g.solve(dev(b), x, rtol=rtol, max_it=100)
        xo, it, hist = fgmres(L.apply, o.vcycle, b, rtol=rtol, max_it=100, restart=RESTART)
        announce(f"solve {name} rtol {rtol}: gpu {info['iterations']} oracle {it}")
        assert info["iterations"] == it
        assert info["rel_residual"] <= rtol
        xo = L.project_pressure(xo)
        assert np.linalg.norm(host(x) - xo) / np.linalg.norm(xo) < 100 * rtol
        if rtol == 1e-10:
            assert np.linalg.norm(host(x) - xo) / np.linalg.norm(xo) < 1e-10


def test_c1_manufactured_solution():
    """C1 (2D, 840 dofs, manufactured forcing assembled by the oracle), FGMRES
    to 1e-10: equals the oracle's bordered direct solve."""
    from oracle.coarse import CoarseSolver
    from oracle.errors import load_vector
    from stmg_inputs import Manufactured2D
    g, o = solver("c1"), oracle_mg("c1")
    L = o.levels[0]
    b = load_vector(L, Manufactured2D(1.0).f)
    x = torch.empty(L.ndofs, dtype=torch.float64, device="cuda")
    info = g.solve(dev(b), x, rtol=1e-10)
    xd = CoarseSolver(L).solve(b)
    assert info["rel_residual"] <= 1e-10
    assert np.linalg.norm(host(x) - xd) / np.linalg.norm(xd) < 1e-9


@pytest.mark.parametrize("name", ["c2_small", "c5_small"])
def test_mixed_precision_solution(name):
    """FP32 V-cycle inside FP64 FGMRES: converges to the same solution
    (within 1e-8 of the FP64 solution when both are solved to 1e-10)."""
    g64 = solver(name)
    g32 = solver(name, precision=1)
    b = dev(rhs(CONFIGS[name], 23))
    x64 = torch.empty_like(b)
    x32 = torch.empty_like(b)
    i64 = g64.solve(b, x64, rtol=1e-10)
    i32 = g32.solve(b, x32, rtol=1e-10)
    announce(f"mixed {name}: fp64 {i64['iterations']} it, fp32 {i32['iterations']} it")
    assert i32["rel_residual"] <= 1e-10
    err = (torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)).item()
    assert err < 1e-8, err
    assert i32["iterations"] <= i64["iterations"] + 3


def test_pressure_projection():
    from gpu_common import oracle_mg as om
    g, o = solver("c5_small"), om("c5_small")
    L = o.levels[0]
    x = np.random.default_rng(16).standard_normal(L.ndofs)
    xg = dev(x)
    g.project_pressure(xg)
    assert rel(host(xg), L.project_pressure(x)) < 1e-12


def test_zero_right_hand_side():
    """b = 0: no iteration, x = 0, relative residual 0."""
    from paper_2502_09159_amd import stmg
    g = solver("c5_small")
    b = torch.zeros(g.ndofs(0), dtype=torch.float64, device="cuda")
    x = torch.full_like(b, 7.0)
    info = g.solve(b, x, rtol=1e-8)
    announce(f"zero rhs: {info['iterations']} iterations")
    assert info["iterations"] == 0
    assert torch.count_nonzero(x).item() == 0
