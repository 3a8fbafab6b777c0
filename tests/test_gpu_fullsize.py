"""Parity at the benchmark's full size (C5: 3D Q3/P2disc x DG(1), 32^3
deformed hex mesh, slab of 8 subintervals, nu(x) = exp(0.5 g(x)), 49,051,184
dofs), in the configuration bench.py times, on sampled outputs that the
oracle computes one by one (oracle/sampled.py):

  * rows of the FP64 operator (the FGMRES operator) -- every kind of row:
    interior and Dirichlet velocity rows of every temporal dof, pressure rows,
    first and later subintervals;
  * entries of the smoother correction on the finest level, in the mixed
    context the benchmark runs (FP32 local solves on the matrix cores) and in
    an FP64 context;
  * rows of the FP32 operator of the mixed V-cycle, whose cell kernel walks
    all 8 subintervals of a cell in one wave (the jump term carried in
    registers), the launch configuration the benchmark times;
  * entries of the learned correction on the Q2/P1 x DG(1) level below the
    finest (32^3, N = 8: 262,144 space-time cells, four inference chunks);
  * operator rows on every level of the C2 hierarchy (16^3 Q3/P2 x DG(2),
    N = 4, k -> 0) and of the C4 training hierarchy (16^3 Q2/P1 x DG(1),
    N = 2).

Tolerances: the FP64 operator is a sum-factorized evaluation of the same
integrals the oracle assembles, so rows agree to rounding (1e-12 of the
largest sampled row; measured 1e-17).  The FP64 correction applies inverses
factored in FP64, 1e-12 relative (measured 2e-15).  The FP32 correction
carries the FP32 rounding (unit roundoff 6e-8) of the stored factors and of
the products: 1e-5 relative, about 170 unit roundoffs (measured 9e-8).  The
FP32 operator rows: 1e-5 of the largest sampled row.  The learned
correction runs BF16 operands with FP32 accumulation against the FP64 oracle
network: 2e-2 relative L2 per sampled set."""
import numpy as np
import pytest
import torch

from gpu_common import announce, dev, host
from stmg_inputs import FourierViscosity, random_rhs

pytestmark = pytest.mark.gpu

C5 = dict(dim=3, n_cells_1d=32, n_coarse_1d=2, r=2, k=1, n_sub=8, deform_amp=0.03, k_min=1, tau=0.05, nu=1.0,
          omega=0.8)


@pytest.fixture(scope="module")
def nu():
    return FourierViscosity(5)


@pytest.fixture(scope="module")
def oracle_level(nu):
    from oracle.sampled import SampledLevel
    return SampledLevel(3, 32, 2, 1, 8, 0.05, 0.03, nu)


def sample_rows(S, rng):
    """Stratified sample: velocity rows (interior and Dirichlet) and pressure
    rows in the first, a middle and the last subinterval, every temporal dof."""
    rows = []
    for n in (0, 3, S.N - 1):
        for a in range(S.nt):
            for comp in range(S.d):
                g_in = rng.integers(1, S.nn - 1, size=(12, 3))
                for gc in g_in:
                    rows.append(S.v_dof(n, a, comp, S.node_index(list(gc))))
                # nodes on cell faces / edges / corners (shared by 2, 4, 8 cells)
                for _ in range(6):
                    gc = [int(rng.integers(1, S.n)) * S.q for _ in range(3)]
                    gc[int(rng.integers(0, 3))] = int(rng.integers(1, S.nn - 1))
                    rows.append(S.v_dof(n, a, comp, S.node_index(gc)))
                gc = [int(rng.integers(0, S.nn)) for _ in range(3)]
                gc[int(rng.integers(0, 3))] = 0
                rows.append(S.v_dof(n, a, comp, S.node_index(gc)))           # Dirichlet
            for c in rng.integers(0, S.n ** 3, size=6):
                for l in (0, S.C - 1):
                    rows.append(S.p_dof(n, a, int(c), l))
    return np.array(rows)


def test_fullsize_fp64_operator_rows(nu, oracle_level):
    from paper_2502_09159_amd import stmg
    S = oracle_level
    g = stmg.Solver(nu_fn=nu, precision=stmg.MIXED_FP32, **C5)
    try:
        assert g.ndofs(0) == S.ndofs
        rng = np.random.default_rng(51)
        x = rng.standard_normal(S.ndofs)
        yd = torch.empty(S.ndofs, dtype=torch.float64, device="cuda")
        g.apply(dev(x), yd)
        y = host(yd)
        rows = sample_rows(S, rng)
        ref = S.operator_rows(x, rows)
        err = np.max(np.abs(y[rows] - ref)) / np.max(np.abs(ref))
        announce(f"C5 full size: FP64 operator, {len(rows)} sampled rows, max error / max row {err:.2e}")
        assert err <= 1e-12
    finally:
        g.close()


def correction_samples(S, rng):
    rows = []
    for c in rng.integers(0, S.n ** 3, size=4):
        n = int(rng.integers(0, S.N))
        for a in range(S.nt):
            for l in range(S.C):
                rows.append(S.p_dof(n, a, int(c), l))
    for _ in range(6):
        n = int(rng.integers(0, S.N))
        gc = [int(v) for v in rng.integers(1, S.nn - 1, size=3)]
        if _ % 2 == 0:
            gc[0] = int(rng.integers(1, S.n)) * S.q   # on a cell face: two owning cells or more
        for a in range(S.nt):
            for comp in range(S.d):
                rows.append(S.v_dof(n, a, comp, S.node_index(gc)))
    return np.array(rows)


@pytest.mark.parametrize("prec", ["mixed", "fp64", "mixed_coupled"])
def test_fullsize_smoother_correction(nu, oracle_level, prec):
    """Decoupled local solves (the default) in the mixed and FP64 contexts,
    and the Schur-factored space-time form in the mixed context."""
    from paper_2502_09159_amd import stmg
    S = oracle_level
    p = stmg.FP64 if prec == "fp64" else stmg.MIXED_FP32
    mode = stmg.VANKA_FACTORED if prec == "mixed_coupled" else stmg.VANKA_DECOUPLED
    g = stmg.Solver(nu_fn=nu, precision=p, vanka_mode=mode, **C5)
    try:
        r = random_rhs(3, 32, 2, 1, 8, 52)
        rng = np.random.default_rng(53)
        r += 0.1 * rng.standard_normal(S.ndofs) * (r != 0)          # velocity rows
        nv = S.nt * S.Mv
        for n in range(S.N):                                          # pressure rows
            o = n * S.slab + nv
            r[o:o + S.nt * S.Mp] = rng.standard_normal(S.nt * S.Mp)
        x = torch.zeros(S.ndofs, dtype=torch.float64, device="cuda")
        g.vanka_correction(dev(r), x, level=0)
        u = host(x) / C5["omega"]
        rows = correction_samples(S, rng)
        ref = np.array([S.correction_entry(r, i) for i in rows])
        err = np.linalg.norm(u[rows] - ref) / np.linalg.norm(ref)
        announce(f"C5 full size: smoother correction ({prec}), {len(rows)} sampled entries, rel L2 error {err:.2e}")
        assert err <= (1e-12 if prec == "fp64" else 1e-5)
    finally:
        g.close()


def test_fullsize_fp32_operator_rows(nu, oracle_level):
    """The FP32 operator of the mixed V-cycle at C5 (8 subintervals per wave)."""
    from paper_2502_09159_amd import stmg
    S = oracle_level
    g = stmg.Solver(nu_fn=nu, precision=stmg.MIXED_FP32, **C5)
    try:
        rng = np.random.default_rng(54)
        x = rng.standard_normal(S.ndofs)
        yd = torch.empty(S.ndofs, dtype=torch.float64, device="cuda")
        g.apply_vcycle_precision(dev(x), yd)
        y = host(yd)
        rows = sample_rows(S, rng)
        ref = S.operator_rows(x, rows)
        err = np.max(np.abs(y[rows] - ref)) / np.max(np.abs(ref))
        announce(f"C5 full size: FP32 operator, {len(rows)} sampled rows, max error / max row {err:.2e}")
        assert err <= 1e-5
    finally:
        g.close()


def test_fullsize_learned_correction(nu):
    """The learned correction on the Q2/P1 x DG(1) level of C5 (level 1, 32^3,
    N = 8), four chunks of 65,536 space-time cells, against the oracle
    network cell by cell."""
    from oracle import learned as ln
    from oracle.sampled import SampledLevel
    from paper_2502_09159_amd import stmg
    from paper_2502_09159_amd.learned import he_init
    S = SampledLevel(3, 32, 1, 1, 8, 0.05, 0.03, nu)
    g = stmg.Solver(nu_fn=nu, precision=stmg.MIXED_FP32, **C5)
    try:
        assert g.ndofs(1) == S.ndofs
        w = he_init(17)
        g.learned_load(w)
        Ws = ln.unpack(w.astype(np.float64))
        rng = np.random.default_rng(55)
        r = rng.standard_normal(S.ndofs)
        u = host(g.learned_correction(dev(r), level=1))
        rows = []
        for n in (0, 3, 7):
            for c in rng.integers(0, S.n ** 3, size=3):
                for a in range(2):
                    rows += [S.p_dof(n, a, int(c), l) for l in range(4)]
            for _ in range(8):
                gc = [int(v) for v in rng.integers(1, S.nn - 1, size=3)]
                if _ % 2 == 0:
                    gc[_ % 3] = int(rng.integers(1, S.n)) * S.q
                for a in range(2):
                    for comp in range(3):
                        rows.append(S.v_dof(n, a, comp, S.node_index(gc)))
        rows = np.array(rows)
        ref = np.array([S.learned_correction_entry(Ws, r, i) for i in rows])
        err = np.linalg.norm(u[rows] - ref) / np.linalg.norm(ref)
        announce(f"C5 level 1: learned correction, {len(rows)} sampled entries, rel L2 error {err:.2e}")
        assert err <= 2e-2
    finally:
        g.close()


HIERARCHIES = {
    # C2: 16^3 deformed, Q3/P2 x DG(2), 4 subintervals, k -> 0
    "c2": dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=2, k=2, n_sub=4, deform_amp=0.03, k_min=0),
    # C4 training: 16^3 deformed, Q2/P1 x DG(1), 2 subintervals
    "c4_train": dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=1, k=1, n_sub=2, deform_amp=0.03, k_min=1),
}


@pytest.mark.parametrize("name", sorted(HIERARCHIES))
def test_operator_rows_every_level(name):
    """FP64 operator rows (sampled: interior, shared and Dirichlet velocity
    rows, pressure rows) on every level of the hierarchy at full size."""
    from oracle.sampled import SampledLevel
    from paper_2502_09159_amd import stmg
    cfg = HIERARCHIES[name]
    levels = stmg.hierarchy(**cfg)
    g = stmg.Solver(tau=0.05, nu=1.0, omega=0.8, **cfg)
    try:
        rng = np.random.default_rng(56)
        for l, (n, r, k, N) in enumerate(levels):
            S = SampledLevel(3, n, r, k, N, 0.05, 0.03, 1.0)
            assert g.ndofs(l) == S.ndofs
            x = rng.standard_normal(S.ndofs)
            yd = torch.empty(S.ndofs, dtype=torch.float64, device="cuda")
            g.apply(dev(x), yd, level=l)
            y = host(yd)
            rows = []
            for nn_ in sorted({0, N - 1}):
                for a in range(S.nt):
                    for comp in range(3):
                        for _ in range(4):
                            gc = [int(v) for v in rng.integers(1, S.nn - 1, size=3)]
                            if _ % 2 == 1:
                                gc[_ % 3] = int(rng.integers(1, S.n)) * S.q if S.n > 1 else gc[_ % 3]
                            rows.append(S.v_dof(nn_, a, comp, S.node_index(gc)))
                        gc = [int(v) for v in rng.integers(0, S.nn, size=3)]
                        gc[comp] = S.nn - 1
                        rows.append(S.v_dof(nn_, a, comp, S.node_index(gc)))
                    for c in rng.integers(0, S.n ** 3, size=2):
                        rows += [S.p_dof(nn_, a, int(c), 0), S.p_dof(nn_, a, int(c), S.C - 1)]
            rows = np.array(rows)
            ref = S.operator_rows(x, rows)
            err = np.max(np.abs(y[rows] - ref)) / np.max(np.abs(ref))
            announce(f"{name} level {l} ({n}^3 r{r} k{k} N{N}): {len(rows)} rows, max error / max row {err:.2e}")
            assert err <= 1e-12
    finally:
        g.close()
