"""CPU checks of the byte and flop accounting the benchmark's roofline
entries divide by: the counts are written out here by hand for C5 (3D
Q3/P2disc x DG(1), 32^3 cells, 8 subintervals) and compared with the
formulas in bench.py."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

C5 = bench.WORKLOADS["c5"]


def test_c5_sizes():
    d, nl, nt, C, N, ncells, ndofs = bench.element_sizes(C5)
    assert (d, nl, nt, C, N, ncells) == (3, 64, 2, 10, 8, 32768)
    # velocity: 3 components on the (3 * 32 + 1)^3 Gauss-Lobatto grid; pressure:
    # 10 Legendre modes per cell; both for 2 temporal dofs of 8 subintervals
    assert ndofs == 8 * 2 * (3 * 97 ** 3 + 32768 * 10) == 49_051_184


def test_c5_decoupled_local_solve_bytes():
    # per cell: Re and Im of the one complex 64 x 64 spatial inverse, symmetric
    # and stored as its 10 upper 16 x 16 tiles (2 * 10 * 256), B (10 x 3 x 64),
    # F (3 x 64 rows of 10 complex values), H^-1 (10 x 10 complex)
    per_cell = 2 * 10 * 256 + 10 * 3 * 64 + 3 * 64 * 2 * 10 + 10 * 2 * 10
    assert per_cell == 11_080
    corrections = 32768 * 3 * 2 * 64 * 8  # E: every cell's velocity correction once
    pressure = 2 * 32768 * 10 * 2 * 8     # the pressure unknowns read and written
    expected = 4 * (32768 * per_cell + 49_051_184 + corrections + pressure)
    assert bench.vanka_form(C5) == "decoupled"
    assert bench.vanka_local_bytes(C5, 4) == expected == 2_093_078_720


def test_c5_operator_bytes():
    # x, b and r once, plus the per-Gauss-point metric (1 + 9 + 6 values at the
    # 64 points of each cell)
    assert bench.operator_bytes(C5, 4) == 4 * (3 * 49_051_184 + 32768 * 16 * 64)


def test_schedule_defaults():
    assert (bench.PRE, bench.POST, bench.OMEGA) == (1, 2, 0.8)
    p = bench.solver_params(dict(C5), 1)
    assert (p["nu_pre"], p["nu_post"], p["omega"]) == (1, 2, 0.8)
