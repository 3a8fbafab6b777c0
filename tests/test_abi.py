"""CPU checks of the C ABI: the library loads without a GPU, exports every
function include/stmg.h declares, and its host-only calls (parameters,
hierarchy) behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2502_09159_amd", "libstmg.so")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "stmg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stmg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libstmg.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2502_09159_amd import stmg
    assert set(declared_functions()) <= set(stmg.EXPORTED)


def test_binding_constants_match_the_header():
    from paper_2502_09159_amd import stmg
    text = open(os.path.join(ROOT, "include", "stmg.h")).read()
    defines = dict(re.findall(r"#define\s+(STMG_[A-Z_]+)\s+(\d+)", text))
    assert int(defines["STMG_RESTART"]) == stmg.RESTART
    assert int(defines["STMG_NET_PARAMS"]) == stmg.NET_PARAMS


def test_hierarchy_matches_oracle_rule():
    from oracle.hierarchy import build_levels
    from paper_2502_09159_amd import stmg
    cases = [dict(dim=2, n_cells_1d=4, n_coarse_1d=1, r=1, k=1, n_sub=2),
             dict(dim=2, n_cells_1d=4, n_coarse_1d=1, r=1, k=1, n_sub=2, time_h_coarsening=1),
             dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=2, k=2, n_sub=4, k_min=0, time_h_coarsening=1),
             dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=2, k=2, n_sub=4, k_min=0),
             dict(dim=3, n_cells_1d=32, n_coarse_1d=2, r=2, k=1, n_sub=8),
             dict(dim=3, n_cells_1d=8, n_coarse_1d=1, r=2, k=2, n_sub=8, time_h_coarsening=0),
             dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=2, k=2, n_sub=4, k_min=0, placement=1),
             dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=2, k=2, n_sub=4, k_min=0, placement=1,
                  time_h_coarsening=1),
             dict(dim=3, n_cells_1d=32, n_coarse_1d=2, r=2, k=1, n_sub=8, time_h_coarsening=1),
             dict(dim=3, n_cells_1d=6, n_coarse_1d=3, r=1, k=1, n_sub=1),
             dict(dim=3, n_cells_1d=12, n_coarse_1d=3, r=2, k=0, n_sub=2, k_min=0)]
    for c in cases:
        got = stmg.hierarchy(**c)
        ref = build_levels(c["n_cells_1d"], c["r"], c["k"], c["n_sub"], c["n_coarse_1d"], c.get("r_min", 1),
                           c.get("k_min", 1), c.get("time_h_coarsening", 0) == 1,
                           "top" if c.get("placement", 0) == 1 else "paper")
        assert got == [(l["n"], l["r"], l["k"], l["N"]) for l in ref]


def test_invalid_parameters_are_rejected():
    from paper_2502_09159_amd import stmg
    with pytest.raises(stmg.StmgError):
        stmg.hierarchy(dim=4)
    with pytest.raises(stmg.StmgError):
        stmg.hierarchy(n_cells_1d=6)                  # 6 = 2 * 3: not n_coarse_1d (2) times a power of two
    with pytest.raises(stmg.StmgError):
        stmg.hierarchy(n_cells_1d=4, n_coarse_1d=8)
    with pytest.raises(stmg.StmgError):
        stmg.hierarchy(r=3)
    with pytest.raises(stmg.StmgError):
        stmg.hierarchy(n_sub=16)
