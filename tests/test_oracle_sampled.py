"""The sampled evaluation used at full size (oracle/sampled.py) against the
assembled oracle on small deformed meshes: every operator row and every
smoother-correction entry it produces must equal SpaceTimeLevel.apply and
Vanka.correction."""
import numpy as np
import pytest

from oracle.assembly import SpatialLevel
from oracle.sampled import SampledLevel
from oracle.spacetime import SpaceTimeLevel
from oracle.vanka import Vanka
from stmg_inputs import FourierViscosity

CASES = [
    dict(d=3, n=3, r=2, k=1, N=2, tau=0.05, amp=0.03, nu="fourier"),
    dict(d=3, n=2, r=1, k=2, N=3, tau=0.1, amp=0.03, nu=1.0),
    dict(d=2, n=4, r=2, k=1, N=2, tau=0.05, amp=0.05, nu=1.7),
]


def build(c):
    nu = FourierViscosity(5) if c["nu"] == "fourier" else c["nu"]
    if c["d"] == 2 and callable(nu):
        nu = 1.0
    sp = SpatialLevel(c["d"], c["n"], c["r"], c["amp"], nu)
    L = SpaceTimeLevel(sp, c["k"], c["N"], c["tau"])
    S = SampledLevel(c["d"], c["n"], c["r"], c["k"], c["N"], c["tau"], c["amp"], nu)
    return L, S


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"{c['d']}d_n{c['n']}_r{c['r']}_k{c['k']}")
def test_sampled_operator_rows_equal_the_assembled_operator(c):
    L, S = build(c)
    assert S.ndofs == L.ndofs
    rng = np.random.default_rng(3)
    x = rng.standard_normal(L.ndofs)
    y = L.apply(x)
    rows = np.arange(L.ndofs) if L.ndofs < 3000 else rng.choice(L.ndofs, 1500, replace=False)
    ys = S.operator_rows(x, rows)
    assert np.max(np.abs(ys - y[rows])) <= 1e-13 * np.max(np.abs(y))


@pytest.mark.parametrize("c", CASES[:2], ids=lambda c: f"{c['d']}d_n{c['n']}_r{c['r']}_k{c['k']}")
def test_sampled_correction_equals_the_vanka_correction(c):
    L, S = build(c)
    V = Vanka(L, 0.8)
    rng = np.random.default_rng(4)
    r = rng.standard_normal(L.ndofs)
    r[L.dirichlet_mask()] = 0.0
    u = V.correction(r)
    rows = rng.choice(L.ndofs, 120, replace=False)
    us = np.array([S.correction_entry(r, i) for i in rows])
    assert np.max(np.abs(us - u[rows])) <= 1e-10 * np.max(np.abs(u))


def test_sampled_learned_correction_equals_the_oracle_network():
    """learned_correction_entry (per cell, used at full size) against
    learned.correction over the whole level (reading G15: valence-weighted
    scatter of every cell's scaled network output, pressure per cell)."""
    from oracle import learned as ln
    L = SpaceTimeLevel(SpatialLevel(3, 3, 1, 0.03, 1.0), 1, 2, 0.05)
    S = SampledLevel(3, 3, 1, 1, 2, 0.05, 0.03, 1.0)
    W = ln.init_weights(3)
    rng = np.random.default_rng(6)
    r = rng.standard_normal(L.ndofs)
    u = ln.correction(L, W, r)
    rows = np.arange(L.ndofs)
    us = np.array([S.learned_correction_entry(W, r, i) for i in rows])
    assert np.max(np.abs(us - u)) <= 1e-13 * np.max(np.abs(u))
