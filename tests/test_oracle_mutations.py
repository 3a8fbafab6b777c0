"""Plant plausible mistakes in the oracle (on the CPU, one at a time, undone
after each test) and show that the pins of tests/test_oracle_mg_pins.py
catch each of them: a dropped valence weight, a dropped pre- or
postsmoothing step, a temporal index error in the prolongation and a wrong
pressure head of the learned correction."""
import numpy as np
import pytest

import oracle.learned as ln
import oracle.transfer as tr
from oracle import elements as el
from oracle.mg import Multigrid
from oracle.vanka import Vanka

import test_oracle_mg_pins as pins

CAUGHT = 1e-6  # every pin passes at <= 1e-12; a planted mistake must exceed this


def test_dropped_valence_weight_is_caught(monkeypatch):
    init = Vanka.__init__

    def no_valence(self, *a, **kw):
        init(self, *a, **kw)
        self.inv_val = np.ones_like(self.inv_val)

    monkeypatch.setattr(Vanka, "__init__", no_valence)
    assert pins.check_partition_of_unity(2, 3, 1, 1, 2) > CAUGHT
    assert pins.check_partition_of_unity(3, 2, 1, 1, 2) > CAUGHT


def _vcycle_without(step):
    def vcycle(self, b, level=0):
        if level == len(self.levels) - 1:
            return self.coarse.solve(b)
        L, sm = self.levels[level], self.smoothers[level]
        x = np.zeros_like(b)
        if step != "pre":
            x = sm.smooth(b, x, self.nu_pre, L.apply)
        y = self.vcycle(self.P[level].T @ (b - L.apply(x)), level + 1)
        x = x + self.P[level] @ y
        if step != "post":
            x = sm.smooth(b, x, self.nu_post, L.apply)
        return x
    return vcycle


@pytest.mark.parametrize("step,nu_pre,nu_post", [("post", 0, 1), ("pre", 1, 0)])
def test_dropped_smoothing_step_is_caught(monkeypatch, step, nu_pre, nu_post):
    assert pins.check_vcycle_whole_domain(2, nu_pre, nu_post) < 1e-12
    monkeypatch.setattr(Multigrid, "vcycle", _vcycle_without(step))
    assert pins.check_vcycle_whole_domain(2, nu_pre, nu_post) > CAUGHT


def test_temporal_index_errors_are_caught(monkeypatch):
    orig = tr.time_prolongation

    def swapped(kf, Nf, kc, Nc):  # the coarse temporal dofs of a subinterval swapped
        P = orig(kf, Nf, kc, Nc).copy()
        if kc >= 1:
            P[:, [0, 1]] = P[:, [1, 0]]
        return P

    def no_half_offset(kf, Nf, kc, Nc):  # both fine halves mapped like the first one
        tf, tc = el.radau_right(kf)[0], el.radau_right(kc)[0]
        ratio = Nf // Nc
        P = np.zeros((Nf * (kf + 1), Nc * (kc + 1)))
        for nf in range(Nf):
            nc = nf // ratio
            s = tf if ratio == 1 else (tf - 1) / 2.0
            P[nf * (kf + 1):(nf + 1) * (kf + 1), nc * (kc + 1):(nc + 1) * (kc + 1)] = el.lagrange_values(tc, s)
        return P

    monkeypatch.setattr(tr, "time_prolongation", swapped)
    assert pins.check_composite_prolongation(pins.PAIRS[0]) > CAUGHT
    assert pins.check_galerkin(pins.PAIRS[0]) > CAUGHT
    monkeypatch.setattr(tr, "time_prolongation", no_half_offset)
    assert pins.check_composite_prolongation(pins.PAIRS[1]) > CAUGHT
    assert pins.check_galerkin(pins.PAIRS[1]) > CAUGHT


def test_wrong_pressure_head_is_caught(monkeypatch):
    L = pins.level(3, 2, 1, 1, 2, amp=0.03)
    Ws = ln.init_weights(6)
    r_ = np.random.default_rng(7).standard_normal(L.ndofs)
    r_[L.dirichlet_mask()] = 0.0
    ref = pins.hand_built_learned(r_, Ws, 2, 2)
    monkeypatch.setattr(ln, "head", lambda y, mask: (y[:, :6, :] * (1.0 - mask[:, None, :]), y[:, 6:, 0]))
    assert pins.rel(ln.correction(L, Ws, r_), ref) > CAUGHT


def _march_cases():
    import test_oracle_marching as tm
    return tm, tm.CASES[0]


def test_wrong_sign_of_the_previous_slab_term_is_caught(monkeypatch):
    """C^1 V_0 entered with the wrong sign breaks reproduction and chaining."""
    import oracle.marching as mr
    tm, c = _march_cases()
    orig = mr.full_apply

    def flipped(L, x, v0=None):
        return orig(L, x, None if v0 is None else -v0)

    monkeypatch.setattr(mr, "full_apply", flipped)
    with pytest.raises(AssertionError):
        tm.test_constant_flow_is_reproduced(c)
    with pytest.raises(AssertionError):
        tm.test_two_slabs_equal_one_slab_of_twice_the_length(c)


def test_dropped_dirichlet_columns_in_the_lifting_are_caught(monkeypatch):
    """Lifting with the homogeneous operator (Dirichlet columns zero) loses
    the boundary data's coupling into the free rows."""
    import oracle.marching as mr
    tm, c = _march_cases()

    def homogeneous(L, x, v0=None):
        y = L.apply(x)
        if v0 is not None:
            for a in range(L.nt):
                y[L.v_index(0, a)] -= L.Ctau[a, -1] * (L.sp.Mh @ v0)
        return y

    monkeypatch.setattr(mr, "full_apply", homogeneous)
    with pytest.raises(AssertionError):
        tm.test_linear_in_time_flow_is_reproduced(c)
