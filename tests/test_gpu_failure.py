"""Failure handling of the solve: a V-cycle whose output is not finite (forced
from the host with the STMG_OPT_INJECT_NONFINITE test hook, which overwrites
one preconditioner output with NaN after every kernel has finished normally,
as an FP32 overflow would leave it) is detected in the Gram-Schmidt
coefficients, its step is redone with the unpreconditioned direction, and
the solve still converges to the same solution."""
import numpy as np
import pytest
import torch

from gpu_common import CONFIGS, announce, dev, make_solver, rhs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [1, 0], ids=["mixed", "fp64"])
@pytest.mark.parametrize("which", [1, 3])
def test_nonfinite_vcycle_falls_back(precision, which):
    from paper_2502_09159_amd import stmg
    g = make_solver(CONFIGS["c5_small"], precision=precision)
    try:
        b = dev(rhs(CONFIGS["c5_small"], 81))
        x0, x1 = torch.empty_like(b), torch.empty_like(b)
        plain = g.solve(b, x0, rtol=1e-10)
        g.set_option(stmg.OPT_INJECT_NONFINITE, which)
        info = g.solve(b, x1, rtol=1e-10)
        g.set_option(stmg.OPT_INJECT_NONFINITE, 0)
        err = (torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0)).item()
        announce(f"non-finite V-cycle #{which} (precision {precision}): fallbacks {info['vcycle_fallbacks']}, "
                 f"{info['iterations']} iterations against {plain['iterations']}, solution difference {err:.1e}")
        assert plain["vcycle_fallbacks"] == 0
        assert info["vcycle_fallbacks"] == 1
        assert info["rel_residual"] <= 1e-10
        assert np.isfinite(info["rel_residual"])
        assert err < 1e-8
        assert info["iterations"] <= plain["iterations"] + 3
    finally:
        g.close()
