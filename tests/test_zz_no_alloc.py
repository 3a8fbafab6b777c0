"""The allocation-free Vanka correction (stmg_vanka_correction_noalloc) against
stmg_vanka_correction through the C ABI: the same kernels on a fixed scratch
buffer, so the results are equal bit for bit.  Two calls in a row share the
buffer, the second on a smaller level; a level whose scratch exceeds the
buffer is rejected with STMG_EINVAL."""
import numpy as np
import pytest
import torch

from gpu_common import announce, dev

pytestmark = pytest.mark.gpu

CFG = dict(dim=3, n_cells_1d=8, n_coarse_1d=2, r=2, k=1, n_sub=4, deform_amp=0.03, k_min=1, tau=0.05, nu=1.0,
           omega=0.8)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_noalloc_correction_equals_the_allocating_one(precision):
    from paper_2502_09159_amd import stmg
    g = stmg.Solver(precision=precision, **CFG)
    try:
        rng = np.random.default_rng(61)
        for level in (0, 1):                      # the second call: a smaller level
            n = g.ndofs(level)
            r = dev(rng.standard_normal(n))
            x0 = dev(rng.standard_normal(n))
            xa = x0.clone()
            g.vanka_correction(r, xa, level=level)
            xb = x0.clone()
            g.vanka_correction_noalloc(r, xb, level=level)
            torch.cuda.synchronize()
            diff = (xa - xb).abs().max().item()
            announce(f"noalloc precision {precision} level {level} ({n} dofs): max difference {diff:.1e}")
            assert torch.equal(xa, xb)
            assert (xa - x0).abs().max().item() > 0
    finally:
        g.close()


def test_noalloc_rejects_a_level_beyond_the_buffer():
    from paper_2502_09159_amd import stmg
    cfg = dict(CFG, n_cells_1d=16, n_sub=8)       # E of level 0: 4096 cells x 3 x 2 x 64 x 8 doubles = 100 MB
    g = stmg.Solver(precision=0, **cfg)
    try:
        n = g.ndofs(0)
        r = torch.zeros(n, dtype=torch.float64, device="cuda")
        x = torch.zeros_like(r)
        with pytest.raises(stmg.StmgError) as e:
            g.vanka_correction_noalloc(r, x, level=0)
        assert e.value.code == -1
        assert "scratch" in str(e.value)
    finally:
        g.close()
