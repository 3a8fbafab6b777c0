"""The diagonal Vanka's patch matrices (oracle/vanka.py, reading G22) against
the exact ones built independently from the literal global matrix: every
off-diagonal entry of a spatial velocity block vanishes, its diagonal and
the temporal and divergence couplings are those of the exact patch matrix."""
import numpy as np
import pytest

from oracle.assembly import SpatialLevel
from oracle.spacetime import SpaceTimeLevel
from oracle.vanka import local_matrices_diagonal, local_matrices_literal


@pytest.mark.parametrize("d,n,r,k", [(2, 3, 1, 1), (3, 2, 1, 2), (2, 2, 2, 0)])
def test_diagonal_patch_matrices_against_the_literal_ones(d, n, r, k):
    L = SpaceTimeLevel(SpatialLevel(d, n, r, 0.03, 1.3), k, 2, 0.07)
    exact = local_matrices_literal(L)
    diag = local_matrices_diagonal(L)
    s = L.sp
    nv = L.nt * d * s.nloc
    for A, Ad in zip(exact, diag):
        # pressure rows and columns identical
        assert np.allclose(Ad[nv:], A[nv:], rtol=0, atol=1e-13 * np.abs(A).max())
        assert np.allclose(Ad[:, nv:], A[:, nv:], rtol=0, atol=1e-13 * np.abs(A).max())
        for a in range(L.nt):
            for b in range(L.nt):
                for c1 in range(d):
                    for c2 in range(d):
                        r0 = (a * d + c1) * s.nloc
                        q0 = (b * d + c2) * s.nloc
                        blk, blk_d = A[r0:r0 + s.nloc, q0:q0 + s.nloc], Ad[r0:r0 + s.nloc, q0:q0 + s.nloc]
                        off = ~np.eye(s.nloc, dtype=bool)
                        assert np.all(blk_d[off] == 0.0)
                        if c1 == c2:
                            assert np.allclose(np.diag(blk_d), np.diag(blk), rtol=0, atol=1e-13 * np.abs(A).max())
                        else:
                            assert np.all(blk_d == 0.0)
