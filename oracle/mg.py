"""The hp space-time V-cycle (test infrastructure).

Alg. 1 with the subroutines Alg. 4-7: presmoothing (Eq. (Alg:VGMGPre)),
residual and restriction to the next coarser level of the list (p- or
h-transfer, whichever the pair of levels differs in), recursion or the
coarsest-level direct solve, prolongation and correction, postsmoothing
(Eq. (Alg:VGMGPost)).  Levels are rediscretised (Eq. (LSMG)).  The V-cycle
starts from a zero initial guess and is used as the preconditioner of
(F)GMRES (Sec. 4.4).
"""
import numpy as np

from .assembly import SpatialLevel
from .coarse import CoarseSolver
from .hierarchy import build_levels
from .spacetime import SpaceTimeLevel
from .transfer import prolongation
from .vanka import Vanka


class Multigrid:
    def __init__(self, d, n, r, k, N, tau, nu=1.0, amp=0.0, n_coarse=1, r_min=1,
                 k_min=1, time_h=False, omega=0.8, nu_pre=1, nu_post=1, literal=None,
                 placement="paper", smoother="exact"):
        self.spec = build_levels(n, r, k, N, n_coarse, r_min, k_min, time_h, placement)
        spatial = {}
        self.levels = []
        for s in self.spec:
            key = (s["n"], s["r"])
            if key not in spatial:
                spatial[key] = SpatialLevel(d, s["n"], s["r"], amp, nu)
            self.levels.append(SpaceTimeLevel(spatial[key], s["k"], s["N"], tau * N / s["N"]))
        self.P = [prolongation(self.levels[i], self.levels[i + 1]) for i in range(len(self.levels) - 1)]
        self.smoothers = [Vanka(L, omega, literal, smoother) for L in self.levels[:-1]]
        self.coarse = CoarseSolver(self.levels[-1])
        self.nu_pre, self.nu_post = nu_pre, nu_post

    def apply(self, level, x):
        return self.levels[level].apply(x)

    def vcycle(self, b, level=0):
        """x = V(b) with zero initial guess on `level` (0 = finest)."""
        if level == len(self.levels) - 1:
            return self.coarse.solve(b)
        L = self.levels[level]
        sm = self.smoothers[level]
        x = np.zeros_like(b)
        x = sm.smooth(b, x, self.nu_pre, L.apply)
        r = b - L.apply(x)
        bc = self.P[level].T @ r
        y = self.vcycle(bc, level + 1)
        x = x + self.P[level] @ y
        x = sm.smooth(b, x, self.nu_post, L.apply)
        return x
