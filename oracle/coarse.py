"""Direct solve on the coarsest level (test infrastructure).

Alg. 1 step 3 solves the coarsest system exactly.  The level matrix is
singular (one constant pressure per slice); the solution is sought in the
mean-zero pressure space (Eq. (DefRsSs)), here by bordering
[[S, Z], [Z^T, 0]] with one column Z = (0, M_h^p c_1) per slice (reading G6).
"""
import numpy as np
import scipy.linalg as sla

from .spacetime import SpaceTimeLevel


class CoarseSolver:
    def __init__(self, L: SpaceTimeLevel):
        self.L = L
        S = L.csr().toarray()
        Z = L.constraint_vectors().T
        m = Z.shape[1]
        A = np.block([[S, Z], [Z.T, np.zeros((m, m))]])
        self.n = S.shape[0]
        self.m = m
        self.lu = sla.lu_factor(A)

    def solve(self, b):
        rhs = np.concatenate([b, np.zeros(self.m)])
        return sla.lu_solve(self.lu, rhs)[: self.n]
