"""Element and global spatial matrices (test infrastructure).

Eq. (DefMAB): velocity mass M_h, vector Laplacian A_h (with the viscosity
nu(x) inside the integral, from the weak form of Problem (DVP); reading G2),
divergence B_h and pressure mass M_h^p.  Quadrature: tensor Gauss rule with
r+2 points per direction (reading G11).  Velocity matrices are assembled for one
scalar component; the d-component blocks are I_d (x) scalar, component-major.
"""
import numpy as np
import scipy.sparse as sp

from . import elements as el
from .mesh import Mesh, VelocityDofs


def quad_rule(d, npts):
    x1, w1 = el.gauss_01(npts)
    return el.tensor_points(x1, d), el.tensor_weights(w1, d)


class SpatialLevel:
    """All spatial data of one (mesh, r) pair.

    nu: constant, or callable nu(points (n, d)) -> (n,) evaluated at the
    physical quadrature points.
    """

    def __init__(self, d, n, r, amp=0.0, nu=1.0):
        self.d, self.n, self.r = d, n, r
        self.mesh = Mesh(d, n, amp)
        self.vdofs = VelocityDofs(self.mesh, r)
        self.Q = r + 2
        self.C = el.n_pressure(d, r)
        self.nloc = self.Q ** d
        self.n_nodes = self.vdofs.n_nodes
        self.Mv = d * self.n_nodes          # velocity dofs per slice
        self.Mp = self.mesh.n_cells * self.C  # pressure dofs per slice
        self.nu = nu
        self._element_matrices()
        self._assemble()

    # ------------------------------------------------------------ elements
    def _element_matrices(self):
        d, r = self.d, self.r
        xq, wq = quad_rule(d, r + 2)
        phi, dphi = el.velocity_basis(d, r, xq)
        psi = el.pressure_values(d, r, xq)
        nc, nl, C = self.mesh.n_cells, self.nloc, self.C
        self.Me = np.zeros((nc, nl, nl))
        self.Ae = np.zeros((nc, nl, nl))
        self.Be = np.zeros((nc, C, d, nl))   # B[l, comp, node]
        self.Mpe = np.zeros((nc, C, C))
        self.moments = np.zeros((nc, C))     # int_K psi_l dx
        self.volume = np.zeros(nc)
        for c in range(nc):
            x, J = self.mesh.map(c, xq)
            det = np.linalg.det(J)
            if np.any(det <= 0):
                raise ValueError("inverted cell")
            Jinv = np.linalg.inv(J)                    # [p, j, i] = dxi_j/dx_i
            nu = self.nu(x) if callable(self.nu) else np.full(len(wq), float(self.nu))
            jxw = det * wq
            grad = np.einsum("pij,pnj->pni", np.transpose(Jinv, (0, 2, 1)), dphi)  # physical grads
            self.Me[c] = np.einsum("p,pa,pb->ab", jxw, phi, phi)
            self.Ae[c] = np.einsum("p,pai,pbi->ab", jxw * nu, grad, grad)
            self.Be[c] = np.einsum("p,pl,pni->lin", jxw, psi, grad)
            self.Mpe[c] = np.einsum("p,pl,pm->lm", jxw, psi, psi)
            self.moments[c] = np.einsum("p,pl->l", jxw, psi)
            self.volume[c] = jxw.sum()

    # ------------------------------------------------------------ globals
    def _assemble(self):
        cn = self.vdofs.cell_nodes
        nc, nl, C, d = self.mesh.n_cells, self.nloc, self.C, self.d
        rows = np.repeat(cn[:, :, None], nl, axis=2).ravel()
        cols = np.repeat(cn[:, None, :], nl, axis=1).ravel()
        N = self.n_nodes
        self.Ms = sp.csr_matrix((self.Me.ravel(), (rows, cols)), shape=(N, N))
        self.As = sp.csr_matrix((self.Ae.ravel(), (rows, cols)), shape=(N, N))
        # B: pressure row (cell, l), velocity column comp*N + node
        prow = (np.arange(nc)[:, None, None, None] * C + np.arange(C)[None, :, None, None])
        prow = np.broadcast_to(prow, (nc, C, d, nl)).ravel()
        vcol = (np.arange(d)[None, None, :, None] * N + cn[:, None, None, :])
        vcol = np.broadcast_to(vcol, (nc, C, d, nl)).ravel()
        self.B = sp.csr_matrix((self.Be.ravel(), (prow, vcol)), shape=(nc * C, d * N))
        self.Mh = sp.kron(sp.identity(d), self.Ms, format="csr")
        self.Ah = sp.kron(sp.identity(d), self.As, format="csr")
        self.Mp_glob = sp.block_diag(list(self.Mpe), format="csr")
        self.vel_boundary = np.tile(self.vdofs.boundary, d)      # per velocity dof
        self.vel_valence = np.tile(self.vdofs.valence, d)
        self.mom_glob = self.moments.ravel()                      # M_h^p 1 per pressure dof
