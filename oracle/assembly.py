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


def reference_tables(d, r):
    """Gauss rule with r+2 points per direction, velocity basis values and
    reference gradients, pressure basis values at those points."""
    xq, wq = quad_rule(d, r + 2)
    phi, dphi = el.velocity_basis(d, r, xq)
    psi = el.pressure_values(d, r, xq)
    return xq, wq, phi, dphi, psi


def cell_matrices(mesh, c, ref, nu):
    """Element matrices of cell c: mass, viscous Laplacian (nu inside),
    divergence B[l, comp, node], pressure mass, pressure moments, volume."""
    xq, wq, phi, dphi, psi = ref
    x, J = mesh.map(c, xq)
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("inverted cell")
    Jinv = np.linalg.inv(J)                    # [p, j, i] = dxi_j/dx_i
    nuq = nu(x) if callable(nu) else np.full(len(wq), float(nu))
    jxw = det * wq
    grad = np.einsum("pij,pnj->pni", np.transpose(Jinv, (0, 2, 1)), dphi)  # physical grads
    Me = np.einsum("p,pa,pb->ab", jxw, phi, phi)
    Ae = np.einsum("p,pai,pbi->ab", jxw * nuq, grad, grad)
    Be = np.einsum("p,pl,pni->lin", jxw, psi, grad)
    Mpe = np.einsum("p,pl,pm->lm", jxw, psi, psi)
    moments = np.einsum("p,pl->l", jxw, psi)
    return Me, Ae, Be, Mpe, moments, jxw.sum()


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
        d, nc, nl, C = self.d, self.mesh.n_cells, self.nloc, self.C
        self.Me = np.zeros((nc, nl, nl))
        self.Ae = np.zeros((nc, nl, nl))
        self.Be = np.zeros((nc, C, d, nl))   # B[l, comp, node]
        self.Mpe = np.zeros((nc, C, C))
        self.moments = np.zeros((nc, C))     # int_K psi_l dx
        self.volume = np.zeros(nc)
        ref = reference_tables(d, self.r)
        for c in range(nc):
            (self.Me[c], self.Ae[c], self.Be[c], self.Mpe[c], self.moments[c],
             self.volume[c]) = cell_matrices(self.mesh, c, ref, self.nu)

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
