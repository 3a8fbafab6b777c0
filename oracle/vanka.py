"""Space-time cell Vanka smoother (test infrastructure).

Eq. (vanka0), (vanka): for every space-time cell T = K x I_n the local matrix
A_T = R_T S R_T^T over all dofs of T (all k+1 temporal dofs of I_n; reading
G7: the assembled level matrix restricted to T, neighbour contributions
included), the additive sum of local solves weighted by the inverse valence
(the remark on patch construction in Sec. 4.2; reading G9), and
x <- x + omega * D^{-1} sum_T R_T^T A_T^{-1} R_T (b - S x).

Since Dirichlet rows and columns of S are the identity, taking ALL dofs of the
cell (Dirichlet ones included) pads A_T with identity rows/columns; the update
is masked to zero on Dirichlet dofs.  A_T is the same for every subinterval
(uniform tau), so one inverse per spatial cell is stored.

On a mesh of one cell the patch K x I_n holds every spatial dof of its
subinterval, and A_T is singular exactly like the level matrix: the constant
pressure of each temporal dof is in its kernel (Eq. (DefRsSs)).  Such a patch
is solved in the mean-zero pressure space, bordered with the constraint
<p_a, M_h^p c_1> = 0 per temporal dof as the coarse solve is (reading G6).
"""
import numpy as np

from .spacetime import SpaceTimeLevel


def cell_dofs(L: SpaceTimeLevel, n):
    """Global indices of all dofs of every space-time cell K x I_n:
    array (n_cells, b) in the local order [a][comp][node] then [a][mode]."""
    s = L.sp
    cn = s.vdofs.cell_nodes                                  # (nc, Q^d)
    nc = s.mesh.n_cells
    parts = []
    for a in range(L.nt):
        base = L.v_index(n, a).start
        for c in range(s.d):
            parts.append(base + c * s.n_nodes + cn)
    for a in range(L.nt):
        base = L.p_index(n, a).start
        parts.append(base + np.arange(nc)[:, None] * s.C + np.arange(s.C)[None, :])
    return np.concatenate(parts, axis=1)


def local_matrices_literal(L: SpaceTimeLevel):
    """A_T = S[idx_T, idx_T] extracted from the literal global CSR."""
    S = L.csr()
    idx = cell_dofs(L, 0)
    return np.array([S[i][:, i].toarray() for i in idx])


def local_matrices_factored(L: SpaceTimeLevel, cells=None):
    """The same blocks built from the spatial matrices (Kronecker form of the
    per-subinterval block D); used where the literal CSR is too large.
    `cells` restricts the construction to a subset of cells."""
    s = L.sp
    cn = s.vdofs.cell_nodes
    nc, d, C, nt = s.mesh.n_cells, s.d, s.C, L.nt
    out = []
    for T in (range(nc) if cells is None else cells):
        iv = np.concatenate([c * s.n_nodes + cn[T] for c in range(d)])
        ip = T * C + np.arange(C)
        fv = ~s.vel_boundary[iv]
        keep = np.outer(fv, fv).astype(float)
        Mloc = s.Mh[iv][:, iv].toarray() * keep
        Aloc = s.Ah[iv][:, iv].toarray() * keep
        Bloc = s.B[ip][:, iv].toarray() * fv[None, :].astype(float)
        Avv = np.kron(L.K, Mloc) + np.kron(L.Mtau, Aloc)
        Avv += np.kron(np.eye(nt), np.diag((~fv).astype(float)))
        Avp = -np.kron(L.Mtau, Bloc.T)
        Apv = -np.kron(L.Mtau, Bloc)
        App = np.zeros((nt * C, nt * C))
        out.append(np.block([[Avv, Avp], [Apv, App]]))
    return np.array(out)


def local_matrices_diagonal(L: SpaceTimeLevel, cells=None):
    """The cheaper patch matrices of the diagonal Vanka (reading G22): A_T of
    `local_matrices_factored` with its spatial velocity blocks replaced by
    their diagonals, K (x) diag(M_T) + M^tau (x) diag(A_T), while the coupling
    of the k+1 temporal dofs and the divergence blocks stay exact (same
    Dirichlet padding)."""
    s = L.sp
    cn = s.vdofs.cell_nodes
    nc, d, C, nt = s.mesh.n_cells, s.d, s.C, L.nt
    out = []
    for T in (range(nc) if cells is None else cells):
        iv = np.concatenate([c * s.n_nodes + cn[T] for c in range(d)])
        ip = T * C + np.arange(C)
        fv = ~s.vel_boundary[iv]
        Mdiag = np.diag(s.Mh[iv][:, iv].diagonal() * fv)
        Adiag = np.diag(s.Ah[iv][:, iv].diagonal() * fv)
        Bloc = s.B[ip][:, iv].toarray() * fv[None, :].astype(float)
        Avv = np.kron(L.K, Mdiag) + np.kron(L.Mtau, Adiag)
        Avv += np.kron(np.eye(nt), np.diag((~fv).astype(float)))
        Avp = -np.kron(L.Mtau, Bloc.T)
        Apv = -np.kron(L.Mtau, Bloc)
        App = np.zeros((nt * C, nt * C))
        out.append(np.block([[Avv, Avp], [Apv, App]]))
    return np.array(out)


def bordered_inverse(L: SpaceTimeLevel, A):
    """Inverse of the whole-domain patch matrices A (one cell) in the mean-zero
    pressure space: the top-left block of [[A, Z], [Z^T, 0]]^{-1}, Z holding
    the cell's pressure moments at the pressure slots of each temporal dof."""
    s = L.sp
    b = A.shape[1]
    p0 = L.nt * s.d * s.nloc                      # first pressure slot
    Z = np.zeros((b, L.nt))
    for a in range(L.nt):
        Z[p0 + a * s.C:p0 + (a + 1) * s.C, a] = s.mom_glob
    out = np.empty_like(A)
    for c in range(A.shape[0]):
        Ab = np.block([[A[c], Z], [Z.T, np.zeros((L.nt, L.nt))]])
        out[c] = np.linalg.inv(Ab)[:b, :b]
    return out


class Vanka:
    """kind "exact": the patch matrices of Eq. (vanka0); "diagonal": the
    cheaper ones of `local_matrices_diagonal`."""

    def __init__(self, L: SpaceTimeLevel, omega, literal=None, kind="exact"):
        self.L = L
        self.omega = float(omega)
        if literal is None:
            literal = L.ndofs <= 200_000
        if kind == "diagonal":
            A = local_matrices_diagonal(L)
        else:
            A = local_matrices_literal(L) if literal else local_matrices_factored(L)
        self.inv = bordered_inverse(L, A) if L.sp.mesh.n_cells == 1 else np.linalg.inv(A)
        self.idx = [cell_dofs(L, n) for n in range(L.N)]
        # valence D: number of spatial cells sharing the dof (pressure: 1)
        val = np.zeros(L.ndofs)
        for n in range(L.N):
            np.add.at(val, self.idx[n].ravel(), 1.0)
        self.inv_val = 1.0 / val
        self.dmask = L.dirichlet_mask()

    def correction(self, r):
        """sum_T R_T^T A_T^{-1} R_T r, weighted by 1/valence, zero on Dirichlet."""
        u = np.zeros_like(r)
        for n in range(self.L.N):
            idx = self.idx[n]
            y = np.einsum("cij,cj->ci", self.inv, r[idx])
            u += np.bincount(idx.ravel(), weights=y.ravel(), minlength=len(r))
        u *= self.inv_val
        u[self.dmask] = 0.0
        return u

    def smooth(self, b, x, steps, apply):
        """Eq. (vanka): x <- x + omega * smoother(S, b - S x), `steps` times."""
        for _ in range(steps):
            x = x + self.omega * self.correction(b - apply(x))
        return x
