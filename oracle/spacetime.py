"""The slab operator of Eq. (GloSys) on one level (test infrastructure).

Unknown ordering Eq. (DefX): X = (V_1, P_1, ..., V_N, P_N), V_n = (V_n^1..V_n^{k+1}),
P_n likewise; V_n^a is component-major over the global velocity nodes.

Per subinterval (Eq. (InAlg), (DefDtauh)) with the sign readings G1:
    D = [[K (x) M_h + M^tau (x) A_h,  -M^tau (x) B_h^T],
         [-M^tau (x) B_h,              0             ]]
and sub-diagonal blocks C^n = -C^tau (x) [M_h; 0] (Eq. (DefKMC) n > 1).
Homogeneous Dirichlet velocity dofs get identity rows and zero columns.
"""
import numpy as np
import scipy.sparse as sp

from . import elements as el
from .assembly import SpatialLevel


class SpaceTimeLevel:
    def __init__(self, spatial: SpatialLevel, k, N, tau):
        self.sp = spatial
        self.k, self.N, self.tau = k, N, float(tau)
        self.td = el.temporal_data(k)
        self.nt = k + 1
        self.Mv, self.Mp = spatial.Mv, spatial.Mp
        self.slab = self.nt * (self.Mv + self.Mp)   # dofs per subinterval
        self.ndofs = N * self.slab
        self.K = self.td["K"]
        self.Mtau = 0.5 * self.tau * self.td["M"]
        self.Ctau = np.outer(self.td["phim1"], np.eye(self.nt)[-1])  # C_ab = phi_a(-1) delta_{b,k+1}
        self.free_v = ~spatial.vel_boundary
        self._csr = None

    # --------------------------------------------------------- layout helpers
    def v_index(self, n, a):
        o = n * self.slab + a * self.Mv
        return slice(o, o + self.Mv)

    def p_index(self, n, a):
        o = n * self.slab + self.nt * self.Mv + a * self.Mp
        return slice(o, o + self.Mp)

    def dirichlet_mask(self):
        """True at every Dirichlet velocity entry of a global vector."""
        m = np.zeros(self.ndofs, dtype=bool)
        for n in range(self.N):
            for a in range(self.nt):
                m[self.v_index(n, a)] = self.sp.vel_boundary
        return m

    # ------------------------------------------------------------ factored
    def apply(self, x):
        """y = S x, evaluated block by block from the spatial matrices."""
        s = self.sp
        y = np.zeros_like(x)
        fv = self.free_v.astype(float)
        for n in range(self.N):
            Mx = [s.Mh @ (fv * x[self.v_index(n, b)]) for b in range(self.nt)]
            Ax = [s.Ah @ (fv * x[self.v_index(n, b)]) for b in range(self.nt)]
            if n > 0:
                Mprev = [s.Mh @ (fv * x[self.v_index(n - 1, b)]) for b in range(self.nt)]
            for a in range(self.nt):
                yv = np.zeros(self.Mv)
                yp = np.zeros(self.Mp)
                for b in range(self.nt):
                    yv += self.K[a, b] * Mx[b] + self.Mtau[a, b] * Ax[b]
                    yv -= self.Mtau[a, b] * (s.B.T @ x[self.p_index(n, b)])
                    yp -= self.Mtau[a, b] * (s.B @ (fv * x[self.v_index(n, b)]))
                    if n > 0:
                        yv -= self.Ctau[a, b] * Mprev[b]
                xv = x[self.v_index(n, a)]
                y[self.v_index(n, a)] = np.where(self.free_v, yv, xv)
                y[self.p_index(n, a)] = yp
        return y

    # ------------------------------------------------------------- literal
    def diag_block(self):
        """The per-subinterval block D (identical for every n at uniform tau)."""
        s = self.sp
        K, Mt = sp.csr_matrix(self.K), sp.csr_matrix(self.Mtau)
        Dvv = sp.kron(K, s.Mh) + sp.kron(Mt, s.Ah)
        Dvp = -sp.kron(Mt, s.B.T)
        Dpv = -sp.kron(Mt, s.B)
        Dpp = sp.csr_matrix((self.nt * self.Mp, self.nt * self.Mp))
        return sp.bmat([[Dvv, Dvp], [Dpv, Dpp]], format="csr")

    def coupling_block(self):
        s = self.sp
        Cvv = -sp.kron(sp.csr_matrix(self.Ctau), s.Mh)
        Z1 = sp.csr_matrix((self.nt * self.Mv, self.nt * self.Mp))
        Z2 = sp.csr_matrix((self.nt * self.Mp, self.nt * (self.Mv + self.Mp)))
        return sp.bmat([[sp.hstack([Cvv, Z1])], [Z2]], format="csr")

    def csr(self):
        """Literal global sparse matrix of Eq. (GloSys) with Dirichlet rows and
        columns replaced by the identity (small meshes only)."""
        if self._csr is not None:
            return self._csr
        D = self.diag_block()
        C = self.coupling_block()
        blocks = [[None] * self.N for _ in range(self.N)]
        for n in range(self.N):
            blocks[n][n] = D
            if n > 0:
                blocks[n][n - 1] = C
        S = sp.bmat(blocks, format="csr")
        dm = self.dirichlet_mask()
        keep = sp.diags((~dm).astype(float))
        S = (keep @ S @ keep + sp.diags(dm.astype(float))).tocsr()
        S.eliminate_zeros()
        self._csr = S
        return S

    # ------------------------------------------------------------ pressure
    def project_pressure(self, x):
        """Subtract, per slice, the L2 mean of the pressure (reading G6):
        p <- p - (<p, 1>/|Omega|) * 1, the constant having mode-0 coefficient 1."""
        x = x.copy()
        s = self.sp
        vol = s.volume.sum()
        for n in range(self.N):
            for a in range(self.nt):
                p = x[self.p_index(n, a)].reshape(s.mesh.n_cells, s.C)
                mean = np.sum(p * s.moments) / vol
                p[:, 0] -= mean
                x[self.p_index(n, a)] = p.ravel()
        return x

    def kernel_vectors(self):
        """Right null vectors of S: constant pressure in one slice."""
        vs = []
        for n in range(self.N):
            for a in range(self.nt):
                z = np.zeros(self.ndofs)
                p = np.zeros((self.sp.mesh.n_cells, self.sp.C))
                p[:, 0] = 1.0
                z[self.p_index(n, a)] = p.ravel()
                vs.append(z)
        return np.array(vs)

    def constraint_vectors(self):
        """Per slice, the vector (0, M_h^p c_1) of the mean-zero constraint."""
        vs = []
        for n in range(self.N):
            for a in range(self.nt):
                z = np.zeros(self.ndofs)
                z[self.p_index(n, a)] = self.sp.mom_glob
                vs.append(z)
        return np.array(vs)
