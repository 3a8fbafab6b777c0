"""Sampled outputs of the slab operator and of the cell Vanka on a full-size
level (test infrastructure).

At the benchmark's sizes (32^3 cells, Q3 velocity) the oracle cannot assemble
the global matrices.  One row of S x (Eq. (GloSys)) only involves the cells
that contain its node (or its cell, for a pressure row), and one local Vanka
solve (Eq. (vanka0)) only involves the cells around its cell.  This module
builds the element matrices of those cells alone, with the per-cell routine
of the assembly (`cell_matrices`), and evaluates

  * rows of S x exactly as `SpaceTimeLevel.apply` defines them (Dirichlet
    velocity rows are the identity, Dirichlet columns are zero);
  * entries of the smoother correction sum_T R_T^T A_T^{-1} R_T r weighted by
    1 / valence (zero on Dirichlet rows), with A_T built as in
    `vanka.local_matrices_factored` (the assembled level matrix restricted to
    the cell's dofs, neighbour contributions included).

Dof numbering is that of Eq. (DefX), see `SpaceTimeLevel`.
"""
from itertools import product

import numpy as np

from . import elements as el
from .assembly import cell_matrices, reference_tables
from .mesh import Mesh


class SampledLevel:
    def __init__(self, d, n, r, k, N, tau, amp=0.0, nu=1.0):
        self.d, self.n, self.r, self.k, self.N = d, n, r, k, N
        self.mesh = Mesh(d, n, amp)
        self.nu = nu
        self.Q, self.q = r + 2, r + 1
        self.nn = n * self.q + 1
        self.n_nodes = self.nn ** d
        self.nloc = self.Q ** d
        self.C = el.n_pressure(d, r)
        self.nt = k + 1
        self.Mv = d * self.n_nodes
        self.Mp = n ** d * self.C
        self.slab = self.nt * (self.Mv + self.Mp)
        self.ndofs = N * self.slab
        td = el.temporal_data(k)
        self.K = td["K"]
        self.Mtau = 0.5 * float(tau) * td["M"]
        self.Ctau = np.outer(td["phim1"], np.eye(self.nt)[-1])
        self.ref = reference_tables(d, r)
        self._em = {}
        self._lm = {}

    # ------------------------------------------------------------ geometry
    def node_coords(self, g):
        return [(g // self.nn ** j) % self.nn for j in range(self.d)]

    def node_index(self, gc):
        return sum(gc[j] * self.nn ** j for j in range(self.d))

    def is_boundary(self, g):
        return any(c == 0 or c == self.nn - 1 for c in self.node_coords(g))

    def cell_index(self, cc):
        return sum(cc[j] * self.n ** j for j in range(self.d))

    def cell_nodes(self, c):
        """Global nodes of cell c, local node i = sum_j i_j Q^j."""
        cc = self.mesh.cell_coords(c)
        out = []
        for i in range(self.nloc):
            ii = [(i // self.Q ** j) % self.Q for j in range(self.d)]
            out.append(self.node_index([cc[j] * self.q + ii[j] for j in range(self.d)]))
        return np.array(out)

    def cells_of_node(self, g):
        """Cells containing node g, with the node's local index in each."""
        gc = self.node_coords(g)
        options = []
        for j in range(self.d):
            o = []
            for c in (gc[j] // self.q - 1, gc[j] // self.q):
                i = gc[j] - c * self.q
                if 0 <= c < self.n and 0 <= i < self.Q:
                    o.append((c, i))
            options.append(o)
        out = []
        for combo in product(*options):
            c = self.cell_index([cj for cj, _ in combo])
            i = sum(ij * self.Q ** j for j, (_, ij) in enumerate(combo))
            out.append((c, i))
        return out

    def em(self, c):
        if c not in self._em:
            Me, Ae, Be, _, _, _ = cell_matrices(self.mesh, c, self.ref, self.nu)
            self._em[c] = (Me, Ae, Be, self.cell_nodes(c))
        return self._em[c]

    # --------------------------------------------------------- dof numbering
    def v_dof(self, n, a, comp, g):
        return n * self.slab + a * self.Mv + comp * self.n_nodes + g

    def p_dof(self, n, a, c, l):
        return n * self.slab + self.nt * self.Mv + a * self.Mp + c * self.C + l

    def decode(self, idx):
        n, rem = divmod(int(idx), self.slab)
        if rem < self.nt * self.Mv:
            a, rem = divmod(rem, self.Mv)
            comp, g = divmod(rem, self.n_nodes)
            return ("v", n, a, comp, g)
        a, rem = divmod(rem - self.nt * self.Mv, self.Mp)
        c, l = divmod(rem, self.C)
        return ("p", n, a, c, l)

    # ------------------------------------------------------------- operator
    def operator_row(self, x, idx):
        """(S x)[idx] as SpaceTimeLevel.apply evaluates it."""
        kind, n, a, u, v = self.decode(idx)
        if kind == "v":
            comp, g = u, v
            if self.is_boundary(g):
                return float(x[idx])
            y = 0.0
            for c, i in self.cells_of_node(g):
                Me, Ae, Be, cn = self.em(c)
                free = np.array([not self.is_boundary(h) for h in cn], dtype=float)
                for b in range(self.nt):
                    xv = x[[self.v_dof(n, b, comp, h) for h in cn]] * free
                    y += self.K[a, b] * (Me[i] @ xv) + self.Mtau[a, b] * (Ae[i] @ xv)
                    xp = x[[self.p_dof(n, b, c, l) for l in range(self.C)]]
                    y -= self.Mtau[a, b] * (Be[:, comp, i] @ xp)
                    if n > 0:
                        xq = x[[self.v_dof(n - 1, b, comp, h) for h in cn]] * free
                        y -= self.Ctau[a, b] * (Me[i] @ xq)
            return y
        c, l = u, v
        Me, Ae, Be, cn = self.em(c)
        free = np.array([not self.is_boundary(h) for h in cn], dtype=float)
        y = 0.0
        for b in range(self.nt):
            for comp in range(self.d):
                xv = x[[self.v_dof(n, b, comp, h) for h in cn]] * free
                y -= self.Mtau[a, b] * (Be[l, comp] @ xv)
        return y

    def operator_rows(self, x, rows):
        return np.array([self.operator_row(x, i) for i in rows])

    # ---------------------------------------------------------------- Vanka
    def local_matrix(self, T):
        """A_T of `vanka.local_matrices_factored` for cell T (the same for every
        subinterval), local order [a][comp][node] then [a][mode]."""
        d, nl, C, nt = self.d, self.nloc, self.C, self.nt
        cnT = self.cell_nodes(T)
        pos = {int(h): i for i, h in enumerate(cnT)}
        Ms = np.zeros((nl, nl))
        As = np.zeros((nl, nl))
        cc = self.mesh.cell_coords(T)
        for off in product((-1, 0, 1), repeat=d):
            nb = [cc[j] + off[j] for j in range(d)]
            if any(c < 0 or c >= self.n for c in nb):
                continue
            Me, Ae, _, cn = self.em(self.cell_index(nb))
            loc = [(i2, pos[int(h)]) for i2, h in enumerate(cn) if int(h) in pos]
            for i2, iT in loc:
                for j2, jT in loc:
                    Ms[iT, jT] += Me[i2, j2]
                    As[iT, jT] += Ae[i2, j2]
        fv1 = np.array([not self.is_boundary(h) for h in cnT])
        fv = np.tile(fv1, d)
        keep = np.outer(fv, fv).astype(float)
        Mloc = np.kron(np.eye(d), Ms) * keep
        Aloc = np.kron(np.eye(d), As) * keep
        Be = self.em(T)[2]                                    # (C, d, nl)
        Bloc = Be.reshape(C, d * nl) * fv[None, :].astype(float)
        Avv = np.kron(self.K, Mloc) + np.kron(self.Mtau, Aloc)
        Avv += np.kron(np.eye(nt), np.diag((~fv).astype(float)))
        Avp = -np.kron(self.Mtau, Bloc.T)
        Apv = -np.kron(self.Mtau, Bloc)
        App = np.zeros((nt * C, nt * C))
        return np.block([[Avv, Avp], [Apv, App]])

    def cell_dofs(self, T, n):
        """Global indices of the dofs of K_T x I_n in the local order."""
        cn = self.cell_nodes(T)
        idx = [self.v_dof(n, a, comp, h) for a in range(self.nt) for comp in range(self.d) for h in cn]
        idx += [self.p_dof(n, a, T, l) for a in range(self.nt) for l in range(self.C)]
        return np.array(idx)

    def local_solve(self, T, n, r):
        """A_T^{-1} R_T r (local matrices are cached per cell)."""
        if T not in self._lm:
            self._lm[T] = self.local_matrix(T)
        return np.linalg.solve(self._lm[T], r[self.cell_dofs(T, n)])

    def correction_entry(self, r, idx):
        """[sum_T R_T^T A_T^{-1} R_T r / valence][idx], zero on Dirichlet rows."""
        kind, n, a, u, v = self.decode(idx)
        if kind == "p":
            c, l = u, v
            z = self.local_solve(c, n, r)
            return z[self.nt * self.d * self.nloc + a * self.C + l]
        comp, g = u, v
        if self.is_boundary(g):
            return 0.0
        owners = self.cells_of_node(g)
        s = 0.0
        for c, i in owners:
            z = self.local_solve(c, n, r)
            s += z[(a * self.d + comp) * self.nloc + i]
        return s / len(owners)

    # ------------------------------------------------------ learned correction
    def learned_cell_tensor(self, r, T, n):
        """The 15 x 27 input tensor of space-time cell (T, n) as
        `learned.cell_tensors` builds it (3D Q2/P1 x DG(1) levels), unscaled,
        and the cell's Dirichlet mask."""
        if self.d != 3 or self.r != 1 or self.k != 1:
            raise ValueError("the learned correction acts on 3D Q2/P1 x DG(1) levels")
        cn = self.cell_nodes(T)
        mask = np.array([self.is_boundary(h) for h in cn], dtype=float)
        X = np.zeros((15, 27))
        for a in range(2):
            for comp in range(3):
                X[comp * 2 + a] = r[[self.v_dof(n, a, comp, h) for h in cn]] * (1.0 - mask)
            for l in range(4):
                X[6 + 4 * a + l] = r[self.p_dof(n, a, T, l)]
        X[14] = mask
        return X, mask

    def learned_cell_output(self, Ws, r, T, n):
        """s_T head(net(R_T r / s_T)) of one space-time cell: velocity (6, 27)
        and pressure (8,), with the network and head of `learned`."""
        from . import learned as ln
        if not hasattr(self, "_net"):
            self._net = {}
        if (T, n) not in self._net:
            X, mask = self.learned_cell_tensor(r, T, n)
            s = float(np.sqrt(np.sum(X[:6] ** 2) + np.sum(X[6:14, 0] ** 2)))
            if s == 0.0:
                self._net[(T, n)] = (np.zeros((6, 27)), np.zeros(8))
            else:
                Xn = X.copy()
                Xn[:14] /= s
                vel, pre = ln.head(ln.forward(Ws, Xn[None]), mask[None])
                self._net[(T, n)] = (vel[0] * s, pre[0] * s)
        return self._net[(T, n)]

    def learned_correction_entry(self, Ws, r, idx):
        """[sum_T R_T^T s_T head(net(R_T r / s_T))][idx], velocity divided by
        the valence, zero on Dirichlet rows (`learned.correction`).  The
        per-cell outputs are cached: one r per SampledLevel."""
        kind, n, a, u, v = self.decode(idx)
        if kind == "p":
            return self.learned_cell_output(Ws, r, u, n)[1][4 * a + v]
        comp, g = u, v
        if self.is_boundary(g):
            return 0.0
        owners = self.cells_of_node(g)
        s = sum(self.learned_cell_output(Ws, r, c, n)[0][comp * 2 + a, i] for c, i in owners)
        return s / len(owners)
