"""Canonical grid-transfer operators (test infrastructure).

App. A: prolongation is the embedding of the coarse space into the fine one
(Eq. (DefPrRe), (DeftPrRe), (DefPrRer), (DefPrRek)), restriction its adjoint
(the transpose in coefficient space).  Space and time parts act on different
indices and are composed (Eq. (DefTlspr), (DefoTsl)).

Velocity: the coarse nodal function is evaluated at the fine nodes in
reference (undeformed) coordinates (reading G10); Dirichlet dofs are excluded
on both sides (the level spaces are subspaces of H^1_0).
Pressure: L2 projection in reference coordinates of the coarse cell
polynomial onto the fine cell's P_r basis (exact, it is an embedding).
Time: the coarse Lagrange basis at the fine Radau points, mapped into the
coarse subinterval.
"""
import numpy as np
import scipy.sparse as sp

from . import elements as el


def _node_ref_coord(g, n, q, gll):
    """Undeformed coordinate of global 1D Gauss-Lobatto node g (n cells, degree q)."""
    c = min(g // q, n - 1)
    i = g - c * q
    return (c + gll[i]) / n


def velocity_prolongation(sf, sc):
    """Scalar P_s (fine nodes x coarse nodes) between SpatialLevel objects."""
    d = sf.d
    qf, qc = sf.r + 1, sc.r + 1
    gf, gc = el.gauss_lobatto_01(qf + 1), el.gauss_lobatto_01(qc + 1)
    nnf, nnc = sf.vdofs.nn, sc.vdofs.nn
    Qc = qc + 1
    # every fine node m: its undeformed position X, the coarse cell holding
    # it and the coarse cell's Lagrange basis evaluated there (all vectorised
    # over m; the basis of a tensor-product element is the product of the 1D
    # factors)
    X1 = np.array([_node_ref_coord(g, sf.n, qf, gf) for g in range(nnf)])
    m = np.arange(sf.n_nodes)
    gidx = [(m // nnf ** j) % nnf for j in range(d)]
    X = [X1[g] for g in gidx]
    cc = [np.minimum(np.floor(X[j] * sc.n).astype(np.int64), sc.n - 1) for j in range(d)]
    L = [el.lagrange_values(gc, X[j] * sc.n - cc[j]) for j in range(d)]
    rows, cols, vals = [], [], []
    for i in range(Qc ** d):
        ii = [(i // Qc ** j) % Qc for j in range(d)]
        v = np.ones(sf.n_nodes)
        col = np.zeros(sf.n_nodes, dtype=np.int64)
        for j in range(d):
            v *= L[j][:, ii[j]]
            col += (cc[j] * qc + ii[j]) * nnc ** j
        nz = v != 0.0
        rows.append(m[nz]); cols.append(col[nz]); vals.append(v[nz])
    rows, cols, vals = map(np.concatenate, (rows, cols, vals))
    P = sp.csr_matrix((vals, (rows, cols)), shape=(sf.n_nodes, sc.n_nodes))
    P.sum_duplicates()
    Ff = sp.diags((~sf.vdofs.boundary).astype(float))
    Fc = sp.diags((~sc.vdofs.boundary).astype(float))
    P = (Ff @ P @ Fc).tocsr()
    P.eliminate_zeros()
    return P


def pressure_prolongation(sf, sc):
    """P_p (fine pressure dofs x coarse pressure dofs)."""
    d = sf.d
    ratio = sf.n // sc.n
    xq, wq = el.gauss_01(sf.r + 2)
    pts = el.tensor_points(xq, d)
    w = el.tensor_weights(wq, d)
    psi_f = el.pressure_values(d, sf.r, pts)
    Mf = np.einsum("p,pa,pb->ab", w, psi_f, psi_f)
    rows, cols, vals = [], [], []
    for cf in range(sf.mesh.n_cells):
        ccf = sf.mesh.cell_coords(cf)
        ccc = [x // ratio for x in ccf]
        off = [x % ratio for x in ccf]
        cpar = sum(ccc[j] * sc.n ** j for j in range(d))
        xi_c = (np.array(off)[None, :] + pts) / ratio
        psi_c = el.pressure_values(d, sc.r, xi_c)
        E = np.linalg.solve(Mf, np.einsum("p,pa,pb->ab", w, psi_f, psi_c))
        for a in range(sf.C):
            for b in range(sc.C):
                if abs(E[a, b]) > 1e-14:
                    rows.append(cf * sf.C + a)
                    cols.append(cpar * sc.C + b)
                    vals.append(E[a, b])
    return sp.csr_matrix((vals, (rows, cols)), shape=(sf.Mp, sc.Mp))


def time_prolongation(kf, Nf, kc, Nc):
    """P_t[(n_f, a), (n_c, b)] = phi^c_b(fine Radau point a of subinterval n_f,
    expressed in the reference coordinate of the coarse subinterval)."""
    tf = el.radau_right(kf)[0]
    tc = el.radau_right(kc)[0]
    ratio = Nf // Nc
    P = np.zeros((Nf * (kf + 1), Nc * (kc + 1)))
    for nf in range(Nf):
        nc = nf // ratio
        j = nf % ratio
        s = tf if ratio == 1 else (tf + 2 * j - 1) / 2.0
        P[nf * (kf + 1):(nf + 1) * (kf + 1), nc * (kc + 1):(nc + 1) * (kc + 1)] = el.lagrange_values(tc, s)
    return P


def prolongation(Lf, Lc):
    """Full space-time prolongation between SpaceTimeLevel objects (sparse)."""
    sf, sc = Lf.sp, Lc.sp
    Pv = sp.kron(sp.identity(sf.d), velocity_prolongation(sf, sc), format="coo")
    Pp = pressure_prolongation(sf, sc).tocoo()
    Pt = time_prolongation(Lf.k, Lf.N, Lc.k, Lc.N)
    rows, cols, vals = [], [], []
    for i in range(Pt.shape[0]):
        nf, a = divmod(i, Lf.nt)
        for j in range(Pt.shape[1]):
            t = Pt[i, j]
            if t == 0.0:
                continue
            nc, b = divmod(j, Lc.nt)
            rf, rc = Lf.v_index(nf, a).start, Lc.v_index(nc, b).start
            rows.append(Pv.row + rf); cols.append(Pv.col + rc); vals.append(t * Pv.data)
            rf, rc = Lf.p_index(nf, a).start, Lc.p_index(nc, b).start
            rows.append(Pp.row + rf); cols.append(Pp.col + rc); vals.append(t * Pp.data)
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(Lf.ndofs, Lc.ndofs))
    P.sum_duplicates()
    return P
