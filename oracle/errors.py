"""Space-time error norms and load vectors for manufactured solutions
(test infrastructure).

Load vector Eq. (DefFn): F_n^a,i = Q_n(<f, phi_n^a chi_i>) with the Radau rule
Eq. (GF) in time and a Gauss rule with r+4 points per direction in space
(reading G11).  Errors in L2(0,T; L2) and L2(0,T; H1-seminorm) use Gauss rules
with k+2 points in time and r+4 in space.
"""
import numpy as np

from . import elements as el
from .spacetime import SpaceTimeLevel


def load_vector(L: SpaceTimeLevel, f, t0=0.0):
    """f(x (np, d), t) -> (np, d).  Returns B = (F_n, 0) per Eq. (DefB)."""
    s = L.sp
    d, r = s.d, s.r
    x1, w1 = el.gauss_01(r + 4)
    xq, wq = el.tensor_points(x1, d), el.tensor_weights(w1, d)
    phi, _ = el.velocity_basis(d, r, xq)
    td = L.td
    b = np.zeros(L.ndofs)
    for c in range(s.mesh.n_cells):
        x, J = s.mesh.map(c, xq)
        jxw = np.linalg.det(J) * wq
        nodes = s.vdofs.cell_nodes[c]
        for n in range(L.N):
            for a in range(L.nt):
                # Radau rule: phi_n^a(t_n^mu) = delta, so only mu = a survives
                t = t0 + n * L.tau + 0.5 * L.tau * (td["t"][a] + 1.0)
                fa = f(x, t)
                for comp in range(d):
                    contrib = 0.5 * L.tau * td["w"][a] * (phi.T @ (jxw * fa[:, comp]))
                    idx = L.v_index(n, a).start + comp * s.n_nodes + nodes
                    np.add.at(b, idx, contrib)
    b[L.dirichlet_mask()] = 0.0
    return b


def errors(L: SpaceTimeLevel, X, v_exact, gradv_exact, p_exact, t0=0.0):
    """Returns (||v-v_h||_{L2L2}, ||grad(v-v_h)||_{L2L2}, ||p-p_h||_{L2L2}).
    v_exact(x, t) -> (np, d); gradv_exact(x, t) -> (np, d, d) [comp, dir];
    p_exact(x, t) -> (np,).  X should carry mean-zero pressure."""
    s = L.sp
    d, r = s.d, s.r
    x1, w1 = el.gauss_01(r + 4)
    xq, wq = el.tensor_points(x1, d), el.tensor_weights(w1, d)
    phi, dphi = el.velocity_basis(d, r, xq)
    psi = el.pressure_values(d, r, xq)
    tg, wg = el.gauss_m11(L.k + 2)
    Lt = el.lagrange_values(L.td["t"], tg)            # (nq_t, nt)
    ev = eg = ep = 0.0
    for c in range(s.mesh.n_cells):
        x, J = s.mesh.map(c, xq)
        det = np.linalg.det(J)
        JinvT = np.transpose(np.linalg.inv(J), (0, 2, 1))
        grad = np.einsum("pij,pnj->pni", JinvT, dphi)
        jxw = det * wq
        nodes = s.vdofs.cell_nodes[c]
        for n in range(L.N):
            U = np.array([[X[L.v_index(n, a).start + comp * s.n_nodes + nodes] for comp in range(d)]
                          for a in range(L.nt)])                           # (nt, d, nl)
            P = np.array([X[L.p_index(n, a).start + c * s.C: L.p_index(n, a).start + (c + 1) * s.C]
                          for a in range(L.nt)])                           # (nt, C)
            for it, tt in enumerate(tg):
                t = t0 + n * L.tau + 0.5 * L.tau * (tt + 1.0)
                wt = 0.5 * L.tau * wg[it]
                Ut = np.einsum("a,adn->dn", Lt[it], U)
                Pt = Lt[it] @ P
                vh = (phi @ Ut.T)                                          # (np, d)
                gh = np.einsum("pni,dn->pdi", grad, Ut)
                ph = psi @ Pt
                ev += wt * np.sum(jxw[:, None] * (vh - v_exact(x, t)) ** 2)
                eg += wt * np.sum(jxw[:, None, None] * (gh - gradv_exact(x, t)) ** 2)
                ep += wt * np.sum(jxw * (ph - p_exact(x, t)) ** 2)
    return np.sqrt(ev), np.sqrt(eg), np.sqrt(ep)
