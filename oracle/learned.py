"""Learned correction after a Vanka sweep (test infrastructure).

The paper has no learned component; this follows the network of reading G15:
per space-time cell T = K x I_n of a 3D level with the Q2/P1 x DG(1) element
(r = 1, k = 1; other levels reach it through the next level, see
`correction_through`), the cell residual becomes a 15-channel tensor on the 3x3x3
Gauss-Lobatto nodes:
  channels 0..5  : velocity residual, channel comp*2 + a (component, temporal dof)
  channels 6..13 : pressure residual of mode l at temporal dof a, channel 6 + 4a + l,
                   broadcast to all 27 nodes
  channel 14     : 1 on Dirichlet nodes
scaled by 1/s_T, s_T = ||R_T r||_2 (velocity and pressure entries); a cell
with s_T = 0 gets no correction.
Network: conv(15->32) -> ReLU -> conv(32->32) -> ReLU -> conv(32->14), 3x3x3
kernels, zero padding, no biases (positively homogeneous).  Output: channels
0..5 are the velocity correction at the nodes (zero on Dirichlet nodes),
channels 6..13 averaged over the 27 nodes are the pressure correction; both
multiplied by s_T.  The global correction is sum_T R_T^T (valence-weighted
on velocity nodes), the same patch sum as Eq. (vanka0).

Weights: W[layer] of shape (C_out, C_in, 27), offset o = (dx+1) + 3(dy+1) + 9(dz+1).
"""
import numpy as np

from .spacetime import SpaceTimeLevel
from .vanka import cell_dofs

C_IN, C_HID, C_OUT = 15, 32, 14
SHAPES = [(C_HID, C_IN, 27), (C_HID, C_HID, 27), (C_OUT, C_HID, 27)]


def n_params():
    return sum(int(np.prod(s)) for s in SHAPES)


def unpack(flat):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def init_weights(seed):
    """He-normal initialisation (fan-in = C_in * 27)."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) * np.sqrt(2.0 / (s[1] * 27)) for s in SHAPES]


def _shift_table():
    """nbr[o, p] = neighbour position of p at offset o, or -1 (zero padding)."""
    nbr = np.full((27, 27), -1)
    for o in range(27):
        dx, dy, dz = o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1
        for p in range(27):
            x, y, z = p % 3 + dx, (p // 3) % 3 + dy, p // 9 + dz
            if 0 <= x < 3 and 0 <= y < 3 and 0 <= z < 3:
                nbr[o, p] = x + 3 * y + 9 * z
    return nbr


NBR = _shift_table()


def conv(W, X):
    """out[b, co, p] = sum_ci sum_o W[co, ci, o] X[b, ci, nbr(o, p)]."""
    B, Ci, _ = X.shape
    Xp = np.concatenate([X, np.zeros((B, Ci, 1))], axis=2)        # index -1 -> zero
    G = Xp[:, :, NBR]                                              # (B, Ci, 27 offsets, 27 positions)
    return np.einsum("uio,biop->bup", W, G)


def conv_backward(W, X, dY):
    """Gradients of sum(dY * conv(W, X)) wrt W and X."""
    B, Ci, _ = X.shape
    Xp = np.concatenate([X, np.zeros((B, Ci, 1))], axis=2)
    G = Xp[:, :, NBR]
    dW = np.einsum("bup,biop->uio", dY, G)
    dG = np.einsum("uio,bup->biop", W, dY)
    dXp = np.zeros((B, Ci, 28))
    for o in range(27):
        np.add.at(dXp, (slice(None), slice(None), NBR[o]), dG[:, :, o, :])
    return dW, dXp[:, :, :27]


def forward(Ws, X, keep=False):
    """Raw network output (B, 14, 27) for inputs X (B, 15, 27)."""
    a1 = conv(Ws[0], X)
    h1 = np.maximum(a1, 0.0)
    a2 = conv(Ws[1], h1)
    h2 = np.maximum(a2, 0.0)
    y = conv(Ws[2], h2)
    if keep:
        return y, (X, a1, h1, a2, h2)
    return y


def head(y, mask):
    """Velocity (B, 6, 27) masked on Dirichlet nodes, pressure (B, 8) averages."""
    vel = y[:, :6, :] * (1.0 - mask[:, None, :])
    pre = y[:, 6:, :].mean(axis=2)
    return vel, pre


def loss_and_grads(Ws, X, mask, tv, tp):
    """Loss sum |head(net(X)) - t|^2 / sum |t|^2 over the batch, and dL/dW."""
    y, (X0, a1, h1, a2, h2) = forward(Ws, X, keep=True)
    vel, pre = head(y, mask)
    den = np.sum(tv ** 2) + np.sum(tp ** 2)
    loss = (np.sum((vel - tv) ** 2) + np.sum((pre - tp) ** 2)) / den
    dy = np.zeros_like(y)
    dy[:, :6, :] = 2.0 * (vel - tv) * (1.0 - mask[:, None, :]) / den
    dy[:, 6:, :] = (2.0 * (pre - tp) / den / 27.0)[:, :, None]
    dW3, dh2 = conv_backward(Ws[2], h2, dy)
    da2 = dh2 * (a2 > 0)
    dW2, dh1 = conv_backward(Ws[1], h1, da2)
    da1 = dh1 * (a1 > 0)
    dW1, _ = conv_backward(Ws[0], X0, da1)
    return loss, [dW1, dW2, dW3]


# ------------------------------------------------------------ cell tensors
def _check_level(L: SpaceTimeLevel):
    if L.sp.d != 3 or L.sp.r != 1 or L.k != 1:
        raise ValueError("the learned correction acts on 3D Q2/P1 x DG(1) levels")


def cell_tensors(L: SpaceTimeLevel, v):
    """Per space-time cell (n major, then cell), the 15 x 27 tensor of the
    vector v restricted to the cell, unscaled, and the Dirichlet mask."""
    _check_level(L)
    s = L.sp
    nc = s.mesh.n_cells
    X = np.zeros((L.N * nc, 15, 27))
    bmask = s.vdofs.boundary[s.vdofs.cell_nodes].astype(float)    # (nc, 27)
    for n in range(L.N):
        idx = cell_dofs(L, n)          # [a][comp][node] (2*3*27) then [a][mode] (2*4)
        vals = v[idx]
        blk = slice(n * nc, (n + 1) * nc)
        for a in range(2):
            for comp in range(3):
                o = (a * 3 + comp) * 27
                X[blk, comp * 2 + a, :] = vals[:, o:o + 27] * (1.0 - bmask)
            for l in range(4):
                X[blk, 6 + 4 * a + l, :] = vals[:, 162 + a * 4 + l][:, None]
        X[blk, 14, :] = bmask
    mask = np.tile(bmask, (L.N, 1))
    return X, mask


def scales(X):
    """s_T over the velocity (channels 0..5) and pressure entries of each cell."""
    return np.sqrt(np.sum(X[:, :6, :] ** 2, axis=(1, 2)) + np.sum(X[:, 6:14, 0] ** 2, axis=1))


def net_inputs(L, r):
    X, mask = cell_tensors(L, r)
    s = scales(X)
    Xn = X.copy()
    inv = np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)
    Xn[:, :14, :] *= inv[:, None, None]
    return Xn, mask, s


def correction(L: SpaceTimeLevel, Ws, r):
    """sum_T R_T^T s_T head(net(R_T r / s_T)), velocity weighted by 1/valence."""
    Xn, mask, s = net_inputs(L, r)
    vel, pre = head(forward(Ws, Xn), mask)
    vel *= s[:, None, None]
    pre *= s[:, None]
    sl = L.sp
    nc = sl.mesh.n_cells
    u = np.zeros(L.ndofs)
    for n in range(L.N):
        idx = cell_dofs(L, n)
        blk = slice(n * nc, (n + 1) * nc)
        loc = np.zeros((nc, idx.shape[1]))
        for a in range(2):
            for comp in range(3):
                o = (a * 3 + comp) * 27
                loc[:, o:o + 27] = vel[blk, comp * 2 + a, :]
            for l in range(4):
                loc[:, 162 + a * 4 + l] = pre[blk, 4 * a + l]
        u += np.bincount(idx.ravel(), weights=loc.ravel(), minlength=L.ndofs)
    val = np.zeros(L.ndofs)
    for n in range(L.N):
        np.add.at(val, cell_dofs(L, n).ravel(), 1.0)
    u /= val
    u[L.dirichlet_mask()] = 0.0
    return u


def correction_through(Lc, P, Ws, r):
    """Reading G15 B on a level whose element is not Q2/P1 x DG(1) but whose
    next coarser level Lc has it on the same mesh: the residual restricted
    with the level transfer (App. A), the network correction on Lc, and that
    correction prolongated back: P correction(Lc, P^T r)."""
    return P @ correction(Lc, Ws, P.T @ r)


def targets(L, e, s):
    """Normalised targets of the error e: velocity (B, 6, 27), pressure (B, 8)."""
    E, _ = cell_tensors(L, e)
    inv = np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)
    return E[:, :6, :] * inv[:, None, None], E[:, 6:14, 0] * inv[:, None]
