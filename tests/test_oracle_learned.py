"""Pins of the oracle's learned-correction network (reading G15): the
convolution against a brute-force loop, the gradients against central
differences in FP64, positive homogeneity, and the cell tensors against the
vector layout."""
import numpy as np
import pytest

from oracle import learned as ln
from oracle.assembly import SpatialLevel
from oracle.spacetime import SpaceTimeLevel


def test_conv_matches_brute_force():
    rng = np.random.default_rng(0)
    W = rng.standard_normal((4, 3, 27))
    X = rng.standard_normal((2, 3, 27))
    ref = np.zeros((2, 4, 27))
    for b in range(2):
        for co in range(4):
            for z in range(3):
                for y in range(3):
                    for x in range(3):
                        s = 0.0
                        for ci in range(3):
                            for dz in (-1, 0, 1):
                                for dy in (-1, 0, 1):
                                    for dx in (-1, 0, 1):
                                        xx, yy, zz = x + dx, y + dy, z + dz
                                        if 0 <= xx < 3 and 0 <= yy < 3 and 0 <= zz < 3:
                                            o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
                                            s += W[co, ci, o] * X[b, ci, xx + 3 * yy + 9 * zz]
                        ref[b, co, x + 3 * y + 9 * z] = s
    assert np.allclose(ln.conv(W, X), ref, atol=1e-13)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    Ws = ln.init_weights(2)
    X = rng.standard_normal((3, 15, 27))
    mask = (rng.random((3, 27)) < 0.2).astype(float)
    X[:, 14, :] = mask
    tv = rng.standard_normal((3, 6, 27))
    tp = rng.standard_normal((3, 8))
    loss, grads = ln.loss_and_grads(Ws, X, mask, tv, tp)
    h = 1e-6
    for layer in range(3):
        for _ in range(12):
            idx = tuple(rng.integers(0, s) for s in ln.SHAPES[layer])
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[layer][idx] += h
            Wm[layer][idx] -= h
            fd = (ln.loss_and_grads(Wp, X, mask, tv, tp)[0] - ln.loss_and_grads(Wm, X, mask, tv, tp)[0]) / (2 * h)
            g = grads[layer][idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)) + 1e-9, (layer, idx, fd, g)


def test_network_is_positively_homogeneous():
    rng = np.random.default_rng(3)
    Ws = ln.init_weights(4)
    X = rng.standard_normal((2, 15, 27))
    assert np.allclose(ln.forward(Ws, 3.7 * X), 3.7 * ln.forward(Ws, X), rtol=1e-12, atol=1e-12)


def test_cell_tensors_and_correction_properties():
    s = SpatialLevel(3, 2, 1, 0.03)
    L = SpaceTimeLevel(s, 1, 2, 0.05)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(L.ndofs)
    X, mask = ln.cell_tensors(L, r)
    assert X.shape == (L.N * 8, 15, 27)
    # every velocity residual entry of a free node appears in some cell tensor
    c = 3  # cell (1,1,0) in subinterval 0
    nodes = s.vdofs.cell_nodes[c]
    for comp in range(3):
        for a in range(2):
            vals = r[L.v_index(0, a).start + comp * s.n_nodes + nodes] * (1 - mask[c])
            assert np.allclose(X[c, comp * 2 + a], vals)
    Ws = ln.init_weights(6)
    u = ln.correction(L, Ws, r)
    assert np.all(u[L.dirichlet_mask()] == 0)
    assert np.allclose(ln.correction(L, Ws, 2.5 * r), 2.5 * u, rtol=1e-12, atol=1e-14)
    assert np.all(ln.correction(L, Ws, np.zeros(L.ndofs)) == 0)


def test_correction_through_next_level_properties():
    """P net(P^T r): zero for r = 0, positively homogeneous, zero on the
    fine level's Dirichlet rows, and equal to the plain correction when P is
    the identity (the same level)."""
    from oracle import learned as ln
    from oracle.mg import Multigrid
    import scipy.sparse as sp
    mg = Multigrid(3, 2, 2, 1, 2, 0.05, nu=1.0, amp=0.03, n_coarse=1, k_min=1, omega=0.8)
    Lf, Lc, P = mg.levels[0], mg.levels[1], mg.P[0]
    assert (Lc.sp.r, Lc.k) == (1, 1)
    Ws = ln.init_weights(4)
    rng = np.random.default_rng(8)
    r = rng.standard_normal(Lf.ndofs)
    r[Lf.dirichlet_mask()] = 0.0
    assert np.all(ln.correction_through(Lc, P, Ws, 0 * r) == 0.0)
    u = ln.correction_through(Lc, P, Ws, r)
    assert np.allclose(ln.correction_through(Lc, P, Ws, 3.0 * r), 3.0 * u, rtol=1e-12, atol=0)
    assert np.all(u[Lf.dirichlet_mask()] == 0.0)
    rc = rng.standard_normal(Lc.ndofs)
    I = sp.identity(Lc.ndofs, format="csr")
    assert np.allclose(ln.correction_through(Lc, I, Ws, rc), ln.correction(Lc, Ws, rc), rtol=0, atol=1e-14)
