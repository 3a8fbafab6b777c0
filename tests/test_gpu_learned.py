"""GPU checks of the learned correction (BF16 on the matrix cores, FP32
accumulation) against the FP64 oracle network, the switch-off rule, and what
a trained network gains over plain multigrid."""
import numpy as np
import pytest
import torch

from gpu_common import announce, dev, host
from stmg_inputs import random_rhs

pytestmark = pytest.mark.gpu

CFG = dict(dim=3, n_cells_1d=4, n_coarse_1d=2, r=1, k=1, n_sub=2, deform_amp=0.03, k_min=1, tau=0.05, nu=1.0,
           omega=0.8)


@pytest.fixture(scope="module")
def small():
    from oracle.assembly import SpatialLevel
    from oracle.spacetime import SpaceTimeLevel
    from paper_2502_09159_amd import stmg
    g = stmg.Solver(**CFG)
    L = SpaceTimeLevel(SpatialLevel(3, 4, 1, 0.03, 1.0), 1, 2, 0.05)
    yield g, L
    g.close()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_correction_matches_oracle(small):
    from oracle import learned as ln
    from paper_2502_09159_amd.learned import he_init
    g, L = small
    w = he_init(3)
    g.learned_load(w)
    rng = np.random.default_rng(31)
    r = rng.standard_normal(L.ndofs)
    u = host(g.learned_correction(dev(r)))
    ref = ln.correction(L, ln.unpack(w.astype(np.float64)), r)
    err = rel_l2(u, ref)
    announce(f"learned correction vs oracle: rel L2 {err:.2e}")
    assert err < 2e-2


def test_correction_through_the_next_level_matches_oracle():
    """Reading G15 B: on the Q3/P2 x DG(1) finest level (4^3, N = 2) the
    correction is P net(P^T r) through the Q2/P1 x DG(1) level on the same
    mesh."""
    from oracle import learned as ln
    from oracle.mg import Multigrid
    from paper_2502_09159_amd import stmg
    from paper_2502_09159_amd.learned import he_init
    cfg = dict(dim=3, n_cells_1d=4, n_coarse_1d=2, r=2, k=1, n_sub=2, deform_amp=0.03, k_min=1, tau=0.05, nu=1.0,
               omega=0.8)
    g = stmg.Solver(**cfg)
    try:
        mg = Multigrid(3, 4, 2, 1, 2, 0.05, nu=1.0, amp=0.03, n_coarse=2, k_min=1, omega=0.8)
        Lf, Lc = mg.levels[0], mg.levels[1]
        assert (Lc.sp.r, Lc.k, Lc.sp.n) == (1, 1, 4)
        w = he_init(11)
        g.learned_load(w)
        rng = np.random.default_rng(33)
        r = rng.standard_normal(Lf.ndofs)
        r[Lf.dirichlet_mask()] = 0.0
        u = host(g.learned_correction(dev(r), level=0))
        ref = ln.correction_through(Lc, mg.P[0], ln.unpack(w.astype(np.float64)), r)
        err = rel_l2(u, ref)
        announce(f"learned correction through the next level vs oracle: rel L2 {err:.2e}")
        assert err < 2e-2
    finally:
        g.close()


def test_correction_in_chunks():
    """The inference loop over chunks of space-time cells (8^3, N = 4: 2,048
    cells in 32 chunks of 64) gives the same correction as one chunk, bit for
    bit (every cell's output is independent of the chunking and the
    valence-weighted scatter sums in a fixed order), and matches the oracle."""
    from oracle import learned as ln
    from oracle.assembly import SpatialLevel
    from oracle.spacetime import SpaceTimeLevel
    from paper_2502_09159_amd import stmg
    from paper_2502_09159_amd.learned import he_init
    cfg = dict(CFG, n_cells_1d=8, n_sub=4)
    g = stmg.Solver(**cfg)
    try:
        L = SpaceTimeLevel(SpatialLevel(3, 8, 1, 0.03, 1.0), 1, 4, 0.05)
        w = he_init(7)
        g.learned_load(w)
        r = np.random.default_rng(35).standard_normal(L.ndofs)
        u1 = host(g.learned_correction(dev(r)))
        g.set_option(stmg.OPT_NET_CHUNK, 64)
        u2 = host(g.learned_correction(dev(r)))
        assert np.array_equal(u1, u2)
        err = rel_l2(u2, ln.correction(L, ln.unpack(w.astype(np.float64)), r))
        announce(f"learned correction in 32 chunks vs oracle: rel L2 {err:.2e}")
        assert err < 2e-2
    finally:
        g.close()


def test_gradient_matches_oracle(small):
    from oracle import learned as ln
    from paper_2502_09159_amd.learned import he_init
    g, L = small
    w = he_init(5)
    g.learned_load(w)
    rng = np.random.default_rng(32)
    r = rng.standard_normal(L.ndofs)
    e = rng.standard_normal(L.ndofs)
    grad, loss = g.learned_gradient(dev(r), dev(e))
    Ws = ln.unpack(w.astype(np.float64))
    Xn, mask, s = ln.net_inputs(L, r)
    tv, tp = ln.targets(L, e, s)
    loss_ref, grads = ln.loss_and_grads(Ws, Xn, mask, tv, tp)
    assert abs(loss - loss_ref) < 2e-2 * loss_ref
    off = 0
    for layer, gr in enumerate(grads):
        n = gr.size
        err = rel_l2(grad[off:off + n].astype(np.float64), gr.ravel())
        announce(f"layer {layer + 1} weight gradient vs oracle: rel L2 {err:.2e}")
        assert err < 2e-2
        off += n


def test_train_in_one_call():
    """stmg_learned_train (the call of the boundary that takes n_pairs, seed,
    epochs and lr): forcings generated and solved inside the library, pairs
    recorded, Adam; the held-out loss falls below that of the starting
    weights, and with no weights loaded it starts from its own He-normal
    initialisation."""
    from paper_2502_09159_amd import learned, stmg
    g = stmg.Solver(**CFG)
    try:
        w0 = learned.he_init(0)
        g.learned_load(w0)
        test_b = [random_rhs(3, 4, 1, 1, 2, s) for s in range(2000, 2004)]
        rt, et = learned.make_pairs(g, test_b)

        def held_out():
            return np.mean([g.learned_gradient(rt[i].double().contiguous(), et[i].double().contiguous())[1]
                            for i in range(rt.shape[0])])
        loss0 = held_out()
        w = g.learned_train_seeded(n_pairs=32, seed=5, epochs=4, lr=1e-3)
        loss1 = held_out()
        announce(f"one-call training: held-out loss {loss0:.3f} -> {loss1:.3f}")
        assert np.all(np.isfinite(w)) and not np.array_equal(w, w0)
        assert np.array_equal(w, g.learned_weights())
        assert loss1 < loss0
    finally:
        g.close()
    g2 = stmg.Solver(**CFG)
    try:
        w2 = g2.learned_train_seeded(n_pairs=4, seed=6, epochs=1, lr=1e-3)
        assert np.all(np.isfinite(w2)) and np.abs(w2).max() > 0
    finally:
        g2.close()


@pytest.mark.parametrize("kind", ["nan", "zero"])
def test_switch_off_on_a_bad_network(kind):
    """A network whose correction cannot reduce the residual (non-finite or
    zero output) is switched off at its first application; the solve then
    matches plain multigrid exactly."""
    from paper_2502_09159_amd import stmg
    from paper_2502_09159_amd.learned import he_init
    cfg = dict(CFG, n_cells_1d=8)
    g = stmg.Solver(**cfg)
    try:
        b = dev(random_rhs(3, 8, 1, 1, 2, 41))
        x0 = torch.empty_like(b)
        plain = g.solve(b, x0, rtol=1e-8)
        w = he_init(7)
        w[:] = np.nan if kind == "nan" else 0.0
        g.learned_load(w)
        g.learned_enable(True)
        x1 = torch.empty_like(b)
        info = g.solve(b, x1, rtol=1e-8)
        g.learned_enable(False)
        announce(f"{kind} net: disabled={info['learned_disabled']} it={info['iterations']} "
                 f"plain={plain['iterations']}")
        assert info["learned_disabled"] == 1
        assert info["iterations"] == plain["iterations"]
        assert (torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0)).item() < 1e-12
    finally:
        g.close()


def test_training_and_gain():
    """Train on pairs from random forcings (8^3, Q2/P1 x DG(1), 2 subintervals),
    check the loss falls below the untrained network's on held-out pairs, and
    report iterations and time to 1e-8 with the trained net, an untrained
    net and none (the gain is measured, not assumed)."""
    from paper_2502_09159_amd import learned, stmg
    cfg = dict(CFG, n_cells_1d=8)
    g = stmg.Solver(**cfg)
    try:
        train_b = [random_rhs(3, 8, 1, 1, 2, s) for s in range(1000, 1040)]
        test_b = [random_rhs(3, 8, 1, 1, 2, s) for s in range(2000, 2004)]
        rp, ep = learned.make_pairs(g, train_b)
        rt, et = learned.make_pairs(g, test_b)
        w0 = learned.he_init(0)
        g.learned_load(w0)
        loss0 = np.mean([g.learned_gradient(rt[i].double().contiguous(), et[i].double().contiguous())[1]
                         for i in range(rt.shape[0])])
        w, hist = learned.train(g, rp, ep, seed=1, epochs=6, batch=512, lr=1e-3)
        loss1 = np.mean([g.learned_gradient(rt[i].double().contiguous(), et[i].double().contiguous())[1]
                         for i in range(rt.shape[0])])
        announce(f"held-out loss untrained {loss0:.3f} -> trained {loss1:.3f}; train loss first {hist[:20].mean():.3f} "
                 f"last {hist[-20:].mean():.3f}")
        assert np.all(np.isfinite(hist))
        assert loss1 < loss0
        b = dev(random_rhs(3, 8, 1, 1, 2, 4))
        res = {}
        for name, wts in (("none", None), ("untrained", w0), ("trained", w)):
            x = torch.empty_like(b)
            if wts is None:
                g.learned_enable(False)
            else:
                g.learned_load(wts)
                g.learned_enable(True)
            info = g.solve(b, x, rtol=1e-8)
            res[name] = (info["iterations"], info["t_solve_s"], info["learned_disabled"], info["rel_residual"])
            assert info["rel_residual"] <= 1e-8
        announce("gain (iterations, seconds, disabled): " + str(res))
        g.learned_enable(False)
        # the learned solution, with the FP32 V-cycle, against plain FP64
        # multigrid: both solved to 1e-10, within 1e-8 of each other
        x64 = torch.empty_like(b)
        g.solve(b, x64, rtol=1e-10)
        g32 = stmg.Solver(precision=stmg.MIXED_FP32, **cfg)
        try:
            g32.learned_load(w)
            g32.learned_enable(True)
            x32 = torch.empty_like(b)
            info = g32.solve(b, x32, rtol=1e-10)
            err = (torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)).item()
            announce(f"FP32 + learned vs FP64: {info['iterations']} it, disabled={info['learned_disabled']}, "
                     f"rel error {err:.2e}")
            assert err < 1e-8
        finally:
            g32.close()
    finally:
        g.close()
