"""Train the learned correction for the benchmark workloads (run on a GPU).

Configuration C4 (training): 3D Stokes, Q2/P1disc x DG(1), 16^3 deformed hex
mesh, slab of 2 subintervals, tau = 0.05, nu = 1; 1000 random forcings
(seeds 1000..1999), two (residual, error) pairs each; Adam, lr 1e-3,
batch 4096 space-time cells, 20 epochs.  Writes the FP32 weights (ABI
order) as a .npy file.

    python -m paper_2502_09159_amd.train_c4 OUT.npy [--forcings 1000] [--epochs 20]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--forcings", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    args = ap.parse_args()
    from paper_2502_09159_amd import learned, stmg
    from stmg_inputs import random_rhs
    cfg = dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=1, k=1, n_sub=2, deform_amp=0.03, tau=0.05, nu=1.0,
               omega=0.8)
    S = stmg.Solver(**cfg)
    t0 = time.time()
    forcings = (random_rhs(3, 16, 1, 1, 2, s) for s in range(1000, 1000 + args.forcings))
    rp, ep = learned.make_pairs(S, forcings)
    print(f"[train] {rp.shape[0]} pairs in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    w, hist = learned.train(S, rp, ep, seed=1, epochs=args.epochs, batch=args.batch, lr=args.lr)
    steps = len(hist) // args.epochs
    for e in range(args.epochs):
        print(f"[train] epoch {e}: mean loss {hist[e * steps:(e + 1) * steps].mean():.4f}", flush=True)
    print(f"[train] {len(hist)} steps in {time.time() - t0:.1f} s", flush=True)
    np.save(args.out, w.astype(np.float32), allow_pickle=False)
    S.close()


if __name__ == "__main__":
    main()
