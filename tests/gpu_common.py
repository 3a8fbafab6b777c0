"""Shared set-up of the GPU parity tests: the HIP library and the oracle are
built from the same parameters and fed the same seeded inputs."""
import functools

import numpy as np
import pytest
import torch

from stmg_inputs import FourierViscosity, random_rhs

CONFIGS = {
    # C1: 2D Q2/P1 x DG(1), 4x4 cells, 2 subintervals
    "c1": dict(dim=2, n_cells_1d=4, n_coarse_1d=1, r=1, k=1, n_sub=2, deform_amp=0.0, k_min=1),
    # the C2 element (Q3/P2 x DG(2), k -> 0) on a 4^3 deformed mesh
    "c2_small": dict(dim=3, n_cells_1d=4, n_coarse_1d=2, r=2, k=2, n_sub=2, deform_amp=0.03, k_min=0),
    # Q2/P1 x DG(1) on 8^3, 4 subintervals: two temporal h-steps
    "r1k1_n8": dict(dim=3, n_cells_1d=8, n_coarse_1d=2, r=1, k=1, n_sub=4, deform_amp=0.03, k_min=1),
    # the C3/C5 element (Q3/P2 x DG(1)) on 4^3, 4 subintervals, variable viscosity
    "c5_small": dict(dim=3, n_cells_1d=4, n_coarse_1d=2, r=2, k=1, n_sub=4, deform_amp=0.03, k_min=1, nu_seed=5),
    # the same with temporal h-coarsening at the coarse end (N 4 -> 2 -> 1)
    "r1k1_n8_th": dict(dim=3, n_cells_1d=8, n_coarse_1d=2, r=1, k=1, n_sub=4, deform_amp=0.03, k_min=1,
                       time_h_coarsening=1),
    # the C2 element with r and k halved together on the fine mesh (k -> 0)
    "c2_small_top": dict(dim=3, n_cells_1d=4, n_coarse_1d=2, r=2, k=2, n_sub=2, deform_amp=0.03, k_min=0,
                         placement=1),
    # 2D Q3/P2 x DG(2) on 8x8
    "2d_r2k2": dict(dim=2, n_cells_1d=8, n_coarse_1d=1, r=2, k=2, n_sub=2, deform_amp=0.03, k_min=1),
    # ragged sizes: 6^3 cells (216: no multiple of a block or tile), a 3^3 coarse mesh, one subinterval
    "ragged_n6_N1": dict(dim=3, n_cells_1d=6, n_coarse_1d=3, r=1, k=1, n_sub=1, deform_amp=0.03, k_min=1),
    # DG(0) on the finest level (one temporal dof), Q3/P2 in space, 6^3 -> 3^3
    "k0_n6": dict(dim=3, n_cells_1d=6, n_coarse_1d=3, r=2, k=0, n_sub=2, deform_amp=0.03, k_min=0),
}
TAU = 0.05
OMEGA = 0.8


def nu_field(cfg):
    return FourierViscosity(cfg["nu_seed"]) if "nu_seed" in cfg else None


def gpu_params(cfg, **over):
    p = {k: v for k, v in cfg.items() if k != "nu_seed"}
    p.update(tau=TAU, omega=OMEGA, nu=1.0)
    p.update(over)
    return p


def make_solver(cfg, **over):
    from paper_2502_09159_amd import stmg
    nf = nu_field(cfg)
    return stmg.Solver(nu_fn=nf, **gpu_params(cfg, **over))


@functools.lru_cache(maxsize=None)
def oracle_mg(name, smoother="exact"):
    from oracle.mg import Multigrid
    cfg = CONFIGS[name]
    nf = nu_field(cfg)
    return Multigrid(cfg["dim"], cfg["n_cells_1d"], cfg["r"], cfg["k"], cfg["n_sub"], TAU,
                     nu=nf if nf is not None else 1.0, amp=cfg["deform_amp"], n_coarse=cfg["n_coarse_1d"],
                     k_min=cfg["k_min"], omega=OMEGA, time_h=cfg.get("time_h_coarsening", 0) == 1,
                     placement="top" if cfg.get("placement", 0) == 1 else "paper", smoother=smoother)


def rhs(cfg, seed):
    return random_rhs(cfg["dim"], cfg["n_cells_1d"], cfg["r"], cfg["k"], cfg["n_sub"], seed)


def dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
