"""Training driver of the learned correction: (residual, error) pairs from
random forcings, then Adam on the GPU through the library's own kernels.

Pairs: for each forcing b (velocity entries U[-1,1] on interior nodes,
pressure rows 0), x* from FGMRES to 1e-12, then the library records the
residual and the error after the presmoothing and after the postsmoothing
sweep of the first V-cycle on the finest level (two pairs per forcing).
"""
import numpy as np
import torch

from . import stmg


def make_pairs(solver, forcings, rtol=1e-12):
    """forcings: iterable of host arrays b; returns float32 device tensors
    r_pairs, e_pairs of shape (2 len(forcings), n_dofs)."""
    rs, es = [], []
    for b in forcings:
        bd = torch.tensor(np.asarray(b, dtype=np.float64), device="cuda")
        xs = torch.empty_like(bd)
        solver.solve(bd, xs, rtol=rtol, max_it=200)
        r, e = solver.learned_record(bd, xs)
        rs.append(r.float())
        es.append(e.float())
    return torch.cat(rs).contiguous(), torch.cat(es).contiguous()


def he_init(seed):
    """He-normal weights in the ABI order (layer, c_out, c_in, offset)."""
    rng = np.random.default_rng(seed)
    parts = []
    for cout, cin in ((32, 15), (32, 32), (14, 32)):
        parts.append(rng.standard_normal(cout * cin * 27) * np.sqrt(2.0 / (cin * 27)))
    return np.concatenate(parts).astype(np.float32)


def train(solver, r_pairs, e_pairs, seed=0, epochs=20, batch=4096, lr=1e-3, init_seed=0):
    solver.learned_load(he_init(init_seed))
    hist = solver.learned_train(r_pairs, e_pairs, seed=seed, epochs=epochs, batch=batch, lr=lr)
    return solver.learned_weights(), hist
