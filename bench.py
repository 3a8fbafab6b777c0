"""Benchmark: space-time DoF/s to a 1e-8 relative residual, FGMRES with the
hp space-time multigrid V-cycle, one MI355X: the FP32 V-cycle with the
learned correction (value) against plain FP64 multigrid (reported beside it).

One step = one complete solve of the slab system (FGMRES to ||b - S x|| <=
1e-8 ||b||, explicitly rechecked) with b resident in HBM and the set-up done.
Prints one JSON line (rank 0).  Only N = 1 GPU is supported.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "space-time DoF/s to 1e-8 rel. residual: plain FP64 MG vs FP32+learned MG"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # 3D Stokes, Q3/P2disc x DG(2), 16^3 deformed hexes, slab of 4 subintervals, hp MG k -> 0
    "c2": dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=2, k=2, n_sub=4, deform_amp=0.03, k_min=2, seed=2,
               label="3D Stokes Q3/P2disc x DG(2), 16^3 deformed hex mesh, slab of 4 subintervals, nu=1"),
    # 3D Stokes, Q3/P2disc x DG(1), 32^3 deformed, 4 subintervals
    "c3": dict(dim=3, n_cells_1d=32, n_coarse_1d=2, r=2, k=1, n_sub=4, deform_amp=0.03, k_min=1, seed=3,
               label="3D Stokes Q3/P2disc x DG(1), 32^3 deformed hex mesh, slab of 4 subintervals, nu=1"),
    # 3D Stokes, Q3/P2disc x DG(1), 32^3 deformed, 8 subintervals, nu(x) = exp(0.5 g(x))
    "c5": dict(dim=3, n_cells_1d=32, n_coarse_1d=2, r=2, k=1, n_sub=8, deform_amp=0.03, k_min=1, seed=5,
               nu_seed=5, label="3D Stokes Q3/P2disc x DG(1), 32^3 deformed hex mesh, slab of 8 subintervals, "
                                "nu(x)=exp(0.5 g(x))"),
}
TAU, OMEGA = 0.05, 0.8
WEIGHTS = os.path.join(ROOT, "paper_2502_09159_amd", "weights", "net_c4.npy")


def solver_params(w, precision):
    keys = ("dim", "n_cells_1d", "n_coarse_1d", "r", "k", "n_sub", "deform_amp", "k_min")
    p = {k: w[k] for k in keys}
    p.update(tau=TAU, nu=1.0, omega=OMEGA, precision=precision)
    return p


def vanka_bytes(w, ncells_fine, elem_bytes):
    """Algorithmic bytes of one Vanka correction on the finest level: the
    stored factors of every cell (A_s^{-1}: m^2, B: C d nl, F: d m P, H^{-1}: P^2)
    plus one read of r and one read+write of x."""
    from math import comb
    d, r, k, N = w["dim"], w["r"], w["k"], w["n_sub"]
    nl = (r + 2) ** d
    nt = k + 1
    C = comb(r + d, d)
    m, P = nt * nl, nt * C
    factors = m * m + C * d * nl + d * m * P + P * P
    n = w["n_cells_1d"]
    ndofs = N * nt * (d * (n * (r + 1) + 1) ** d + n ** d * C)
    return (ncells_fine * factors + 3 * ndofs) * elem_bytes


def cpu_baseline(w):
    """The oracle as it stands, timed on this host: FGMRES + V-cycle to 1e-8 on
    the same discretisation and slab on a 4^3 mesh (the oracle's set-up of
    the full mesh alone takes minutes)."""
    from oracle.fgmres import fgmres
    from oracle.mg import Multigrid
    from stmg_inputs import FourierViscosity, random_rhs
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    n = 4
    nu = FourierViscosity(w["nu_seed"]) if "nu_seed" in w else 1.0
    mg = Multigrid(w["dim"], n, w["r"], w["k"], w["n_sub"], TAU, nu=nu, amp=w["deform_amp"], n_coarse=2,
                   k_min=w["k_min"], omega=OMEGA)
    L = mg.levels[0]
    b = random_rhs(w["dim"], n, w["r"], w["k"], w["n_sub"], w["seed"])
    t0 = time.perf_counter()
    x, it, _ = fgmres(L.apply, mg.vcycle, b, rtol=1e-8, max_it=100)
    t = time.perf_counter() - t0
    return {"value": L.ndofs / t, "unit": "space-time DoF/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle FGMRES+V-cycle to 1e-8 on the same element/slab with a 4^3 mesh "
                      f"({L.ndofs} dofs, {it} iterations, {t:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="learned", choices=["learned", "mixed", "fp64"])
    ap.add_argument("--weights", default=WEIGHTS, help="trained network (from paper_2502_09159_amd.train_c4)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--k-min", type=int, default=None, help="override the temporal p-coarsening floor")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (multi-GPU sharding is a design, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2502_09159_amd import stmg
    from stmg_inputs import FourierViscosity, random_rhs

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = dict(WORKLOADS[args.workload])
    if args.k_min is not None:
        w["k_min"] = args.k_min
    nu_fn = FourierViscosity(w["nu_seed"]) if "nu_seed" in w else None
    prec = stmg.FP64 if args.variant == "fp64" else stmg.MIXED_FP32
    t0 = time.perf_counter()
    S = stmg.Solver(nu_fn=nu_fn, **solver_params(w, prec))
    if args.variant == "learned":
        S.learned_load(np.load(args.weights, allow_pickle=False))
        S.learned_enable(True)
    setup_s = time.perf_counter() - t0
    print(f"[bench] setup {args.workload} {args.variant}: {setup_s:.1f} s", file=sys.stderr, flush=True)
    ndofs = S.ndofs(0)
    b = torch.tensor(random_rhs(w["dim"], w["n_cells_1d"], w["r"], w["k"], w["n_sub"], w["seed"]), device="cuda")
    x = torch.empty_like(b)
    for i in range(args.warmup):
        info = S.solve(b, x, rtol=1e-8, max_it=200)
        print(f"[bench] warmup {i}: {info['iterations']} it, {info['t_solve_s']*1e3:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    its, disabled = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        info = S.solve(b, x, rtol=1e-8, max_it=200)
        its.append(info["iterations"])
        disabled.append(info["learned_disabled"])
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms_per_step = 1e3 * t / args.steps
    value = ndofs / (t / args.steps)
    print(f"[bench] timed: {ms_per_step:.1f} ms/solve, {its} it", file=sys.stderr, flush=True)

    # dominant kernel: the Vanka correction on the finest level, event-timed
    # on the stream the library launches on (torch's current stream)
    stream = torch.cuda.current_stream()
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lib_ms = S.kernel_time(0, level=0, reps=reps)
    e1.record(stream)
    torch.cuda.synchronize()
    ev_ms = e0.elapsed_time(e1) / reps
    elem = 4 if prec == stmg.MIXED_FP32 else 8
    ncell = w["n_cells_1d"] ** w["dim"]
    nbytes = vanka_bytes(w, ncell, elem)
    achieved = nbytes / (lib_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_vanka_mfma + k_vanka_gather (finest level)", "ms_per_launch_group": round(lib_ms, 4),
                "ms_event_bracket": round(ev_ms, 4), "algorithmic_bytes": nbytes}
    op_ms = S.kernel_time(1, level=0, reps=reps)

    extra = {}
    if args.variant == "learned":
        extra["learned_switched_off"] = disabled
    if not args.no_compare and args.variant == "learned":
        # the same FP32 context with the network off
        S.learned_enable(False)
        x32 = torch.empty_like(b)
        S.solve(b, x32, rtol=1e-8, max_it=200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info32 = S.solve(b, x32, rtol=1e-8, max_it=200)
        torch.cuda.synchronize()
        t32 = time.perf_counter() - t0
        S.learned_enable(True)
        extra.update({"fp32_plain_dofs_per_s": ndofs / t32, "fp32_plain_iterations": info32["iterations"]})
    if not args.no_compare and args.variant != "fp64":
        S64 = stmg.Solver(nu_fn=nu_fn, **solver_params(w, stmg.FP64))
        x64 = torch.empty_like(b)
        info64 = S64.solve(b, x64, rtol=1e-8, max_it=200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info64 = S64.solve(b, x64, rtol=1e-8, max_it=200)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        extra.update({"fp64_dofs_per_s": ndofs / t64, "fp64_iterations": info64["iterations"],
                      "speedup_vs_fp64": (ndofs / (t / args.steps)) / (ndofs / t64),
                      "rel_err_vs_fp64": (torch.linalg.norm(x - x64) / torch.linalg.norm(x64)).item()})
        S64.close()
    cpu = None if args.no_cpu_baseline else cpu_baseline(w)
    line = {
        "metric": METRIC, "value": value, "unit": "space-time DoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"learned": "f32+bf16+f64", "mixed": "f32+f64", "fp64": "f64"}[args.variant],
        "data": "synthetic",
        "config": {"workload": w["label"], "ndofs": ndofs, "variant": args.variant,
                   "solver": "FGMRES(CGS2) + hp space-time MG V-cycle, cell Vanka (1 pre/1 post), omega 0.8"
                             + (", learned correction on Q2/P1 x DG(1) levels" if args.variant == "learned" else ""),
                   "iterations": its[-1], "setup_s": round(setup_s, 2),
                   "operator_residual_ms": round(op_ms, 4), **extra},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    S.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
