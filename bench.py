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


def element_sizes(w):
    from math import comb
    d, r, k, N = w["dim"], w["r"], w["k"], w["n_sub"]
    nl = (r + 2) ** d
    nt = k + 1
    C = comb(r + d, d)
    n = w["n_cells_1d"]
    ncells = n ** d
    ndofs = N * nt * (d * (n * (r + 1) + 1) ** d + ncells * C)
    return d, nl, nt, C, N, ncells, ndofs


def vanka_local_bytes(w, elem_bytes):
    """Algorithmic bytes of the Vanka local solves on the finest level (the
    kernel k_vanka_mfma): the stored factors of every cell (A_s^{-1} padded to
    16: mp^2, B: C d nl, F: d m P, H^{-1}: P^2), one read of the residual,
    the cell-local velocity corrections written once, and the pressure
    unknowns read and written once."""
    d, nl, nt, C, N, ncells, ndofs = element_sizes(w)
    m, P = nt * nl, nt * C
    mp = (m + 15) // 16 * 16
    factors = mp * mp + C * d * nl + d * m * P + P * P
    corrections = ncells * d * m * N
    pressure = 2 * ncells * C * nt * N
    return (ncells * factors + ndofs + corrections + pressure) * elem_bytes


def apply_cell_flops(w):
    """Floating-point operations of the operator's cell kernel on the finest
    level, counting every sum-factorized contraction once (an FMA is 2 flops):
    per cell and subinterval, the interpolation of the d(k+1) velocity fields
    (3 contractions of Q^4 FMAs each), then per (component, temporal dof) the
    mass/jump term (k+2 FMAs a point), the reference gradient (3 contractions),
    the flux with the metric and pressure (about 5d FMAs a point), the
    transposed gradient and interpolation (6 contractions), plus the pressure
    interpolation and the divergence test (C FMAs a point each, per temporal
    dof)."""
    d, nl, nt, C, N, ncells, ndofs = element_sizes(w)
    Q = w["r"] + 2
    contraction = nl * Q  # one 1D contraction of a cell
    interp = d * nt * d * contraction
    per_field = nl * (nt + 1) + d * contraction + nl * 5 * d + 2 * d * contraction
    pres = 2 * nt * nl * C
    return 2.0 * ncells * N * (interp + d * nt * per_field + pres)


def apply_cell_bytes(w):
    """Algorithmic HBM bytes of the operator's cell kernel on the finest level
    (FP32): the input vector once, the per-Gauss-point metric once (JxW, JxW
    J^-1 and nu JxW J^-1 J^-T: 1 + d^2 + d(d+1)/2 values a point), the
    cell-local velocity results E written once and the pressure rows written
    once."""
    d, nl, nt, C, N, ncells, ndofs = element_sizes(w)
    metric = 1 + d * d + d * (d + 1) // 2
    return 4.0 * (ndofs + ncells * metric * nl + ncells * d * nt * nl * N + ncells * C * nt * N)


def measured_traffic(kernel_prefix, grid):
    """Scaled HBM bytes per launch of a kernel from the counter summary kept
    in profiles/ (FETCH_SIZE and WRITE_SIZE runs), or None when the kernel
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_counters.json")
    src = os.path.join(ROOT, "paper_2502_09159_amd", "csrc", "kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hip_sha256") != sha:
        return None
    for k in rec.get("kernels", []):
        if k["name"].startswith(kernel_prefix) and k["grid"] == grid:
            return k["fetch_bytes"] + k["write_bytes"]
    return None


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
        print("bench.py: measures one GPU only (the solver is not sharded across GPUs)",
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

    # dominant kernel: the Vanka local solves on the finest level
    # (k_vanka_mfma), event-timed on the stream the library launches on
    # (torch's current stream); the library's own event timing is reported beside
    stream = torch.cuda.current_stream()
    reps = 10
    elem = 4 if prec == stmg.MIXED_FP32 else 8
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lib_ms = S.kernel_time(2, level=0, reps=reps)
    e1.record(stream)
    torch.cuda.synchronize()
    ev_ms = e0.elapsed_time(e1) / reps
    nbytes = vanka_local_bytes(w, elem)
    achieved = nbytes / (ev_ms * 1e-3) / 1e9
    d_, nl_, nt_, C_, N_, ncells_, _ = element_sizes(w)
    traffic = measured_traffic("k_vanka_mfma", ncells_ * 256)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_vanka_mfma (finest level, local solves of every cell)",
                "ms_per_launch": round(ev_ms, 4), "ms_library_events": round(lib_ms, 4),
                "algorithmic_bytes": nbytes}
    # the operator's cell kernel on the finest level (ALU-bound: flops of the
    # sum-factorized evaluation over its event-timed duration)
    e0.record(stream)
    cell_ms = S.kernel_time(3, level=0, reps=reps)
    e1.record(stream)
    torch.cuda.synchronize()
    cell_ev_ms = e0.elapsed_time(e1) / reps
    flops = apply_cell_flops(w)
    alu_peak = 157.3 if elem == 4 else 78.6
    roofline_apply = {"bound": "alu", "achieved": round(flops / (cell_ev_ms * 1e-3) / 1e12, 2), "peak": alu_peak,
                      "unit": "TFLOP/s", "frac": round(flops / (cell_ev_ms * 1e-3) / 1e12 / alu_peak, 4),
                      "kernel": "k_apply (finest level, cell kernel)", "ms_per_launch": round(cell_ev_ms, 4),
                      "ms_library_events": round(cell_ms, 4), "flops": flops}
    abytes = apply_cell_bytes(w)
    roofline_apply["hbm_view"] = {"achieved": round(abytes / (cell_ev_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": round(abytes / (cell_ev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "algorithmic_bytes": abytes}
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
        "roofline": roofline, "roofline_apply": roofline_apply, "cpu_baseline": cpu,
    }
    S.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
