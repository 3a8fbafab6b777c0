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
    # 3D Stokes, Q3/P2disc x DG(2), 16^3 deformed hexes, slab of 4 subintervals; the temporal degree is kept
    # on every level (the literal k -> 0 hierarchy is workload c2_k0)
    "c2": dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=2, k=2, n_sub=4, deform_amp=0.03, k_min=2, seed=2,
               label="3D Stokes Q3/P2disc x DG(2), 16^3 deformed hex mesh, slab of 4 subintervals, nu=1"),
    # the same with the hp hierarchy k -> 0, r -> 1, then h down to 2^3
    "c2_k0": dict(dim=3, n_cells_1d=16, n_coarse_1d=2, r=2, k=2, n_sub=4, deform_amp=0.03, k_min=0, seed=2,
                  label="3D Stokes Q3/P2disc x DG(2), 16^3 deformed hex mesh, slab of 4 subintervals, nu=1, "
                        "hp hierarchy k -> 0"),
    # the learned form's evaluation: 3D Stokes Q3/P2disc x DG(2), 32^3 deformed, 4 subintervals, with r and k
    # halved together on the fine mesh so that the network's Q2/P1 x DG(1) element is the second level
    "c4": dict(dim=3, n_cells_1d=32, n_coarse_1d=2, r=2, k=2, n_sub=4, deform_amp=0.03, k_min=1, placement=1,
               seed=4, label="3D Stokes Q3/P2disc x DG(2), 32^3 deformed hex mesh, slab of 4 subintervals, nu=1, "
                             "r and k halved together on the fine mesh"),
    # 3D Stokes, Q3/P2disc x DG(1), 32^3 deformed, 4 subintervals
    "c3": dict(dim=3, n_cells_1d=32, n_coarse_1d=2, r=2, k=1, n_sub=4, deform_amp=0.03, k_min=1, seed=3,
               label="3D Stokes Q3/P2disc x DG(1), 32^3 deformed hex mesh, slab of 4 subintervals, nu=1"),
    # 3D Stokes, Q3/P2disc x DG(1), 32^3 deformed, 8 subintervals, nu(x) = exp(0.5 g(x))
    "c5": dict(dim=3, n_cells_1d=32, n_coarse_1d=2, r=2, k=1, n_sub=8, deform_amp=0.03, k_min=1, seed=5,
               nu_seed=5, label="3D Stokes Q3/P2disc x DG(1), 32^3 deformed hex mesh, slab of 8 subintervals, "
                                "nu(x)=exp(0.5 g(x))"),
}
TAU, OMEGA = 0.05, 0.8
# Vanka sweeps before and after the coarse-grid correction on the slab
# workloads: the fastest schedule at C5 for the FP32 and the FP64 V-cycle
# alike in a sweep over (pre, post) in {1, 2}^2 and omega in {0.6, ..., 0.95}
PRE, POST = 1, 2
WEIGHTS = os.path.join(ROOT, "paper_2502_09159_amd", "weights", "net_c4.npy")


def solver_params(w, precision):
    keys = ("dim", "n_cells_1d", "n_coarse_1d", "r", "k", "n_sub", "deform_amp", "k_min", "placement")
    p = {k: w[k] for k in keys if k in w}
    p.update(tau=TAU, nu=1.0, omega=w.get("omega", OMEGA), precision=precision)
    p.update(nu_pre=w.get("pre", PRE), nu_post=w.get("post", POST), local_solver=w.get("local_solver", 0))
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


def vanka_form(w):
    """Stored form of the finest level's local inverses under the library's
    default: decoupled in time on levels with 64 or more velocity nodes per
    cell, Schur-factored space-time blocks below."""
    d, nl = w["dim"], (w["r"] + 2) ** w["dim"]
    return "decoupled" if nl >= 64 else "coupled"


def vanka_local_bytes(w, elem_bytes):
    """Algorithmic bytes of the Vanka local solves on the finest level, for
    the stored form the library uses there, plus one read of the residual,
    the cell-local velocity corrections written once, and the pressure
    unknowns read and written once.
      coupled (k_vanka_mfma): A_s^{-1} padded to 16 (mp^2, m = (k+1) nl),
        B (C d nl), F (d m P), H^{-1} (P^2), P = (k+1) C;
      decoupled (k_vanka_tdec): the k+1 real nl x nl blocks (padded to 16) of
        the real and complex spatial inverses, each symmetric and stored as
        its upper 16 x 16 tiles (nkb (nkb + 1) / 2 of them, nkb = nl / 16
        rounded up), B, F (J d nl complex) and H^{-1} (J C^2 complex),
        J = ceil((k+1)/2) blocks."""
    d, nl, nt, C, N, ncells, ndofs = element_sizes(w)
    if vanka_form(w) == "decoupled":
        nkb = (nl + 15) // 16
        J = (nt + 1) // 2
        factors = nt * nkb * (nkb + 1) // 2 * 256 + C * d * nl + J * d * nl * 2 * C + J * C * 2 * C
    else:
        m, P = nt * nl, nt * C
        mp = (m + 15) // 16 * 16
        factors = mp * mp + C * d * nl + d * m * P + P * P
    corrections = ncells * d * nt * nl * N
    pressure = 2 * ncells * C * nt * N
    return (ncells * factors + ndofs + corrections + pressure) * elem_bytes


def operator_bytes(w, elem_bytes):
    """Algorithmic HBM bytes of one residual apply r = b - S x on the finest
    level (cell kernel and node gather together): x, b and r once, and the
    per-Gauss-point metric once (1 + d^2 + d(d+1)/2 values a point)."""
    d, nl, nt, C, N, ncells, ndofs = element_sizes(w)
    metric = 1 + d * d + d * (d + 1) // 2
    return elem_bytes * (3.0 * ndofs + ncells * metric * nl)


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


def cpu_baseline(w, n):
    """The oracle as it stands, timed on this host: set-up (level matrices,
    local inverses, transfers) and then FGMRES + V-cycle to 1e-8 on the same
    element, slab and viscosity with an n^d mesh (the full mesh does not fit
    the oracle's assembled matrices in host memory)."""
    import platform
    from oracle.fgmres import fgmres
    from oracle.mg import Multigrid
    from stmg_inputs import FourierViscosity, random_rhs
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    cpu = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    nu = FourierViscosity(w["nu_seed"]) if "nu_seed" in w else 1.0
    t0 = time.perf_counter()
    mg = Multigrid(w["dim"], n, w["r"], w["k"], w["n_sub"], TAU, nu=nu, amp=w["deform_amp"], n_coarse=2,
                   k_min=w["k_min"], omega=w.get("omega", OMEGA), nu_pre=w.get("pre", PRE),
                   nu_post=w.get("post", POST), placement="top" if w.get("placement", 0) == 1 else "paper")
    setup = time.perf_counter() - t0
    L = mg.levels[0]
    b = random_rhs(w["dim"], n, w["r"], w["k"], w["n_sub"], w["seed"])
    t0 = time.perf_counter()
    x, it, _ = fgmres(L.apply, mg.vcycle, b, rtol=1e-8, max_it=100)
    t = time.perf_counter() - t0
    return {"value": L.ndofs / t, "unit": "space-time DoF/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle FGMRES+V-cycle to 1e-8 on the same element/slab/viscosity with a {n}^{w['dim']} "
                      f"mesh ({L.ndofs} dofs, {it} iterations, solve {t:.1f} s, set-up {setup:.1f} s; {cpu})"}


def timed_solves(S, b, x, steps, warmup, label, max_it=200):
    """Time `steps` solves to 1e-8 after `warmup` untimed ones; a solve that
    stops at max_it first is reported, not raised (its relative residual is
    returned)."""
    for i in range(warmup):
        info = S.solve(b, x, rtol=1e-8, max_it=max_it, raise_on_noconv=False)
        print(f"[bench] {label} warmup {i}: {info['iterations']} it, {info['t_solve_s']*1e3:.1f} ms",
              file=sys.stderr, flush=True)
    import torch
    torch.cuda.synchronize()
    its, disabled = [], []
    t0 = time.perf_counter()
    for i in range(steps):
        info = S.solve(b, x, rtol=1e-8, max_it=max_it, raise_on_noconv=False)
        its.append(info["iterations"])
        disabled.append(info["learned_disabled"])
    timed_solves.learned_steps = info["learned_steps"]
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    timed_solves.last_rel = info["rel_residual"]
    print(f"[bench] {label} timed: {t*1e3:.1f} ms/solve, {its} it, rel. residual {info['rel_residual']:.2e}",
          file=sys.stderr, flush=True)
    return t, its, disabled


def event_ms(S, which, level, reps=10):
    """Mean duration of one launch of kernel class `which` on `level`, with
    torch events on the stream the library launches on; the library's own
    event timing is returned beside it."""
    import torch
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lib_ms = S.kernel_time(which, level=level, reps=reps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, lib_ms


def run_lid(args):
    """The paper's lid-driven cavity (Sec. 5.2) at reduced size, by time
    marching: [0,1]^3 x [0,8], uniform mesh refined c times (2^c cells per
    direction, 2^(c+4) time steps of one subinterval each), Q3/P2disc x DG(2)
    (r = k = 2), lid velocity (sin(pi t / 4), 0, 0) on the face z = 1, no-slip
    walls, v0 = 0, nu = 0.1, every slab to 1e-8.  One step is the whole march;
    value = all space-time dofs / its wall time (the paper's throughput)."""
    import torch

    from paper_2502_09159_amd import stmg
    from stmg_inputs import lid_dirichlet
    c = args.lid_c
    n, n_slabs, r, k = 2 ** c, 2 ** (c + 4), 2, 2
    tau = 8.0 / n_slabs
    out = {}
    for prec, tag in ((stmg.MIXED_FP32, "mixed"), (stmg.FP64, "fp64")):
        for k_min in (1, k):
            S = stmg.Solver(dim=3, n_cells_1d=n, n_coarse_1d=2, r=r, k=k, n_sub=1, deform_amp=0.0, k_min=k_min,
                            tau=tau, nu=0.1, omega=OMEGA, precision=prec, nu_pre=args.nsm, nu_post=args.nsm,
                            local_solver=1 if args.local_solver == "diagonal" else 0)
            nd = S.ndofs(0)
            t_hat = S.time_nodes()
            G = torch.empty(n_slabs * nd, dtype=torch.float64, device="cuda")
            for s in range(n_slabs):
                G[s * nd:(s + 1) * nd] = torch.from_numpy(lid_dirichlet(3, n, r, k, 1, tau, s * tau, t_hat))
            x = torch.empty_like(G)
            nw = min(4, n_slabs)
            S.march(nw, x[: nw * nd], g=G[: nw * nd], rtol=1e-8, max_it=200)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = S.march(n_slabs, x, g=G, rtol=1e-8, max_it=200)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            key = f"{tag}_kmin{k_min}"
            out[key] = {"seconds": round(t, 3), "dofs_per_s": n_slabs * nd / t,
                        "iterations_avg": float(np.mean(its)), "iterations_max": int(np.max(its))}
            print(f"[bench] lid c={c} {key}: {t:.2f} s, {n_slabs * nd / t / 1e6:.1f} M dof/s, "
                  f"iterations avg {np.mean(its):.2f} max {np.max(its)}", file=sys.stderr, flush=True)
            del G, x
            S.close()
    best = out["mixed_kmin1"]
    line = {"metric": "space-time DoF/s of the time-marching lid-driven cavity (all slabs to 1e-8)",
            "value": best["dofs_per_s"], "unit": "space-time DoF/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": 1e3 * best["seconds"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": f"3D lid-driven cavity, c={c}: {n}^3 cells, {n_slabs} time steps of tau={tau}, "
                                   f"Q3/P2disc x DG(2), nu=0.1, time marching one subinterval per slab, "
                                   f"{args.local_solver} cell Vanka, n_sm={args.nsm}",
                       "ndofs_per_slab": nd, "ndofs_total": n_slabs * nd, "variants": out,
                       "paper_context": "Table 3 (c=4, r=2, n_sm=1): 18.14 GMRES iterations per step; Table 4: "
                                        "302,520,576 dofs in 149.4 s on 13,824 MPI ranks"}}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS) + ["lid"])
    ap.add_argument("--lid-c", type=int, default=4, help="refinement level c of the lid-driven cavity")
    ap.add_argument("--variant", default="learned", choices=["learned", "mixed", "fp64"])
    ap.add_argument("--weights", default=WEIGHTS, help="trained network (from paper_2502_09159_amd.train_c4)")
    ap.add_argument("--nsm", type=int, default=None,
                    help="Vanka sweeps before and after the coarse correction (n_sm of Tables 3 and 4; default "
                         f"{PRE} before and {POST} after on the slab workloads, 2 and 2 for the lid-driven cavity)")
    ap.add_argument("--pre", type=int, default=None, help="Vanka sweeps before the coarse correction")
    ap.add_argument("--post", type=int, default=None, help="Vanka sweeps after the coarse correction")
    ap.add_argument("--omega", type=float, default=OMEGA, help="Vanka relaxation")
    ap.add_argument("--local-solver", default="exact", choices=["exact", "diagonal"],
                    help="exact patch inverses or the diagonal Vanka")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=8, help="mesh of the oracle baseline sample (n^d cells)")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--max-it", type=int, default=None, help="FGMRES iteration cap (default 200; 600 for c4)")
    ap.add_argument("--k-min", type=int, default=None, help="override the temporal p-coarsening floor")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only (the solver is not sharded across GPUs)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "lid":
        if args.nsm is None:
            args.nsm = 2
        run_lid(args)
        return

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
    w["pre"] = args.pre if args.pre is not None else (args.nsm if args.nsm is not None else PRE)
    w["post"] = args.post if args.post is not None else (args.nsm if args.nsm is not None else POST)
    w["omega"] = args.omega
    w["local_solver"] = 1 if args.local_solver == "diagonal" else 0
    if args.max_it is None:
        args.max_it = 600 if args.workload == "c4" else 200
    if args.k_min is not None:
        w["k_min"] = args.k_min
    nu_fn = FourierViscosity(w["nu_seed"]) if "nu_seed" in w else None
    prec = stmg.FP64 if args.variant == "fp64" else stmg.MIXED_FP32
    weights = np.load(args.weights, allow_pickle=False) if args.variant == "learned" else None
    t0 = time.perf_counter()
    S = stmg.Solver(nu_fn=nu_fn, **solver_params(w, prec))
    if weights is not None:
        S.learned_load(weights)
        S.learned_enable(True)
    setup_s = time.perf_counter() - t0
    print(f"[bench] setup {args.workload} {args.variant}: {setup_s:.1f} s", file=sys.stderr, flush=True)
    ndofs = S.ndofs(0)
    b = torch.tensor(random_rhs(w["dim"], w["n_cells_1d"], w["r"], w["k"], w["n_sub"], w["seed"]), device="cuda")
    x = torch.empty_like(b)
    max_it = args.max_it
    t, its, disabled = timed_solves(S, b, x, args.steps, args.warmup, args.variant, max_it)
    rel_final = timed_solves.last_rel
    ms_per_step = 1e3 * t
    value = ndofs / t

    # dominant kernel: the Vanka local solves on the finest level (the
    # decoupled k_vanka_tdec or the Schur-factored k_vanka_mfma), event-timed
    elem = 4 if prec == stmg.MIXED_FP32 else 8
    form = vanka_form(w)
    kname = "k_vanka_tdec" if form == "decoupled" else "k_vanka_mfma"
    ev_ms, lib_ms = event_ms(S, 2, 0)
    nbytes = vanka_local_bytes(w, elem)
    achieved = nbytes / (ev_ms * 1e-3) / 1e9
    d_, nl_, nt_, C_, N_, ncells_, _ = element_sizes(w)
    traffic = measured_traffic(kname, ncells_ * 256)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"{kname} (finest level, {form} local solves of every cell)",
                "ms_per_launch": round(ev_ms, 4), "ms_library_events": round(lib_ms, 4),
                "algorithmic_bytes": nbytes}
    # the operator's cell kernel on the finest level (VALU-bound: flops of the
    # sum-factorized evaluation over its event-timed duration)
    cell_ev_ms, cell_ms = event_ms(S, 3, 0)
    flops = apply_cell_flops(w)
    # non-packed vector peak: packed FP32 instructions are not used (78.6 TFLOP/s for FP32 and FP64 alike)
    alu_peak = 78.6
    roofline_apply = {"bound": "alu", "achieved": round(flops / (cell_ev_ms * 1e-3) / 1e12, 2), "peak": alu_peak,
                      "unit": "TFLOP/s", "frac": round(flops / (cell_ev_ms * 1e-3) / 1e12 / alu_peak, 4),
                      "peak_note": "vector FMA issue without packed FP32 (157.3 TFLOP/s with it)",
                      "kernel": "k_apply (finest level, cell kernel)", "ms_per_launch": round(cell_ev_ms, 4),
                      "ms_library_events": round(cell_ms, 4), "flops": flops}
    abytes = apply_cell_bytes(w)
    roofline_apply["hbm_view"] = {"achieved": round(abytes / (cell_ev_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": round(abytes / (cell_ev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "algorithmic_bytes": abytes}
    # the whole residual apply b - S x (cell kernel and node gather) against HBM
    op_ev_ms, op_ms = event_ms(S, 1, 0)
    obytes = operator_bytes(w, elem)
    roofline_operator = {"bound": "alu", "kernel": "operator residual b - S x (k_apply + k_node_gather)",
                         "ms_per_launch": round(op_ev_ms, 4), "ms_library_events": round(op_ms, 4),
                         "hbm": {"achieved": round(obytes / (op_ev_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": round(obytes / (op_ev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "algorithmic_bytes": obytes},
                         "alu": {"achieved": round(flops / (op_ev_ms * 1e-3) / 1e12, 2), "peak": alu_peak,
                                 "unit": "TFLOP/s", "frac": round(flops / (op_ev_ms * 1e-3) / 1e12 / alu_peak, 4)}}

    extra = {}
    if args.variant == "learned":
        extra["learned_switched_off"] = disabled
        extra["learned_steps_applied"] = timed_solves.learned_steps
    if not args.no_compare and args.variant == "learned":
        # the same FP32 context with the network off, and the network on the
        # network's own element levels only (reading A)
        S.learned_enable(False)
        x32 = torch.empty_like(b)
        t32, its32, _ = timed_solves(S, b, x32, 1, 1, "fp32 (no network)", max_it)
        extra.update({"fp32_plain_dofs_per_s": ndofs / t32, "fp32_plain_iterations": its32[-1],
                      "fp32_plain_rel_residual": timed_solves.last_rel})
        if args.workload == "c4":
            S.learned_enable(True, element_levels_only=True)
            xa = torch.empty_like(b)
            ta, itsa, da = timed_solves(S, b, xa, 1, 1, "fp32 + network, r1k1 levels only", max_it)
            rela = timed_solves.last_rel
            from paper_2502_09159_amd.learned import he_init
            S.learned_load(he_init(0))
            S.learned_enable(True)
            xu = torch.empty_like(b)
            tu, itsu, du = timed_solves(S, b, xu, 1, 1, "fp32 + untrained network", max_it)
            extra.update({"learned_element_levels_only": {"dofs_per_s": ndofs / ta, "iterations": itsa[-1],
                                                           "switched_off": da[-1], "rel_residual": rela},
                          "untrained_network": {"dofs_per_s": ndofs / tu, "iterations": itsu[-1],
                                                "switched_off": du[-1], "rel_residual": timed_solves.last_rel}})
            S.learned_load(weights)
        S.learned_enable(True)
    if not args.no_compare and args.variant != "fp64":
        S64 = stmg.Solver(nu_fn=nu_fn, **solver_params(w, stmg.FP64))
        x64 = torch.empty_like(b)
        t64, its64, _ = timed_solves(S64, b, x64, 1, 1, "fp64", max_it)
        extra.update({"fp64_dofs_per_s": ndofs / t64, "fp64_iterations": its64[-1],
                      "fp64_rel_residual": timed_solves.last_rel,
                      "speedup_vs_fp64": value / (ndofs / t64),
                      "rel_err_vs_fp64": (torch.linalg.norm(x - x64) / torch.linalg.norm(x64)).item()})
        S64.close()
        if args.workload == "c4":
            # plain FP64 multigrid with the library's default hierarchy for
            # this discretisation (temporal degree kept on every level)
            w2 = dict(w, k_min=w["k"])
            w2.pop("placement", None)
            S2 = stmg.Solver(nu_fn=nu_fn, **solver_params(w2, stmg.FP64))
            x2 = torch.empty_like(b)
            t2, its2, _ = timed_solves(S2, b, x2, 1, 1, "fp64, default hierarchy", max_it)
            extra["fp64_default_hierarchy"] = {"dofs_per_s": ndofs / t2, "iterations": its2[-1],
                                               "rel_residual": timed_solves.last_rel}
            S2.close()
    cpu = None if args.no_cpu_baseline else cpu_baseline(w, args.cpu_n)
    line = {
        "metric": METRIC, "value": value, "unit": "space-time DoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"learned": "f32+bf16+f64", "mixed": "f32+f64", "fp64": "f64"}[args.variant],
        "data": "synthetic",
        "config": {"workload": w["label"], "ndofs": ndofs, "variant": args.variant,
                   "solver": f"FGMRES(CGS2) + hp space-time MG V-cycle, {args.local_solver} cell Vanka "
                             f"({w['pre']} pre/{w['post']} post), omega {w['omega']}"
                             + (", learned correction on Q2/P1 x DG(1) levels" if args.variant == "learned" else ""),
                   "iterations": its[-1], "rel_residual": rel_final, "setup_s": round(setup_s, 2),
                   "operator_residual_ms": round(op_ms, 4), **extra},
        "roofline": roofline, "roofline_apply": roofline_apply, "roofline_operator": roofline_operator,
        "cpu_baseline": cpu,
    }
    S.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
