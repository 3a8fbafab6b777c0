"""Per-kernel HBM traffic from two rocprofv3 --pmc runs (FETCH_SIZE, then
WRITE_SIZE; rocpd databases), scaled by what the same counter reads for the
reference 1 GiB device copy (bench.py --calibrate-copy).

Usage: python -m paper_2502_09159_amd.pmc_summary <fetch.db> <write.db> [kernel-substring ...]
           [--json out.json]

With --json, the per-dispatch bytes of the selected kernels are also written
to out.json together with the SHA-256 of csrc/kernels.hip (bench.py reports
them as `traffic` only while that source is unchanged).
"""
import hashlib
import json
import os
import sqlite3
import sys

COPY_KIB = 1 << 20  # the reference copy moves 1 GiB


def per_kernel(path, counter):
    db = sqlite3.connect(path)
    rows = db.execute("select kernel_name, grid_size, value from counters_collection where counter_name = ?",
                      (counter,)).fetchall()
    agg = {}
    for name, grid, val in rows:
        k = (name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("stmg::", ""),
             grid)
        a = agg.setdefault(k, [0, 0.0])
        a[0] += 1
        a[1] += val
    return agg


def reference(agg):
    """Counter value (KiB) of the first large copyBuffer dispatch group (the 1 GiB copy)."""
    vals = [v[1] / v[0] for (n, g), v in agg.items() if "copyBuffer" in n and v[1] / v[0] > 100000]
    return max(vals) if vals else None


def main(fetch_db, write_db, *subs):
    subs = list(subs)
    out_json = None
    if "--json" in subs:
        i = subs.index("--json")
        out_json = subs[i + 1]
        del subs[i:i + 2]
    f, w = per_kernel(fetch_db, "FETCH_SIZE"), per_kernel(write_db, "WRITE_SIZE")
    rf, rw = reference(f), reference(w)
    sf = COPY_KIB / rf if rf else 1.0
    sw = COPY_KIB / rw if rw else 1.0
    print(f"reference 1 GiB copy: FETCH_SIZE {rf:.0f} KiB (scale {sf:.3f}), WRITE_SIZE {rw:.0f} KiB (scale {sw:.3f})")
    print(f"{'kernel':50s} {'grid':>10s} {'calls':>6s} {'fetch_MB':>10s} {'write_MB':>10s}   (per dispatch, scaled)")
    rows = []
    for key in sorted(f, key=lambda k: -f[k][1] / f[k][0]):
        name, grid = key
        if subs and not any(s in name for s in subs):
            continue
        n, fv = f[key]
        wv = w.get(key, [1, 0.0])
        print(f"{name[:50]:50s} {grid:10d} {n:6d} {fv / n * sf / 1024:10.1f} {wv[1] / wv[0] * sw / 1024:10.1f}")
        rows.append({"name": name, "grid": grid, "dispatches": n, "fetch_bytes": int(fv / n * sf * 1024),
                     "write_bytes": int(wv[1] / wv[0] * sw * 1024)})
    if out_json:
        src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "kernels.hip")
        rec = {"fetch_scale": sf, "write_scale": sw, "reference": "1 GiB device copy (bench.py --calibrate-copy)",
               "kernels_hip_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(), "kernels": rows}
        with open(out_json, "w") as fh:
            json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main(*sys.argv[1:])
