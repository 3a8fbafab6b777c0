"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) per kernel:
calls, total and average duration, share of GPU time, VGPR/scratch use.

Usage: python -m paper_2502_09159_amd.prof_summary <results.db> [title]
"""
import sqlite3
import sys


def short(name):
    name = name.replace("(anonymous namespace)::", "").split("(")[0]
    return name.replace("void ", "").replace("stmg::", "")[:90]


def main(path, title=""):
    db = sqlite3.connect(path)
    rows = db.execute("select name, duration, grid_x, workgroup_x, vgpr_count, accum_vgpr_count, scratch_size, "
                      "lds_size from kernels").fetchall()
    agg = {}
    for name, dur, gx, wx, vg, avg, scr, lds in rows:
        k = short(name)
        a = agg.setdefault(k, [0, 0.0, vg, avg, scr, lds])
        a[0] += 1
        a[1] += dur
    total = sum(a[1] for a in agg.values())
    print(f"# {title}".rstrip())
    print(f"kernels: {len(rows)} dispatches, {total / 1e6:.3f} ms GPU time")
    print(f"{'kernel':60s} {'calls':>6s} {'total_ms':>9s} {'avg_us':>9s} {'%':>6s} {'vgpr':>5s} {'scr':>5s} {'lds':>6s}")
    for k, (n, t, vg, avg, scr, lds) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"{k[:60]:60s} {n:6d} {t / 1e6:9.3f} {t / n / 1e3:9.2f} {100 * t / total:6.2f} {vg:5d} {scr:5d} "
              f"{lds:6d}")


if __name__ == "__main__":
    main(sys.argv[1], " ".join(sys.argv[2:]))
