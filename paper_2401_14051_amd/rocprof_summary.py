"""Summaries of rocprofv3 result databases (the SQLite ``*_results.db``).

Kernel timings:
    python -m paper_2401_14051_amd.rocprof_summary times DB [--title T --command C] > out.md

HBM traffic of a kernel's largest launches from two counter runs (FETCH_SIZE,
then WRITE_SIZE), scaled by what the same counters read for a plain copy
kernel of known size:
    python -m paper_2401_14051_amd.rocprof_summary traffic --fetch DB1 --write DB2 \\
        --kernel k_features --copy-kernel elementwise --copy-bytes B > out.json

Per-dispatch (and per-wave) averages of other counters of a kernel's largest
launches:
    python -m paper_2401_14051_amd.rocprof_summary counters DB1 DB2 --kernel k_features > out.md

The traffic summary records a hash of the kernel's source files, so that the
benchmark reports it only while the kernel is unchanged.
"""

import argparse
import collections
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# sources each measured kernel depends on
KERNEL_SOURCES = {
    "features": ["csrc/k_features.hip", "csrc/mfma.h", "csrc/launch_args.h", "csrc/nis_internal.h"],
    "backbone": ["csrc/k_mlp.hip", "csrc/mfma.h", "csrc/launch_args.h", "csrc/nis_internal.h"],
    "sweep": ["csrc/k_volume.hip", "csrc/launch_args.h", "csrc/nis_internal.h"],
}


def source_hash(kernel):
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_times(db):
    """Rows (name, workgroups, calls, avg, min, max, total duration in ns), one
    per kernel and launch size, so that launches of one kernel over different
    batch sizes are not averaged together."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, (grid_x * grid_y * grid_z) / (workgroup_x * workgroup_y * workgroup_z), "
                       "count(*), avg(duration), min(duration), max(duration), sum(duration) from kernels "
                       "group by name, grid_x, grid_y, grid_z order by sum(duration) desc").fetchall()
    return rows


def counters(db, counter):
    """{kernel name: {grid size in work-items: [value per dispatch]}} of one counter."""
    con = sqlite3.connect(db)
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, grid, val in con.execute("select kernel_name, grid_size, value from counters_collection "
                                       "where counter_name = ? order by dispatch_id", (counter,)):
        out[name][grid].append(val)
    return out


def pick(d, key):
    hits = [k for k in d if key in k]
    if len(hits) != 1:
        raise SystemExit("kernel %r matches %r" % (key, hits))
    return d[hits[0]]


def cmd_times(a):
    rows = kernel_times(a.db)
    total = sum(r[6] for r in rows)
    print("# %s\n" % (a.title or "Kernel times"))
    if a.command:
        print("Command:\n\n```\n%s\n```\n" % a.command)
    print("One row per kernel and launch size (workgroups).\n")
    print("| kernel | workgroups | calls | avg (us) | min (us) | max (us) | total (us) | share |")
    print("|---|---|---|---|---|---|---|---|")
    for name, wgs, n, avg, mn, mx, tot in rows:
        print("| `%s` | %d | %d | %.1f | %.1f | %.1f | %.1f | %.1f%% |" % (name[:80], wgs, n, avg / 1e3, mn / 1e3,
                                                                          mx / 1e3, tot / 1e3, 100.0 * tot / total))


def cmd_traffic(a):
    fetch = counters(a.fetch, "FETCH_SIZE")
    write = counters(a.write, "WRITE_SIZE")
    cf = [v for g in pick(fetch, a.copy_kernel).values() for v in g]
    cw = [v for g in pick(write, a.copy_kernel).values() for v in g]
    # the kernel's largest launches: those of a whole frame
    kfg, kwg = pick(fetch, a.kernel), pick(write, a.kernel)
    grid = max(kfg)
    if grid not in kwg:
        raise SystemExit("launch size %d missing from the WRITE_SIZE run" % grid)
    kf, kw = kfg[grid], kwg[grid]
    # counters are in KiB per dispatch; the copy kernel moves copy_bytes each way
    f_scale = a.copy_bytes / (1024.0 * max(cf))
    w_scale = a.copy_bytes / (1024.0 * max(cw))
    fetch_b = 1024.0 * sum(kf) / len(kf) * f_scale
    write_b = 1024.0 * sum(kw) / len(kw) * w_scale
    out = {"kernel": a.name, "source_hash": source_hash(a.name), "grid_work_items": grid,
           "fetch_bytes_per_launch": fetch_b,
           "write_bytes_per_launch": write_b, "traffic_bytes_per_launch": fetch_b + write_b,
           "copy_calibration": {"kernel": a.copy_kernel, "bytes": a.copy_bytes,
                                "fetch_kib": max(cf), "write_kib": max(cw),
                                "fetch_scale": f_scale, "write_scale": w_scale},
           "raw_kib": {"fetch": kf, "write": kw}, "commands": a.command}
    json.dump(out, sys.stdout, indent=1)
    print()


def cmd_counters(a):
    """Per-dispatch averages of every counter in the given runs for the
    kernel's largest launches, and per wave where SQ_WAVES was counted."""
    vals = {}
    for db in a.db:
        con = sqlite3.connect(db)
        names = [r[0] for r in con.execute("select distinct counter_name from counters_collection")]
        for c in names:
            per = collections.defaultdict(lambda: collections.defaultdict(list))
            for name, grid, val in con.execute("select kernel_name, grid_size, value from counters_collection "
                                               "where counter_name = ?", (c,)):
                per[name][grid].append(val)
            g = pick(per, a.kernel)
            top = max(g)
            vals[c] = (top, sum(g[top]) / len(g[top]), len(g[top]))
    print("# %s\n" % (a.title or "Counters"))
    for cmd in a.command:
        print("```\n%s\n```\n" % cmd)
    waves = vals.get("SQ_WAVES", (0, 0.0, 0))[1]
    print("| counter | launch work-items | dispatches | per dispatch | per wave |")
    print("|---|---|---|---|---|")
    for c in sorted(vals):
        grid, avg, n = vals[c]
        pw = "%.1f" % (avg / waves) if waves else "-"
        print("| %s | %d | %d | %.4g | %s |" % (c, grid, n, avg, pw))
    if "SQ_VALU_MFMA_BUSY_CYCLES" in vals and "GRBM_GUI_ACTIVE" in vals:
        # GRBM_GUI_ACTIVE sums the XCDs' clocks; the MFMA busy cycles sum the SIMDs
        cyc = vals["GRBM_GUI_ACTIVE"][1] / a.xcds
        busy = vals["SQ_VALU_MFMA_BUSY_CYCLES"][1]
        print("\nDerived (%d XCDs, %d SIMDs):\n" % (a.xcds, a.simds))
        print("* kernel cycles per XCD (GRBM_GUI_ACTIVE / %d): %.4g" % (a.xcds, cyc))
        print("* MFMA busy fraction (SQ_VALU_MFMA_BUSY_CYCLES / (cycles x %d SIMDs)): %.3f"
              % (a.simds, busy / (cyc * a.simds)))
        for c in sorted(vals):
            if c.startswith("SQ_INSTS_VALU_MFMA_MOPS_") and vals[c][1] > 0:
                print("* %s x 512: %.4g MFMA FLOP per dispatch" % (c, vals[c][1] * 512))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("times")
    t.add_argument("db")
    t.add_argument("--title")
    t.add_argument("--command")
    r = sub.add_parser("traffic")
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--kernel", required=True, help="substring of the measured kernel's name")
    r.add_argument("--name", required=True, choices=sorted(KERNEL_SOURCES))
    r.add_argument("--copy-kernel", required=True)
    r.add_argument("--copy-bytes", type=float, required=True)
    r.add_argument("--command", action="append", default=[])
    c = sub.add_parser("counters")
    c.add_argument("db", nargs="+")
    c.add_argument("--kernel", required=True, help="substring of the measured kernel's name")
    c.add_argument("--title")
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--xcds", type=int, default=8)
    c.add_argument("--simds", type=int, default=1024)
    a = ap.parse_args(argv)
    {"times": cmd_times, "traffic": cmd_traffic, "counters": cmd_counters}[a.cmd](a)


if __name__ == "__main__":
    main()
