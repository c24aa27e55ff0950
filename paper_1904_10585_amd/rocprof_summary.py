"""Summaries of rocprofv3 output for the extraction kernels.

    python -m paper_1904_10585_amd.rocprof_summary trace <results.db> [--steps K]
        per-kernel call count, total and average duration from a
        ``rocprofv3 --kernel-trace`` SQLite database;
    python -m paper_1904_10585_amd.rocprof_summary counters <run.csv>... --kernel NAME
        per-dispatch mean of every counter of one kernel over one or more
        ``rocprofv3 --pmc`` runs (CSV output);
    python -m paper_1904_10585_amd.rocprof_summary bytes <fetch.csv> <write.csv> --kernel NAME [--kernel NAME2]
        HBM bytes per dispatch of one kernel (plus the kernels that complete
        each of its launches, e.g. a split-K slab sum) from two ``rocprofv3 --pmc``
        runs (FETCH_SIZE, then WRITE_SIZE, CSV output), each scaled by what
        the same counter reads for the runtime's device-to-device copy of a
        known size (``bench.py --calib-copy``: 256 MiB read, 256 MiB written).
"""
import argparse
import collections
import csv
import re
import sqlite3

CALIB_KERNEL = "__amd_rocclr_copyBuffer"
CALIB_BYTES = 256 << 20


def short_name(name):
    s = name.replace("(anonymous namespace)::", "").replace("pfx::", "")
    s = re.sub(r"^void ", "", s)
    return re.sub(r"\(.*", "", s)


def trace(db, steps):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
                       "from kernels group by name order by sum(duration) desc").fetchall()
    print(f"| kernel | calls | total ms | avg us | min us | max us |" + (" ms/step |" if steps else ""))
    print("|---|---:|---:|---:|---:|---:|" + ("---:|" if steps else ""))
    for name, n, tot, avg, mn, mx in rows:
        line = f"| `{short_name(name)[:80]}` | {n} | {tot / 1e6:.3f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} |"
        if steps:
            line += f" {tot / 1e6 / steps:.4f} |"
        print(line)


def counter_means(path):
    """Mean counter value per (kernel, counter).  For the calibration copy
    only the dispatches of the largest grid count (the 256 MiB copy; the
    runtime uses the same kernel for small copies)."""
    rows = list(csv.DictReader(open(path)))
    calib_grid = max((int(r["Grid_Size"]) for r in rows if short_name(r["Kernel_Name"]) == CALIB_KERNEL),
                     default=0)
    agg = collections.defaultdict(list)
    for row in rows:
        name = short_name(row["Kernel_Name"])
        if name == CALIB_KERNEL and int(row["Grid_Size"]) != calib_grid:
            continue
        agg[(name, row["Counter_Name"])].append(float(row["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}


def bytes_per_dispatch(fetch_csv, write_csv, kernels):
    """HBM bytes per launch of the first kernel, summed over the kernels
    given (e.g. a product and the slab sum that completes it), each
    weighted by its dispatches per dispatch of the first."""
    f = counter_means(fetch_csv)
    w = counter_means(write_csv)
    cf, nf = f[(CALIB_KERNEL, "FETCH_SIZE")]
    cw, nw = w[(CALIB_KERNEL, "WRITE_SIZE")]
    sf = cf * 1024 / CALIB_BYTES            # counter bytes per byte moved
    sw = cw * 1024 / CALIB_BYTES
    print(f"- calibration copy FETCH_SIZE per dispatch: {cf:.1f} KiB over {nf} dispatches (scale {sf:.5f})")
    print(f"- calibration copy WRITE_SIZE per dispatch: {cw:.1f} KiB over {nw} dispatches (scale {sw:.5f})")
    fetch_b = write_b = 0.0
    n0 = None
    for kernel in kernels:
        kf, nkf = f[(kernel, "FETCH_SIZE")]
        kw, nkw = w[(kernel, "WRITE_SIZE")]
        n0 = nkf if n0 is None else n0
        weight = nkf / n0
        print(f"- `{kernel}` FETCH_SIZE per dispatch: {kf:.1f} KiB over {nkf} dispatches; "
              f"WRITE_SIZE {kw:.1f} KiB over {nkw}")
        fetch_b += weight * kf * 1024 / sf
        write_b += weight * kw * 1024 / sw
    print(f"- fetch_bytes_per_launch: {fetch_b:.0f}")
    print(f"- write_bytes_per_launch: {write_b:.0f}")
    print(f"- traffic_bytes_per_launch: {fetch_b + write_b:.0f}")


def counters(paths, kernel):
    for path in paths:
        for (name, counter), (mean, cnt) in sorted(counter_means(path).items()):
            if name == kernel:
                print(f"- {counter}: {mean:.6g} per dispatch over {cnt} dispatches")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--steps", type=float, default=0)
    b = sub.add_parser("bytes")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--kernel", required=True, action="append",
                   help="kernel name (repeat to add the kernels that complete one launch of the first)")
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    c.add_argument("--kernel", required=True)
    a = ap.parse_args()
    if a.cmd == "trace":
        trace(a.db, a.steps)
    elif a.cmd == "counters":
        counters(a.csv, a.kernel)
    else:
        bytes_per_dispatch(a.fetch_csv, a.write_csv, a.kernel)


if __name__ == "__main__":
    main()
