"""Summaries of rocprofv3 output for the extraction kernels.

    python -m paper_1904_10585_amd.rocprof_summary trace <results.db> [--steps K] [--match TEXT]
        per-kernel call count, total and average duration from a
        ``rocprofv3 --kernel-trace`` SQLite database (optionally only the
        kernels whose name contains TEXT);
    python -m paper_1904_10585_amd.rocprof_summary counters <run.csv>... --kernel NAME
        per-dispatch mean of every counter of one kernel over one or more
        ``rocprofv3 --pmc`` runs (CSV output);
    python -m paper_1904_10585_amd.rocprof_summary bytes <fetch.csv> <write.csv> --kernel NAME [--kernel NAME2]
        HBM bytes per dispatch of one kernel (plus the kernels that complete
        each of its launches, e.g. a split-K slab sum) from two ``rocprofv3 --pmc``
        runs (FETCH_SIZE, then WRITE_SIZE, CSV output), each scaled by what
        the same counter reads for the runtime's device-to-device copy of a
        known size (``bench.py --calib-copy``: 256 MiB read, 256 MiB written);
    python -m paper_1904_10585_amd.rocprof_summary product <results.db> --kernel NAME [--kernel NAME2]
        average duration of one launch of a kernel together with the kernels
        that complete it, from a ``rocprofv3 --kernel-trace`` database.

A completing kernel (NAME2, ...) is counted with the launch of NAME that it
directly follows in dispatch order (on the same queue): when the same
completing kernel also follows other products in the run (a slab sum shared
by several filter forms), only its dispatches after a NAME launch count.
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


def trace(db, steps, match=None):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
                       "from kernels group by name order by sum(duration) desc").fetchall()
    if match:
        rows = [r for r in rows if any(m in short_name(r[0]) for m in match)]
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


def attribute(seq, kernels):
    """Group a dispatch-ordered sequence of (queue, name, value) by launch of
    kernels[0]: each group holds that launch and the dispatches of
    kernels[1:] that directly follow it on its queue.  Returns, per kernel,
    the list of values attributed to it, and the number of groups."""
    first, rest = kernels[0], set(kernels[1:])
    per = {k: [] for k in kernels}
    open_q = {}                                   # queue -> a group is open
    groups = 0
    for queue, name, value in seq:
        if name == first:
            open_q[queue] = True
            groups += 1
            per[first].append(value)
        elif name in rest and open_q.get(queue):
            per[name].append(value)
        else:
            open_q[queue] = False
    return per, groups


def counter_seq(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(r["Queue_Id"], short_name(r["Kernel_Name"]), float(r["Counter_Value"])) for r in rows]


def bytes_per_dispatch(fetch_csv, write_csv, kernels):
    """HBM bytes per launch of the first kernel, with the dispatches of the
    other kernels given (e.g. the slab sum that completes a product) that
    directly follow each launch of it."""
    f = counter_means(fetch_csv)
    w = counter_means(write_csv)
    cf, nf = f[(CALIB_KERNEL, "FETCH_SIZE")]
    cw, nw = w[(CALIB_KERNEL, "WRITE_SIZE")]
    sf = cf * 1024 / CALIB_BYTES            # counter bytes per byte moved
    sw = cw * 1024 / CALIB_BYTES
    print(f"- calibration copy FETCH_SIZE per dispatch: {cf:.1f} KiB over {nf} dispatches (scale {sf:.5f})")
    print(f"- calibration copy WRITE_SIZE per dispatch: {cw:.1f} KiB over {nw} dispatches (scale {sw:.5f})")
    pf_, gf = attribute(counter_seq(fetch_csv, "FETCH_SIZE"), kernels)
    pw_, gw = attribute(counter_seq(write_csv, "WRITE_SIZE"), kernels)
    fetch_b = write_b = 0.0
    for kernel in kernels:
        vf, vw = pf_[kernel], pw_[kernel]
        if not vf or not vw:
            raise SystemExit(f"no dispatches of {kernel} after {kernels[0]}")
        print(f"- `{kernel}` FETCH_SIZE per dispatch: {sum(vf) / len(vf):.1f} KiB over {len(vf)} dispatches; "
              f"WRITE_SIZE {sum(vw) / len(vw):.1f} KiB over {len(vw)}")
        fetch_b += sum(vf) / gf * 1024 / sf
        write_b += sum(vw) / gw * 1024 / sw
    print(f"- launches of `{kernels[0]}`: {gf}")
    print(f"- fetch_bytes_per_launch: {fetch_b:.0f}")
    print(f"- write_bytes_per_launch: {write_b:.0f}")
    print(f"- traffic_bytes_per_launch: {fetch_b + write_b:.0f}")


def product(db, kernels):
    """Average duration of a launch of kernels[0] plus the completing
    kernels that directly follow it, and the average span from its start to
    the end of its last completing kernel (gaps included)."""
    con = sqlite3.connect(db)
    rows = con.execute("select queue_id, name, start, end from kernels order by start").fetchall()
    seq = [(q, short_name(n), (s, e)) for q, n, s, e in rows]
    per, groups = attribute(seq, kernels)
    total = 0.0
    for kernel in kernels:
        d = [e - s for s, e in per[kernel]]
        total += sum(d)
        print(f"- `{kernel}`: {len(d)} dispatches, average {sum(d) / max(len(d), 1) / 1e3:.2f} us")
    # spans: walk the same attribution again, keeping the first start and last end per group
    first, rest = kernels[0], set(kernels[1:])
    spans, cur, open_q = [], {}, {}
    for q, n, (s, e) in seq:
        if n == first:
            if q in cur:
                spans.append(cur[q][1] - cur[q][0])
            cur[q] = [s, e]
            open_q[q] = True
        elif n in rest and open_q.get(q):
            cur[q][1] = e
        else:
            open_q[q] = False
            if q in cur:
                spans.append(cur[q][1] - cur[q][0])
                del cur[q]
    spans += [v[1] - v[0] for v in cur.values()]
    print(f"- launches of `{first}`: {groups}")
    print(f"- product_avg_us (kernel durations summed): {total / max(groups, 1) / 1e3:.2f}")
    print(f"- product_span_avg_us (first start to last end): {sum(spans) / max(len(spans), 1) / 1e3:.2f}")


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
    t.add_argument("--match", action="append",
                   help="keep only kernels whose short name contains this text (repeatable)")
    b = sub.add_parser("bytes")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--kernel", required=True, action="append",
                   help="kernel name (repeat to add the kernels that complete one launch of the first)")
    pr = sub.add_parser("product")
    pr.add_argument("db")
    pr.add_argument("--kernel", required=True, action="append",
                    help="kernel name (repeat to add the kernels that complete one launch of the first)")
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    c.add_argument("--kernel", required=True)
    a = ap.parse_args()
    if a.cmd == "trace":
        trace(a.db, a.steps, a.match)
    elif a.cmd == "counters":
        counters(a.csv, a.kernel)
    elif a.cmd == "product":
        product(a.db, a.kernel)
    else:
        bytes_per_dispatch(a.fetch_csv, a.write_csv, a.kernel)


if __name__ == "__main__":
    main()
