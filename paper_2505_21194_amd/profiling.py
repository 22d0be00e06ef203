"""Summaries of rocprofv3 output for libseqcdc's kernels.

rocprofv3 writes its results as an SQLite database (``-o run`` gives
``run_results.db``).  This module turns such databases into the short text
and JSON summaries kept with the project:

* ``stats DB``: per-kernel dispatch count, total and average duration
  (from ``--kernel-trace``);
* ``traffic FETCH_DB WRITE_DB``: HBM bytes per dispatch of one kernel from
  two ``--pmc`` runs (``FETCH_SIZE`` and ``WRITE_SIZE``, reported in KiB per
  dispatch), scaled by what the same counters read for a plain copy kernel of
  known size in the same run.

Usage::

    python -m paper_2505_21194_amd.profiling stats run_results.db --command "..."
    python -m paper_2505_21194_amd.profiling traffic fetch.db write.db --kernel mark_kernel \\
        --copy-kernel elementwise --copy-bytes 1073741824 --cmd-fetch "..." --cmd-write "..." --out traffic.json
"""
import argparse
import collections
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# sources whose change invalidates a stored traffic measurement of the mark kernel
MARK_SOURCES = ("csrc/seqcdc_mark.h", "csrc/seqcdc_mark.hip", "csrc/seqcdc_device.h", "csrc/seqcdc_internal.h")


def source_digest(paths=MARK_SOURCES):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(HERE, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name):
    """Kernel name without namespace, template arguments and parameter list."""
    base = name.split("(")[0]
    base = base.split("<")[0]
    return base.split("::")[-1].strip()


def kernel_stats(db, by_grid=False):
    """[(kernel, calls, total_ns, avg_ns)], largest total first; by_grid keys kernels by their grid size too."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end, grid_x from kernels").fetchall()
    acc = collections.OrderedDict()
    for name, s, e, gx in rows:
        k = short_name(name) + ("[grid %d]" % gx if by_grid else "")
        c, t = acc.get(k, (0, 0))
        acc[k] = (c + 1, t + (e - s))
    return [(k, c, t, t / c) for k, (c, t) in sorted(acc.items(), key=lambda kv: -kv[1][1])]


def counter_per_dispatch(db, counter):
    """{short kernel name: [value per dispatch]} for one counter (summed over its instances)."""
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, sum(value) from counters_collection "
                       "where counter_name = ? group by dispatch_id order by dispatch_id", (counter,)).fetchall()
    out = collections.OrderedDict()
    for _, kn, v in rows:
        out.setdefault(short_name(kn), []).append(float(v))
    return out


def _median(xs):
    xs = sorted(xs)
    m = len(xs) // 2
    return xs[m] if len(xs) % 2 else 0.5 * (xs[m - 1] + xs[m])


def traffic(fetch_db, write_db, kernel, copy_kernel, copy_bytes):
    """Bytes per dispatch of `kernel`, each counter scaled so that the copy kernel reads / writes copy_bytes."""
    f = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    w = counter_per_dispatch(write_db, "WRITE_SIZE")

    def pick(d, name):
        for k, v in d.items():
            if name in k:
                return v
        raise KeyError("no dispatch of %s (have %s)" % (name, list(d)))

    cf, cw = _median(pick(f, copy_kernel)), _median(pick(w, copy_kernel))
    kf, kw = _median(pick(f, kernel)), _median(pick(w, kernel))
    sf, sw = copy_bytes / cf, copy_bytes / cw  # bytes per counter unit
    return {"kernel": kernel, "fetch_bytes_per_launch": kf * sf, "write_bytes_per_launch": kw * sw,
            "bytes_per_launch": kf * sf + kw * sw,
            "raw": {"kernel_fetch_kib": kf, "kernel_write_kib": kw, "copy_fetch_kib": cf, "copy_write_kib": cw},
            "calibration": {"copy_kernel": copy_kernel, "copy_bytes": copy_bytes,
                            "fetch_scale": sf / 1024.0, "write_scale": sw / 1024.0}}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--command", default="")
    s.add_argument("--title", default="")
    s.add_argument("--by-grid", action="store_true", help="separate launches of one kernel by grid size")
    s.add_argument("--top", type=int, default=0, help="print only the first N rows")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--kernel", default="mark_kernel")
    t.add_argument("--copy-kernel", default="elementwise")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--n", type=int, default=0, help="input bytes per launch of the kernel")
    t.add_argument("--cmd-fetch", default="")
    t.add_argument("--cmd-write", default="")
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        if a.title:
            print(a.title)
        if a.command:
            print("command: " + a.command)
        print("%-40s %8s %14s %12s" % ("kernel", "calls", "total_us", "avg_us"))
        rows = kernel_stats(a.db, a.by_grid)
        for k, c, tot, avg in rows[:a.top] if a.top else rows:
            print("%-40s %8d %14.1f %12.2f" % (k, c, tot / 1e3, avg / 1e3))
    else:
        r = traffic(a.fetch_db, a.write_db, a.kernel, a.copy_kernel, a.copy_bytes)
        r["n"] = a.n
        r["source_sha256"] = source_digest()
        r["commands"] = {"fetch": a.cmd_fetch, "write": a.cmd_write}
        with open(a.out, "w") as f:
            json.dump(r, f, indent=1)
        json.dump(r, sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
