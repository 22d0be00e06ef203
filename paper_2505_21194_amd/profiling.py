"""Summaries of rocprofv3 output for libseqcdc's kernels.

rocprofv3 writes its results as an SQLite database (``-o run`` gives
``run_results.db``).  This module turns such databases into the short text
and JSON summaries kept with the project:

* ``stats DB``: per-kernel dispatch count, total and average duration
  (from ``--kernel-trace``);
* ``traffic FETCH_DB WRITE_DB``: HBM bytes per dispatch of one kernel from
  two ``--pmc`` runs (``FETCH_SIZE`` and ``WRITE_SIZE``, reported in KiB per
  dispatch), scaled by what the same counters read for a plain copy kernel of
  known size in the same run;
* ``step FETCH_DB WRITE_DB``: the same for a whole chunking step, summed over
  every kernel the library launched in the run and divided by the number of
  steps the run made (each step launches the same kernels once);
* ``counters DB [DB ...]``: any other counters (one ``--pmc`` pass per
  database), summed per kernel of the step, per step and per unit of work
  (for instance per cut), as a short text table.

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
# kernels of a chunking step (the library's own; uploads and the caller's copies are not counted)
STEP_KERNELS = ("clear_kernel", "mark_kernel", "chains_kernel", "continue_kernel", "stitch_kernel", "compact_kernel")


def source_digest(paths=MARK_SOURCES):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(HERE, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# sources of a chunking step: its kernels, their launchers and the runtime that lays a call out (the autotuner,
# serving loop, dedup, calibration and graph capture only choose settings or run other work)
STEP_SOURCES = ("csrc/seqcdc_api.cpp", "csrc/seqcdc_device.h", "csrc/seqcdc_internal.h", "csrc/seqcdc_launch.h",
                "csrc/seqcdc_mark.h", "csrc/seqcdc_mark.hip", "csrc/seqcdc_resolve.hip", "csrc/seqcdc_runtime.h",
                "csrc/seqcdc_workspace.h")


def all_sources_digest():
    """Digest of the step's sources: a whole-step measurement holds while none of them changes."""
    return source_digest(STEP_SOURCES)


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


def step_traffic(fetch_db, write_db, steps, copy_kernel, copy_bytes):
    """HBM bytes of one chunking step: FETCH_SIZE and WRITE_SIZE summed over every dispatch of the step's
    kernels in each run, divided by `steps`, each counter scaled by the copy kernel's reading; per kernel too."""
    f = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    w = counter_per_dispatch(write_db, "WRITE_SIZE")

    def pick(d, name):
        for k, v in d.items():
            if name in k:
                return v
        raise KeyError("no dispatch of %s (have %s)" % (name, list(d)))

    # the calibration copies are the copy kernel's largest dispatches (small uploads and read-backs also run it)
    sf = copy_bytes / _median(sorted(pick(f, copy_kernel))[-5:])
    sw = copy_bytes / _median(sorted(pick(w, copy_kernel))[-5:])
    per = collections.OrderedDict()
    for k in STEP_KERNELS:
        fk = sum(f.get(k, [])) * sf / steps
        wk = sum(w.get(k, [])) * sw / steps
        if fk or wk:
            per[k] = {"fetch_bytes": fk, "write_bytes": wk, "dispatches_per_step": len(f.get(k, [])) / steps}
    tf = sum(v["fetch_bytes"] for v in per.values())
    tw = sum(v["write_bytes"] for v in per.values())
    return {"steps": steps, "fetch_bytes_per_step": tf, "write_bytes_per_step": tw, "bytes_per_step": tf + tw,
            "per_kernel": per, "calibration": {"copy_kernel": copy_kernel, "copy_bytes": copy_bytes,
                                               "fetch_scale": sf / 1024.0, "write_scale": sw / 1024.0}}


def counter_table(dbs, steps, units):
    """{kernel: {counter: value per step}} over the step's kernels, summed over each kernel's dispatches."""
    acc = collections.OrderedDict((k, collections.OrderedDict()) for k in STEP_KERNELS)
    for db in dbs:
        con = sqlite3.connect(db)
        rows = con.execute("select kernel_name, counter_name, sum(value) from counters_collection "
                           "group by kernel_name, counter_name").fetchall()
        for kn, cn, v in rows:
            k = short_name(kn)
            if k in acc:
                acc[k][cn] = acc[k].get(cn, 0.0) + float(v) / steps
    return {k: v for k, v in acc.items() if v}


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
    st = sub.add_parser("step")
    st.add_argument("fetch_db")
    st.add_argument("write_db")
    st.add_argument("--steps", type=int, required=True, help="chunking steps the profiled run made")
    st.add_argument("--workload", required=True)
    st.add_argument("--input-bytes", type=int, required=True)
    st.add_argument("--copy-kernel", default="copyBuffer")
    st.add_argument("--copy-bytes", type=float, required=True)
    st.add_argument("--cmd-fetch", default="")
    st.add_argument("--cmd-write", default="")
    st.add_argument("--out", required=True)
    cs = sub.add_parser("counters")
    cs.add_argument("dbs", nargs="+")
    cs.add_argument("--steps", type=int, required=True, help="chunking steps the profiled run made")
    cs.add_argument("--units", type=float, default=0, help="units of work per step (e.g. cuts) for per-unit columns")
    cs.add_argument("--unit-name", default="cut")
    cs.add_argument("--title", default="")
    cs.add_argument("--commands", nargs="*", default=[])
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        if a.title:
            print(a.title)
        for c in a.commands:
            print("command: " + c)
        print("per step%s; SQ_*CYCLES and SQ_WAIT_* count 4-cycle units" %
              (" and per %s (%d %ss per step)" % (a.unit_name, a.units, a.unit_name) if a.units else ""))
        for k, cnt in counter_table(a.dbs, a.steps, a.units).items():
            print(k)
            for cn, v in cnt.items():
                print("  %-24s %16.0f%s" % (cn, v, ("  %12.2f" % (v / a.units)) if a.units else ""))
    elif a.cmd == "stats":
        if a.title:
            print(a.title)
        if a.command:
            print("command: " + a.command)
        print("%-40s %8s %14s %12s" % ("kernel", "calls", "total_us", "avg_us"))
        rows = kernel_stats(a.db, a.by_grid)
        for k, c, tot, avg in rows[:a.top] if a.top else rows:
            print("%-40s %8d %14.1f %12.2f" % (k, c, tot / 1e3, avg / 1e3))
    elif a.cmd == "step":
        r = step_traffic(a.fetch_db, a.write_db, a.steps, a.copy_kernel, a.copy_bytes)
        r["workload"] = a.workload
        r["input_bytes"] = a.input_bytes
        r["bytes_per_input_byte"] = r["bytes_per_step"] / a.input_bytes
        r["source_sha256"] = all_sources_digest()
        r["commands"] = {"fetch": a.cmd_fetch, "write": a.cmd_write}
        with open(a.out, "w") as f:
            json.dump(r, f, indent=1)
        json.dump(r, sys.stdout, indent=1)
        print()
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
