"""Chunking throughput of SeqCDC on one MI355X.

Workload of a step (the whole hot path over one batch of synthetic input):
  plain:   one 1 GiB backup-like mixed stream (1 MiB blocks: 50% uniform bytes, 30% Zipf(1.1) text over 64
           printable symbols, 20% zero / repeated-16-byte runs), Increasing mode, 8 KiB target average (Table I:
           SeqLength 5, SkipTrigger 50, SkipSize 256; min 4 KiB, max 16 KiB).  The stream is resident in HBM when
           the timed region starts; a step is one seqcdc_chunk call (mark, pass A chains, pass B continuations,
           stitch, compaction, count read-back).
Reported beside it (not the headline value):
  batched: 4096 files, log-normal sizes (median 256 KiB, sigma 1.5, clamped 4 KiB..64 MiB), each a mixed stream
           under its own seed, 16 KiB average (SeqLength 5, 50 / 512, min 8 KiB, max 32 KiB): one
           seqcdc_chunk_batch call per step, against one seqcdc_chunk call per file.
  serving: Poisson arrivals of requests (log-normal sizes, median 1 MiB, sigma 1.5, clamped 1 KiB..256 MiB) that
           are slices of a device-resident snapshot series, 8 and 32 KiB averages mixed; offered load at 10/40/80 %
           of the server's saturated rate; p50/p99 latency and GB/s, against the plain per-request path.
  sweep:   the other plain variants (both modes at 8 / 16 / 32 KiB averages and SeqLength 6 on the 1 GiB stream;
           8 MiB of uniform bytes at 8 KiB with max 16 and 64 KiB).
Settings (segment length, mark span, chain occupancy, resolve mode) come from the library's autotuner, run
untimed on each workload first (--no-tune: defaults).
value = plain input bytes per second (GB/s = 1e9 B/s).
"""
import argparse
import ctypes
import json
import os
import sys
import threading
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
METRIC = "chunking GB/s on 1 MI355X (batched vs plain) + % HBM peak; p99 request latency"
RUN7 = np.array([10, 20, 30, 40, 50, 5, 3], np.uint8)  # a 7-byte pattern holding a run of 5 increasing bytes
PROBE_STEPS = 6  # chunking steps of a whole-step traffic probe (each launches the step's kernels once)
STEP_TRAFFIC = {"plain": os.path.join(HERE, "profiles", "step_traffic_plain1GiB.json"),
                "batched": os.path.join(HERE, "profiles", "step_traffic_batched4096.json"),
                "batched_direct": os.path.join(HERE, "profiles", "step_traffic_batched4096_direct.json")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size-mib", type=int, default=1024)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the other plain variants")
    ap.add_argument("--no-dedup", action="store_true", help="skip the snapshot-series dedup leg")
    ap.add_argument("--no-calib", action="store_true", help="skip the calibration leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the library's autotuner (default settings)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="oracle work to time on the host")
    ap.add_argument("--traffic-probe", choices=["mark", "plain", "batched"], default=None,
                    help="for rocprofv3 --pmc runs: a 1 GiB device copy (the calibration kernel), then only the mark "
                         "kernel, or PROBE_STEPS whole plain or batched steps (default settings, no autotuning)")
    ap.add_argument("--mode", type=int, default=None, help="resolve mode of the probe's plan (0 marked, 1 direct)")
    ap.add_argument("--traffic-json", default=os.path.join(HERE, "profiles", "mark_traffic.json"))
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def mark_roofline(n, kernel_ms, traffic_json):
    """Roofline of the mark kernel from its average duration inside the chunking calls (HIP events around its
    launch on the call's stream) and, when they match the current sources, the PMC bytes per launch."""
    groups = (n + 63) // 64
    ms = kernel_ms
    # algorithmic bytes of one launch: read every input byte, write 2 bits per byte (EO16) and one summary
    # byte per 1 KiB block
    alg = n + 16 * groups + (n + 1023) // 1024
    achieved = alg / (ms * 1e-3) / 1e9
    traffic = None
    try:
        from paper_2505_21194_amd import profiling
        t = json.load(open(traffic_json))
        if t.get("source_sha256") == profiling.source_digest() and t.get("n") == n:
            traffic = round(t["bytes_per_launch"])
    except Exception:
        traffic = None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "mark_kernel",
            "kernel_ms": round(ms, 4), "alg_bytes_per_launch": alg}


def stored_step_traffic(key):
    """HBM bytes per step from the committed whole-step counter summary, if it was taken on the current sources."""
    try:
        from paper_2505_21194_amd import profiling
        t = json.load(open(STEP_TRAFFIC[key]))
        if t.get("source_sha256") == profiling.all_sources_digest():
            return round(t["bytes_per_step"])
    except Exception:
        pass
    return None


def step_roofline(alg_bytes, ms, traffic):
    """Roofline of a whole step: algorithmic bytes and (when measured on these sources) counter bytes per step, over
    the step's time."""
    out = {"bound": "hbm", "alg_bytes": int(alg_bytes), "achieved": round(alg_bytes / (ms * 1e-3) / 1e9, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "traffic": traffic}
    if traffic:
        out["traffic_frac"] = round(traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def mark_alg_bytes(n):
    """Algorithmic bytes of marking n bytes: read every byte, write 2 bits per byte (EO16) and one summary byte per
    1 KiB block."""
    return n + 16 * ((n + 63) // 64) + (n + 1023) // 1024


def batch_workload(seq, torch, dev):
    """The 4096-file batch: device bytes, sizes, parameters, output arrays and marshalled tables."""
    import synth
    nfiles = 4096
    sizes = synth.lognormal_sizes(nfiles, 256 * 1024, 1.5, 4096, 64 << 20, seed=4).astype(np.int64)
    total = int(sizes.sum())
    log("batched: %d files, %.2f GiB" % (nfiles, total / 2 ** 30))
    offs = np.concatenate([[0], np.cumsum(sizes)])
    host = np.empty(total, dtype=np.uint8)
    for f in range(nfiles):
        host[int(offs[f]):int(offs[f + 1])] = synth.mixed(int(sizes[f]), seed=100000 + f)
    buf = torch.from_numpy(host).to(dev)  # one upload
    del host
    pb = seq.seqcdc_params_for_avg(16384)
    cut_offs = [0]
    for s in sizes:
        cut_offs.append(cut_offs[-1] + seq.seqcdc_max_cuts(int(s), pb))
    bcuts = torch.empty(cut_offs[-1], dtype=torch.int64, device=dev)
    bcounts = torch.empty(nfiles, dtype=torch.int64, device=dev)
    files = [(buf.data_ptr() + int(offs[f]), int(sizes[f]), 0) for f in range(nfiles)]
    ftab = seq.file_table([f[0] for f in files], sizes)  # marshalled once, like a caller's own table
    otab = seq.offsets_table(cut_offs)
    return buf, sizes, total, pb, cut_offs, bcuts, bcounts, files, ftab, otab


def pipelined_batches(seq, torch, stream, plan, ftab, pb, otab, bcuts, bcounts, total, steps, warmup, in_flight=3):
    """The batch with `in_flight` calls in flight: the given plan on `stream` and further plans on streams of their
    own (default priority), each tuned for the batch and writing its own outputs, the calls taking turns.  Rate =
    batches x bytes over the time of in_flight*steps calls; every output set is compared with the eager call's
    afterwards."""
    torch.cuda.synchronize()
    want_cuts, want_counts = bcuts.cpu().numpy(), bcounts.cpu().numpy()
    lanes = [(plan, stream, bcuts, bcounts)]
    extra = []
    try:
        for _ in range(in_flight - 1):
            st = torch.cuda.Stream()
            pl = seq.seqcdc_plan_create()
            extra.append(pl)
            c, n = torch.empty_like(bcuts), torch.empty_like(bcounts)
            seq.seqcdc_autotune_batch(pl, ftab, [pb], c.data_ptr(), otab, n.data_ptr(), stream=st)
            lanes.append((pl, st, c, n))
        torch.cuda.synchronize()

        def call(i):
            pl, st, c, n = lanes[i % in_flight]
            seq.seqcdc_chunk_batch(ftab, [pb], c.data_ptr(), otab, n.data_ptr(), stream=st, plan=pl)
        for i in range(in_flight * warmup):
            call(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(in_flight * steps):
            call(i)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / (in_flight * steps)
        same = all(bool(np.array_equal(c.cpu().numpy(), want_cuts) and np.array_equal(n.cpu().numpy(), want_counts))
                   for _, _, c, n in lanes)
    finally:
        for pl in extra:
            seq.seqcdc_plan_destroy(pl)
    traffic = stored_step_traffic("batched")
    out = {"in_flight": in_flight, "ms_per_batch": round(dt * 1e3, 3), "GBps": round(total / dt / 1e9, 1),
           "outputs_match": same}
    if traffic:  # counter bytes of one batch step over the time per batch
        out["traffic_frac"] = round(traffic / dt / 1e9 / HBM_PEAK_GBS, 4)
    return out


def batched(seq, torch, stream, plan, steps, warmup, dev, tune):
    nfiles = 4096
    buf, sizes, total, pb, cut_offs, bcuts, bcounts, files, ftab, otab = batch_workload(seq, torch, dev)

    def bstep():
        seq.seqcdc_chunk_batch(ftab, [pb], bcuts.data_ptr(), otab, bcounts.data_ptr(), stream=stream, plan=plan)

    tuning = None
    if tune:  # the library's batch autotuner on this batch (untimed): it sets the plan's settings
        seq.seqcdc_autotune_batch(plan, ftab, [pb], bcuts.data_ptr(), otab, bcounts.data_ptr(), stream=stream)
        seg, span, waves = seq.seqcdc_plan_get_tuning(plan, total, pb)
        tuning = {"segment_bytes": seg, "mark_span_blocks": span, "waves_per_cu": waves}
        log("batched tuning: %s" % tuning)

    for _ in range(warmup):
        bstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bstep()
    torch.cuda.synchronize()
    bdt = (time.perf_counter() - t0) / steps
    counts = bcounts.cpu().numpy()
    # the same batch prepared once and replayed as a hipGraph
    gb = seq.seqcdc_batch_prepare(ftab, [pb], bcuts.data_ptr(), otab, bcounts.data_ptr(), settings=plan)
    try:
        for _ in range(warmup):
            seq.seqcdc_batch_launch(gb, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            seq.seqcdc_batch_launch(gb, stream=stream)
        torch.cuda.synchronize()
        gdt = (time.perf_counter() - t0) / steps
        graph_same = bool(np.array_equal(bcounts.cpu().numpy(), counts))
    finally:
        seq.seqcdc_batch_destroy(gb)
    # three batches in flight: two more plans (tuned the same way) on streams of their own with their own outputs,
    # the calls taking turns, so one batch's resolve overlaps the next ones' marking
    pipelined = pipelined_batches(seq, torch, stream, plan, ftab, pb, otab, bcuts, bcounts, total, steps, warmup)
    # one plain launch per file, the same files and parameters
    pcap = max(cut_offs[i + 1] - cut_offs[i] for i in range(nfiles))
    for f in range(16):
        seq.seqcdc_chunk(files[f][0], files[f][1], pb, bcuts.data_ptr(), pcap, stream=stream, plan=plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(nfiles):
        seq.seqcdc_chunk(files[f][0], files[f][1], pb, bcuts.data_ptr(), pcap, stream=stream, plan=plan)
    torch.cuda.synchronize()
    pdt = time.perf_counter() - t0
    # the same batch in the direct (skip-aware) resolve mode: no mark kernel, chains read only the windows they scan
    dplan = seq.seqcdc_plan_create()
    seq.seqcdc_plan_set_mode(dplan, 1)
    try:
        def dstep():
            seq.seqcdc_chunk_batch(ftab, [pb], bcuts.data_ptr(), otab, bcounts.data_ptr(), stream=stream, plan=dplan)
        for _ in range(warmup):
            dstep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dstep()
        torch.cuda.synchronize()
        ddt = (time.perf_counter() - t0) / steps
        dsame = bool(np.array_equal(bcounts.cpu().numpy(), counts))
    finally:
        seq.seqcdc_plan_destroy(dplan)
    dtraffic = stored_step_traffic("batched_direct")
    direct = {"ms_per_step": round(ddt * 1e3, 3), "GBps": round(total / ddt / 1e9, 1), "counts_match": dsame,
              "traffic": dtraffic,
              "traffic_per_input_byte": round(dtraffic / total, 4) if dtraffic else None}
    # whole-step roofline: the two-phase design's algorithmic bytes (marking every byte, writing the cuts) over
    # the step time; traffic = the counter bytes of every kernel of a step
    alg = sum(mark_alg_bytes(int(x)) for x in sizes) + 8 * int(counts.sum())
    roof = step_roofline(alg, bdt * 1e3, stored_step_traffic("batched"))
    del buf, bcuts
    return {"files": nfiles, "bytes": total, "cuts": int(counts.sum()), "ms_per_step": round(bdt * 1e3, 3),
            "GBps": round(total / bdt / 1e9, 1), "frac_hbm_peak_input": round(total / bdt / 1e9 / HBM_PEAK_GBS, 4),
            "roofline": roof, "direct": direct, "pipelined": pipelined,
            "graph_ms_per_step": round(gdt * 1e3, 3), "graph_GBps": round(total / gdt / 1e9, 1),
            "graph_counts_match": graph_same,
            "per_file_launch_GBps": round(total / pdt / 1e9, 2), "speedup_vs_per_file": round(pdt / bdt, 2),
            "params": "avg 16 KiB: SeqLength 5, SkipTrigger 50, SkipSize 512, min 8 KiB, max 32 KiB",
            "tuning": tuning, "counts": counts}


def serving(seq, torch, dev, streams=2, max_batch=512):
    """Poisson request stream through the serving loop; returns latency percentiles per offered load.  A run's rate is
    its bytes over the time from its first submission to its last result (each request's completion = its submission
    time on the host + the latency the library measured), so the Python loop that collects results is not timed."""
    import synth
    vers = synth.snapshot_series(256 << 20, 3, seed=11, nedits=200, maxlen=4096)
    dvers = [torch.from_numpy(v).to(dev) for v in vers]
    rng = np.random.default_rng(5)
    params = [seq.seqcdc_params_for_avg(8192), seq.seqcdc_params_for_avg(32768)]
    nreq = 400
    sizes = synth.lognormal_sizes(nreq, 1 << 20, 1.5, 1024, 256 << 20, seed=12).astype(np.int64)
    reqs = []
    meta = []  # (version, offset, length, params index) of each request
    for i in range(nreq):
        v = int(rng.integers(len(vers)))
        n = int(min(sizes[i], vers[v].size))
        off = int(rng.integers(vers[v].size - n + 1))
        reqs.append((dvers[v].data_ptr() + off, n, i % 2))
        meta.append((v, off, n, i % 2))
    total = sum(r[1] for r in reqs)
    arr = (seq.seqcdc_params * 2)(*params)
    cfg = seq.seqcdc_server_config(0, 4 << 30, 1024, streams, max_batch, 2, arr)
    h = ctypes.c_void_p()
    if seq.lib.seqcdc_server_create(ctypes.byref(cfg), ctypes.byref(h)):
        raise RuntimeError(seq.last_error())

    def timeline(npasses):
        """Summary of the last npasses pass records: host layout, device time, waits, workspace growth."""
        recs = seq.seqcdc_server_timeline(h)[-npasses:] if npasses else []
        if not recs:
            return None
        g = np.array([r["gpu_ms"] for r in recs])
        return {"passes": len(recs), "requests_per_pass": round(float(np.mean([r["requests"] for r in recs])), 1),
                "gpu_ms_sum": round(float(g.sum()), 3), "gpu_ms_max": round(float(g.max()), 3),
                "layout_ms_mean": round(float(np.mean([r["layout_ms"] for r in recs])), 3),
                "wait_ms_mean": round(float(np.mean([r["wait_ms"] for r in recs])), 3),
                "retire_ms_mean": round(float(np.mean([r["retire_ms"] for r in recs])), 3),
                "grew": int(sum(r["grew"] for r in recs))}

    def passes():
        v = ctypes.c_uint64()
        if seq.lib.seqcdc_server_stats(h, None, ctypes.byref(v), None, None):
            raise RuntimeError(seq.last_error())
        return v.value

    kept = {}

    ftab = seq.file_table([r[0] for r in reqs], [r[1] for r in reqs], [r[2] for r in reqs])

    def run(rate_gbs, keep=False):
        """Submit reqs at Poisson arrival times for an offered load (GB/s); None = all at once.  The library queues
        them (seqcdc_server_submit_many), so the offered rate is not limited by a Python loop.  keep: copy each
        request's cuts for the parity check made after every measurement."""
        p0 = passes()
        at_ms = None
        if rate_gbs:
            mean = total / nreq
            at_ms = np.cumsum(rng.exponential(mean / (rate_gbs * 1e9), nreq)) * 1e3
        tickets, t_sub = seq.seqcdc_server_submit_many(h, ftab, at_ms)
        lat = []
        for i, t in enumerate(tickets):
            res = seq.seqcdc_result()
            if seq.lib.seqcdc_server_wait(h, int(t), 60000.0, ctypes.byref(res)):
                raise RuntimeError(seq.last_error())
            lat.append(res.latency_ms)
            if keep:
                kept[i] = np.ctypeslib.as_array(res.cuts, shape=(res.count,)).copy() if res.count else \
                    np.zeros(0, np.uint64)
            seq.lib.seqcdc_server_release(h, int(t))
        lat = np.array(lat)
        dt = float(np.max(t_sub + lat)) * 1e-3  # first submission -> last result (the call starts at 0)
        np_ = passes() - p0
        return {"offered_GBps": round(rate_gbs, 2) if rate_gbs else None, "GBps": round(total / dt / 1e9, 2),
                "submit_lag_ms_max": round(float(np.max(t_sub - at_ms)), 3) if at_ms is not None else None,
                "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "passes": np_, "timeline": timeline(np_)}

    try:
        for _ in range(3):  # warm-up: the passes' buffers grow to the largest batches they meet
            run(None)
        sat = run(None)
        peak = sat["GBps"]
        loads = [run(frac * peak) for frac in (0.1, 0.4, 0.8)]
        run(None, keep=True)  # the results checked against the oracle after every measurement (untimed)
    finally:
        seq.lib.seqcdc_server_destroy(h)
    # plain per-request path: one seqcdc_chunk call per request, back to back
    cap = max(seq.seqcdc_max_cuts(n, params[pi]) for _, n, pi in reqs)
    cuts = torch.empty(cap, dtype=torch.int64, device=dev)
    plan = seq.seqcdc_plan_create()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ptr, n, pi in reqs:
        t1 = time.perf_counter()
        seq.seqcdc_chunk(ptr, n, params[pi], cuts.data_ptr(), cap, plan=plan)
        lat.append((time.perf_counter() - t1) * 1e3)
    dt = time.perf_counter() - t0
    seq.seqcdc_plan_destroy(plan)
    # for the parity check: each request's bytes (version, offset, length) and parameters
    checks = {"versions": vers, "reqs": meta, "params": params, "got": kept}
    return {"requests": nreq, "bytes": total, "config": {"streams": streams, "max_batch": max_batch, "ring_slots": 1024,
                                                          "budget_bytes": 4 << 30},
            "saturated": sat, "loads": loads, "_checks": checks,
            "plain_per_request": {"GBps": round(total / dt / 1e9, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                                  "p99_ms": round(float(np.percentile(lat, 99)), 3)}}


def sweep(seq, torch, stream, d, steps, tune):
    """GPU rate of the other plain variants: the 1 GiB mixed stream in both modes at 8 / 16 / 32 KiB averages
    (Table I) and at SeqLength 6, and the 8 MiB uniform buffer of seed 0 at 8 KiB with max 16 and 64 KiB."""
    import synth
    out = []
    small = torch.from_numpy(synth.uniform(8 << 20, seed=0)).to(d.device)
    cases = []
    for avg in (8, 16, 32):
        for mode in (0, 1):
            p = seq.seqcdc_params_for_avg(avg << 10)
            p.mode = mode
            cases.append(("1 GiB mixed, %s, avg %d KiB" % ("increasing" if mode == 0 else "decreasing", avg), d, p))
    p6 = seq.seqcdc_params_for_avg(8192)
    p6.seq_length = 6
    cases.append(("1 GiB mixed, increasing, avg 8 KiB parameters with SeqLength 6", d, p6))
    cases.append(("8 MiB uniform (seed 0), increasing, avg 8 KiB, max 16 KiB", small, seq.seqcdc_params_for_avg(8192)))
    # the worst case for speculation: a 7-byte pattern holding an increasing run of 5, repeated: every chunk ends
    # just past a run at the same phase of the pattern, chunk lengths (4096 or 4101 bytes) do not divide the segment
    # length, and chains from different starts never meet, so the exact path is one sequential walk
    p7 = torch.from_numpy(np.resize(RUN7, d.numel())).to(d.device)
    cases.append(("1 GiB periodic 7-byte pattern with a run (never resynchronises), increasing, avg 8 KiB", p7,
                  seq.seqcdc_params_for_avg(8192)))
    p64 = seq.seqcdc_params_for_avg(8192)
    p64.max_size = 65536
    cases.append(("8 MiB uniform (seed 0), increasing, avg 8 KiB, max 64 KiB", small, p64))
    plan = seq.seqcdc_plan_create()
    try:
        for name, t, p in cases:
            n = t.numel()
            cap = seq.seqcdc_max_cuts(n, p)
            cuts = torch.empty(cap, dtype=torch.int64, device=t.device)
            worst = "periodic" in name
            if tune and n >= (64 << 20) and not worst:
                seq.seqcdc_autotune(plan, t.data_ptr(), n, p, stream=stream)
            reps = 2 if worst else steps  # the sequential walk takes a few hundred ms
            for _ in range(1 if worst else 2):
                cnt = seq.seqcdc_chunk(t.data_ptr(), n, p, cuts.data_ptr(), cap, stream=stream, plan=plan)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                cnt = seq.seqcdc_chunk(t.data_ptr(), n, p, cuts.data_ptr(), cap, stream=stream, plan=plan)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            seg, span, waves = seq.seqcdc_plan_get_tuning(plan, n, p)
            out.append({"workload": name, "ms": round(dt * 1e3, 4), "GBps": round(n / dt / 1e9, 1), "cuts": cnt,
                        "tuning": {"segment_bytes": seg, "mark_span_blocks": span, "waves_per_cu": waves}})
            if "periodic" in name:  # its cuts, for the oracle check made after every measurement
                out[-1]["_check"] = (cuts[:cnt].cpu().numpy().astype(np.uint64), p)
            del cuts
    finally:
        seq.seqcdc_plan_destroy(plan)
    return out


def cpu_batched(seq, gpu_counts):
    """Context for the batch: the oracle over the same files (regenerated from their seeds) on the host's cores,
    one file per thread at a time; run after every GPU measurement."""
    import oracle
    import synth
    from concurrent.futures import ThreadPoolExecutor
    nfiles = len(gpu_counts)
    sizes = synth.lognormal_sizes(nfiles, 256 * 1024, 1.5, 4096, 64 << 20, seed=4).astype(np.int64)
    host = [synth.mixed(int(sizes[f]), seed=100000 + f) for f in range(nfiles)]
    pb = seq.seqcdc_params_for_avg(16384)
    kw = dict(mode=pb.mode, seq_length=pb.seq_length, min_size=pb.min_size, max_size=pb.max_size,
              skip_trigger=pb.skip_trigger, skip_size=pb.skip_size)
    cores = min(16, len(os.sched_getaffinity(0)))
    order = sorted(range(nfiles), key=lambda f: -host[f].size)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        counts = dict(zip(order, ex.map(lambda f: oracle.chunk(host[f], **kw).size, order)))
    dt = time.perf_counter() - t0
    return {"value": round(int(sizes.sum()) / dt / 1e9, 2), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": "the whole batch, one file per thread (context, not the baseline)",
            "counts_match": bool(all(counts[f] == int(gpu_counts[f]) for f in range(nfiles)))}


def dedup_leg(seq, torch, stream, steps, warmup, dev):
    """Config 3: a 256 MiB uniform base and 9 versions of 200 seeded edits, chunked by the batched path at 8 KiB and
    deduplicated on the device (SHA-256 per chunk, fingerprint table, byte compare); both timed per step."""
    import synth
    vers = synth.snapshot_series(256 << 20, 10, seed=0, nedits=200, maxlen=4096)
    total = sum(v.size for v in vers)
    log("dedup: %d versions, %.2f GiB" % (len(vers), total / 2 ** 30))
    devs = [torch.from_numpy(v).to(dev) for v in vers]
    p = seq.seqcdc_params_for_avg(8192)
    offs = [0]
    for v in vers:
        offs.append(offs[-1] + seq.seqcdc_max_cuts(v.size, p))
    d_cuts = torch.zeros(offs[-1], dtype=torch.int64, device=dev)
    d_counts = torch.zeros(len(vers), dtype=torch.int64, device=dev)
    ftab = seq.file_table([d.data_ptr() for d in devs], [d.numel() for d in devs])
    otab = seq.offsets_table(offs)
    plan = seq.seqcdc_plan_create()
    try:
        def chunk():
            seq.seqcdc_chunk_batch(ftab, [p], d_cuts.data_ptr(), otab, d_counts.data_ptr(), stream=stream, plan=plan)

        def dedup():
            return seq.seqcdc_dedup_batch(plan, ftab, d_cuts.data_ptr(), otab, d_counts.data_ptr(), stream=stream)

        for _ in range(warmup):
            chunk()
            res = dedup()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            chunk()
        torch.cuda.synchronize()
        cdt = (time.perf_counter() - t0) / steps
        t0 = time.perf_counter()
        for _ in range(steps):
            res = dedup()
        ddt = (time.perf_counter() - t0) / steps
        counts = d_counts.cpu().numpy()
        allc = d_cuts.cpu().numpy().astype(np.uint64)
    finally:
        seq.seqcdc_plan_destroy(plan)
    cuts = [allc[offs[i]:offs[i] + int(counts[i])] for i in range(len(vers))]
    orig, uniq = res
    return {"versions": len(vers), "bytes": total, "chunks": int(counts.sum()), "chunk_ms": round(cdt * 1e3, 3),
            "chunk_GBps": round(total / cdt / 1e9, 1), "dedup_ms": round(ddt * 1e3, 3),
            "dedup_GBps": round(total / ddt / 1e9, 1), "orig_bytes": orig, "unique_bytes": uniq,
            "savings": round((orig - uniq) / orig, 6), "_check": (vers, cuts, p)}


def calibration_leg(seq, torch, stream, dev):
    """Monte-Carlo calibration (Sec. V) on 256 MiB of uniform bytes: a grid of 70 candidates (SeqLength 5 and 6 x 7
    triggers x 5 skip sizes, min = 4 KiB, max = 16 KiB) for an 8 KiB target in one call, and the Table I parameter
    sets at 4 / 8 / 16 KiB for both SeqLength readings."""
    import synth
    n = 256 << 20
    d = torch.from_numpy(synth.uniform(n, seed=29)).to(dev)
    plan = seq.seqcdc_plan_create()
    try:
        seq.calibrate_for_avg(plan, d.data_ptr(), n, 8192, stream=stream)  # warm-up (workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        best, st, grid = seq.calibrate_for_avg(plan, d.data_ptr(), n, 8192, stream=stream)
        dt = time.perf_counter() - t0
        rows = [(4096, 1024, 55, 256), (8192, 4096, 50, 256), (16384, 8192, 50, 512)]
        table1 = {}
        for sl in (5, 6):
            cands = [dict(mode=0, seq_length=sl, min_size=mn, max_size=2 * avg, skip_trigger=t, skip_size=k)
                     for avg, mn, t, k in rows]
            table1["seq_length_%d" % sl] = [round(x["mean"], 1) for x in seq.seqcdc_calibrate(plan, d.data_ptr(), n,
                                                                                               cands, stream=stream)]
    finally:
        seq.seqcdc_plan_destroy(plan)
    return {"sample_bytes": n, "candidates": len(grid), "ms": round(dt * 1e3, 3),
            "GBps": round(len(grid) * n / dt / 1e9, 1),
            "best_for_8KiB": {"seq_length": best.seq_length, "skip_trigger": best.skip_trigger,
                              "skip_size": best.skip_size, "mean": round(st["mean"], 1),
                              "max_share": round(st["max_chunks"] / max(st["chunks"], 1), 4)},
            "table1_means_4_8_16KiB": table1}


def dedup_parity(check, orig, uniq):
    """The oracle's chunking and Eq. 1 over the same series (host side, after the GPU measurements)."""
    import oracle
    vers, cuts, p = check
    kw = dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
              skip_trigger=p.skip_trigger, skip_size=p.skip_size)
    want = [oracle.chunk(v, **kw) for v in vers]
    same_cuts = all(np.array_equal(a, b) for a, b in zip(cuts, want))
    o2, u2, _, _ = oracle.dedup_stats(vers, want)
    return bool(same_cuts and (orig, uniq) == (o2, u2))


def serving_parity(checks):
    """Every request of the saturated serving run against the oracle on its own bytes (host side, after the GPU
    measurements)."""
    import oracle
    ok = True
    for i, (vi, off, n, pi) in enumerate(checks["reqs"]):
        p = checks["params"][pi]
        want = oracle.chunk(checks["versions"][vi][off:off + n], mode=p.mode, seq_length=p.seq_length,
                            min_size=p.min_size, max_size=p.max_size, skip_trigger=p.skip_trigger,
                            skip_size=p.skip_size)
        got = checks["got"].get(i)
        ok = ok and got is not None and got.size == want.size and bool(np.array_equal(got, want))
    return ok


def oracle_chunk(data, p):
    import oracle
    return oracle.chunk(data, mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
                        skip_trigger=p.skip_trigger, skip_size=p.skip_size)


def cpu_baseline(host, p, seconds):
    """The oracle, single-threaded, over whole passes of the same stream until `seconds` of work."""
    import oracle
    kw = dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
              skip_trigger=p.skip_trigger, skip_size=p.skip_size)
    t0 = time.perf_counter()
    cuts = oracle.chunk(host, **kw)
    one = time.perf_counter() - t0
    reps = max(1, int(seconds / max(one, 1e-3)) - 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.chunk(host, **kw)
    dt = (time.perf_counter() - t0 + one) / (reps + 1)
    return cuts, {"value": round(host.size / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
                  "sample": "the whole %d MiB stream, %d passes, one thread" % (host.size >> 20, reps + 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2505_21194_amd as seq
    import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    n = args.size_mib << 20
    log("generating %d MiB mixed stream" % args.size_mib)
    host = synth.mixed(n, seed=2)
    d = torch.from_numpy(host).to(dev)
    p = seq.seqcdc_params_for_avg(8192)

    if args.traffic_probe:
        dst = torch.empty_like(d)
        for _ in range(5):
            dst.copy_(d)  # plain 1 GiB device copy: the calibration kernel
        del dst
        if args.traffic_probe == "mark":
            groups = (n + 63) // 64
            eo = torch.empty(4 * groups, dtype=torch.int32, device=dev)
            for _ in range(5):
                seq.seqcdc_mark(d.data_ptr(), n, p, eo.data_ptr(), stream=stream)
        else:
            plan = seq.seqcdc_plan_create()
            if args.mode is not None:
                seq.seqcdc_plan_set_mode(plan, args.mode)
            if args.traffic_probe == "plain":
                cap = seq.seqcdc_max_cuts(n, p)
                cuts = torch.empty(cap, dtype=torch.int64, device=dev)
                for _ in range(PROBE_STEPS):
                    seq.seqcdc_chunk(d.data_ptr(), n, p, cuts.data_ptr(), cap, stream=stream, plan=plan)
            else:
                del d
                buf, sizes, total, pb, cut_offs, bcuts, bcounts, files, ftab, otab = batch_workload(seq, torch, dev)
                for _ in range(PROBE_STEPS):
                    seq.seqcdc_chunk_batch(ftab, [pb], bcuts.data_ptr(), otab, bcounts.data_ptr(), stream=stream,
                                           plan=plan)
                log("probe input bytes: %d" % total)
            torch.cuda.synchronize()
            seq.seqcdc_plan_destroy(plan)
        torch.cuda.synchronize()
        log("traffic probe done: %s, %d steps" % (args.traffic_probe, PROBE_STEPS))
        return

    cap = seq.seqcdc_max_cuts(n, p)
    cuts = torch.empty(cap, dtype=torch.int64, device=dev)
    plan = seq.seqcdc_plan_create()
    torch.cuda.synchronize()
    tuning = None
    if not args.no_tune:  # the library's autotuner, on the stream itself (untimed)
        seq.seqcdc_autotune(plan, d.data_ptr(), n, p, stream=stream)
        seg, span, waves = seq.seqcdc_plan_get_tuning(plan, n, p)
        tuning = {"segment_bytes": seg, "mark_span_blocks": span, "waves_per_cu": waves}
        log("plain tuning: %s" % tuning)

    def step():
        return seq.seqcdc_chunk(d.data_ptr(), n, p, cuts.data_ptr(), cap, stream=stream, plan=plan)

    for _ in range(args.warmup):
        count = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        count = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    value = n / dt / 1e9
    log("plain: %.3f ms/step, %.1f GB/s, %d cuts" % (dt * 1e3, value, count))

    # per-phase durations of as many more calls: HIP events recorded by the library on the call's stream between
    # its launches (the mark phase is the mark kernel alone, with events right before and after its launch)
    seq.seqcdc_plan_set_timing(plan, True)
    acc = np.zeros(4)
    for _ in range(args.steps):
        step()
        acc += np.array(seq.seqcdc_plan_phase_ms(plan))
    seq.seqcdc_plan_set_timing(plan, False)
    ph = acc / args.steps
    phases = {"mark": round(ph[0], 4), "pass_a": round(ph[1], 4), "pass_b": round(ph[2], 4),
              "stitch_compact": round(ph[3], 4)}
    log("phases (ms): %s" % phases)

    roofline = mark_roofline(n, float(ph[0]), args.traffic_json)
    roofline["step_share"] = round(roofline["kernel_ms"] / (dt * 1e3), 4)
    # the whole step against the same peak: the mark kernel's algorithmic bytes plus the cuts, over the step time,
    # and the counter bytes of every kernel of a step (when taken on these sources)
    step_alg = mark_alg_bytes(n) + 8 * count
    roofline["step_frac"] = round(step_alg / dt / 1e9 / HBM_PEAK_GBS, 4)
    roofline["step"] = step_roofline(step_alg, dt * 1e3, stored_step_traffic("plain"))
    log("mark: %s" % roofline)

    extra = {"phases_ms": phases}
    # context: the same stream as a prepared one-file batch replayed as a hipGraph (one submission, the count
    # left on the device); `value` stays the plain call, which returns the count to the host
    gcounts = torch.zeros(1, dtype=torch.int64, device=dev)
    gb = seq.seqcdc_batch_prepare([(d.data_ptr(), n, 0)], [p], cuts.data_ptr(), [0, cap], gcounts.data_ptr(),
                                  settings=plan)
    try:
        for _ in range(args.warmup):
            seq.seqcdc_batch_launch(gb, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            seq.seqcdc_batch_launch(gb, stream=stream)
        torch.cuda.synchronize()
        gdt = (time.perf_counter() - t0) / args.steps
    finally:
        seq.seqcdc_batch_destroy(gb)
    extra["plain_graph"] = {"ms_per_step": round(gdt * 1e3, 4), "GBps": round(n / gdt / 1e9, 1),
                            "counts_match": int(gcounts.item()) == count}
    log("plain as a prepared graph: %s" % extra["plain_graph"])
    # serving before the batched leg: the streams that leg's batches in flight take from torch's pool stay in
    # the process, and with few hardware queues per process they can share one with a serving pass
    if not args.no_serve:
        extra["serving"] = serving(seq, torch, dev)
        log("serving: %s" % {k: v for k, v in extra["serving"].items() if k != "_checks"})
    if not args.no_batch:
        extra["batched"] = batched(seq, torch, stream, plan, args.steps, args.warmup, dev, not args.no_tune)
        log("batched: %s" % extra["batched"])
    if not args.no_dedup:
        extra["dedup"] = dedup_leg(seq, torch, stream, args.steps, args.warmup, dev)
        log("dedup: %s" % {k: v for k, v in extra["dedup"].items() if k != "_check"})
    if not args.no_calib:
        extra["calibration"] = calibration_leg(seq, torch, stream, dev)
        log("calibration: %s" % extra["calibration"])
    if not args.no_sweep:  # last: its autotuning sets the process-wide choices of more parameter classes
        extra["sweep"] = sweep(seq, torch, stream, d, args.steps, not args.no_tune)
        log("sweep: %s" % [{k: v for k, v in c.items() if k != "_check"} for c in extra["sweep"]])

    cpu = None
    if not args.no_cpu:
        want, cpu = cpu_baseline(host, p, args.cpu_seconds)
        got = cuts[:count].cpu().numpy().astype(np.uint64)
        extra["parity_vs_oracle"] = bool(got.size == want.size and np.array_equal(got, want))
        log("cpu oracle: %s, parity %s" % (cpu, extra["parity_vs_oracle"]))
        if "batched" in extra:
            extra["batched"]["cpu_all_cores"] = cpu_batched(seq, extra["batched"]["counts"])
            log("batched cpu context: %s" % extra["batched"]["cpu_all_cores"])
        if "serving" in extra:
            extra["serving"]["parity_vs_oracle"] = serving_parity(extra["serving"]["_checks"])
            log("serving parity %s" % extra["serving"]["parity_vs_oracle"])
        for case in extra.get("sweep", []):
            if "_check" in case:
                got, pp = case.pop("_check")
                host7 = np.resize(RUN7, n)
                want = oracle_chunk(host7, pp)
                case["parity_vs_oracle"] = bool(got.size == want.size and np.array_equal(got, want))
                log("%s: parity %s" % (case["workload"], case["parity_vs_oracle"]))
        if "dedup" in extra:
            extra["dedup"]["parity_vs_oracle"] = dedup_parity(extra["dedup"]["_check"], extra["dedup"]["orig_bytes"],
                                                              extra["dedup"]["unique_bytes"])
            log("dedup parity %s" % extra["dedup"]["parity_vs_oracle"])

    out = {"metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "plain %d MiB mixed backup-like stream, Increasing, avg 8 KiB (Table I)"
                                  % args.size_mib, "bytes": n, "cuts": count, "parallelism": "single GPU",
                      "tuning": tuning},
           "roofline": roofline, "cpu_baseline": cpu}
    if "batched" in extra:
        extra["batched"].pop("counts", None)
    if "serving" in extra:
        extra["serving"].pop("_checks", None)
    if "dedup" in extra:
        extra["dedup"].pop("_check", None)
    for case in extra.get("sweep", []):
        case.pop("_check", None)
    out.update(extra)
    print(json.dumps(out), flush=True)
    seq.seqcdc_plan_destroy(plan)


if __name__ == "__main__":
    main()
