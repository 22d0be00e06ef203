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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size-mib", type=int, default=1024)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the other plain variants")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the library's autotuner (default settings)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="oracle work to time on the host")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run a 1 GiB device copy and the mark kernel (for rocprofv3 --pmc runs)")
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


def batched(seq, torch, stream, plan, steps, warmup, dev, tune):
    import synth
    nfiles = 4096
    sizes = synth.lognormal_sizes(nfiles, 256 * 1024, 1.5, 4096, 64 << 20, seed=4).astype(np.int64)
    total = int(sizes.sum())
    log("batched: %d files, %.2f GiB" % (nfiles, total / 2 ** 30))
    buf = torch.empty(total, dtype=torch.uint8, device=dev)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    for f in range(nfiles):
        buf[int(offs[f]):int(offs[f + 1])].copy_(torch.from_numpy(synth.mixed(int(sizes[f]), seed=100000 + f)))
    pb = seq.seqcdc_params_for_avg(16384)
    cut_offs = [0]
    for s in sizes:
        cut_offs.append(cut_offs[-1] + seq.seqcdc_max_cuts(int(s), pb))
    bcuts = torch.empty(cut_offs[-1], dtype=torch.int64, device=dev)
    bcounts = torch.empty(nfiles, dtype=torch.int64, device=dev)
    files = [(buf.data_ptr() + int(offs[f]), int(sizes[f]), 0) for f in range(nfiles)]
    ftab = seq.file_table([f[0] for f in files], sizes)  # marshalled once, like a caller's own table
    otab = seq.offsets_table(cut_offs)

    def bstep():
        seq.seqcdc_chunk_batch(ftab, [pb], bcuts.data_ptr(), otab, bcounts.data_ptr(), stream=stream, plan=plan)

    tuning = None
    if tune:  # the autotuner on the batch's bytes taken as one stream, at the batch's parameters (untimed)
        seq.seqcdc_autotune(plan, buf.data_ptr(), total, pb, stream=stream)
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
    del buf, bcuts
    return {"files": nfiles, "bytes": total, "cuts": int(counts.sum()), "ms_per_step": round(bdt * 1e3, 3),
            "GBps": round(total / bdt / 1e9, 1), "frac_hbm_peak_input": round(total / bdt / 1e9 / HBM_PEAK_GBS, 4),
            "graph_ms_per_step": round(gdt * 1e3, 3), "graph_GBps": round(total / gdt / 1e9, 1),
            "graph_counts_match": graph_same,
            "per_file_launch_GBps": round(total / pdt / 1e9, 2), "speedup_vs_per_file": round(pdt / bdt, 2),
            "params": "avg 16 KiB: SeqLength 5, SkipTrigger 50, SkipSize 512, min 8 KiB, max 32 KiB",
            "tuning": tuning, "counts": counts}


def serving(seq, torch, dev, streams=4, max_batch=64):
    """Poisson request stream through the serving loop; returns latency percentiles per offered load."""
    import synth
    vers = synth.snapshot_series(256 << 20, 3, seed=11, nedits=200, maxlen=4096)
    dvers = [torch.from_numpy(v).to(dev) for v in vers]
    rng = np.random.default_rng(5)
    params = [seq.seqcdc_params_for_avg(8192), seq.seqcdc_params_for_avg(32768)]
    nreq = 400
    sizes = synth.lognormal_sizes(nreq, 1 << 20, 1.5, 1024, 256 << 20, seed=12).astype(np.int64)
    reqs = []
    for i in range(nreq):
        v = int(rng.integers(len(vers)))
        n = int(min(sizes[i], vers[v].size))
        off = int(rng.integers(vers[v].size - n + 1))
        reqs.append((dvers[v].data_ptr() + off, n, i % 2))
    total = sum(r[1] for r in reqs)
    arr = (seq.seqcdc_params * 2)(*params)
    cfg = seq.seqcdc_server_config(0, 4 << 30, 256, streams, max_batch, 2, arr)
    h = ctypes.c_void_p()
    if seq.lib.seqcdc_server_create(ctypes.byref(cfg), ctypes.byref(h)):
        raise RuntimeError(seq.last_error())

    def passes():
        v = ctypes.c_uint64()
        if seq.lib.seqcdc_server_stats(h, None, ctypes.byref(v), None, None):
            raise RuntimeError(seq.last_error())
        return v.value

    def run(rate_gbs):
        """Submit reqs at Poisson arrival times for an offered load (GB/s); None = all at once."""
        tickets = [None] * nreq
        p0 = passes()
        if rate_gbs:
            mean = total / nreq
            gaps = rng.exponential(mean / (rate_gbs * 1e9), nreq)
            arrivals = np.cumsum(gaps)
        else:
            arrivals = np.zeros(nreq)
        t0 = time.perf_counter()
        for i, (ptr, n, pi) in enumerate(reqs):
            while time.perf_counter() - t0 < arrivals[i]:
                pass
            t = ctypes.c_uint64()
            if seq.lib.seqcdc_server_submit(h, ctypes.c_void_p(ptr), n, pi, ctypes.byref(t)):
                raise RuntimeError(seq.last_error())
            tickets[i] = t.value
        lat = []
        for t in tickets:
            res = seq.seqcdc_result()
            if seq.lib.seqcdc_server_wait(h, t, 60000.0, ctypes.byref(res)):
                raise RuntimeError(seq.last_error())
            lat.append(res.latency_ms)
            seq.lib.seqcdc_server_release(h, t)
        dt = time.perf_counter() - t0
        lat = np.array(lat)
        return {"offered_GBps": round(rate_gbs, 2) if rate_gbs else None, "GBps": round(total / dt / 1e9, 2),
                "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "passes": passes() - p0}

    try:
        for _ in range(3):  # warm-up: the passes' buffers grow to the largest batches they meet
            run(None)
        sat = run(None)
        peak = sat["GBps"]
        loads = [run(frac * peak) for frac in (0.1, 0.4, 0.8)]
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
    return {"requests": nreq, "bytes": total, "saturated": sat, "loads": loads,
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
    p64 = seq.seqcdc_params_for_avg(8192)
    p64.max_size = 65536
    cases.append(("8 MiB uniform (seed 0), increasing, avg 8 KiB, max 64 KiB", small, p64))
    plan = seq.seqcdc_plan_create()
    try:
        for name, t, p in cases:
            n = t.numel()
            cap = seq.seqcdc_max_cuts(n, p)
            cuts = torch.empty(cap, dtype=torch.int64, device=t.device)
            if tune and n >= (64 << 20):
                seq.seqcdc_autotune(plan, t.data_ptr(), n, p, stream=stream)
            for _ in range(2):
                cnt = seq.seqcdc_chunk(t.data_ptr(), n, p, cuts.data_ptr(), cap, stream=stream, plan=plan)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                cnt = seq.seqcdc_chunk(t.data_ptr(), n, p, cuts.data_ptr(), cap, stream=stream, plan=plan)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            seg, span, waves = seq.seqcdc_plan_get_tuning(plan, n, p)
            out.append({"workload": name, "ms": round(dt * 1e3, 4), "GBps": round(n / dt / 1e9, 1), "cuts": cnt,
                        "tuning": {"segment_bytes": seg, "mark_span_blocks": span, "waves_per_cu": waves}})
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
        groups = (n + 63) // 64
        eo = torch.empty(4 * groups, dtype=torch.int32, device=dev)
        for _ in range(5):
            seq.seqcdc_mark(d.data_ptr(), n, p, eo.data_ptr(), stream=stream)
        torch.cuda.synchronize()
        log("traffic probe done")
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
    if not args.no_batch:
        extra["batched"] = batched(seq, torch, stream, plan, args.steps, args.warmup, dev, not args.no_tune)
        log("batched: %s" % extra["batched"])
    if not args.no_serve:
        extra["serving"] = serving(seq, torch, dev)
        log("serving: %s" % extra["serving"])
    if not args.no_sweep:  # last: its autotuning sets the process-wide choices of more parameter classes
        extra["sweep"] = sweep(seq, torch, stream, d, args.steps, not args.no_tune)
        log("sweep: %s" % extra["sweep"])

    cpu = None
    if not args.no_cpu:
        want, cpu = cpu_baseline(host, p, args.cpu_seconds)
        got = cuts[:count].cpu().numpy().astype(np.uint64)
        extra["parity_vs_oracle"] = bool(got.size == want.size and np.array_equal(got, want))
        log("cpu oracle: %s, parity %s" % (cpu, extra["parity_vs_oracle"]))
        if "batched" in extra:
            extra["batched"]["cpu_all_cores"] = cpu_batched(seq, extra["batched"]["counts"])
            log("batched cpu context: %s" % extra["batched"]["cpu_all_cores"])

    out = {"metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "plain %d MiB mixed backup-like stream, Increasing, avg 8 KiB (Table I)"
                                  % args.size_mib, "bytes": n, "cuts": count, "parallelism": "single GPU",
                      "tuning": tuning},
           "roofline": roofline, "cpu_baseline": cpu}
    if "batched" in extra:
        extra["batched"].pop("counts", None)
    out.update(extra)
    print(json.dumps(out), flush=True)
    seq.seqcdc_plan_destroy(plan)


if __name__ == "__main__":
    main()
