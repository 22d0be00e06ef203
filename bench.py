"""Chunking throughput of SeqCDC on one MI355X.

Workload (one step = one pass of the whole hot path over the batch):
  plain:   one 1 GiB mixed backup-like stream (1 MiB blocks: 50% uniform, 30% Zipf(1.1) text over 64 printable
           symbols, 20% zero / repeated-16-byte runs), Increasing mode, 8 KiB target average (Table I: SeqLength 5,
           SkipTrigger 50, SkipSize 256; min 4 KiB, max 16 KiB).  Stream resident in HBM; a step is one
           seqcdc_chunk call (mark, speculative chains, continuations, stitch, compaction, count read-back).
  batched: 4096 files, log-normal sizes (median 256 KiB, sigma 1.5, clamped 4 KiB..64 MiB), each a mixed stream
           under its own seed, 16 KiB average (SeqLength 5, 50 / 512, min 8 KiB, max 32 KiB), one
           seqcdc_chunk_batch call per step, compared with one seqcdc_chunk call per file.
value = plain input bytes per second (GB/s = 1e9 B/s).  Roofline: the mark kernel, the dominant one.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size-mib", type=int, default=1024)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--traffic-json", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                                           "mark_traffic.json"))
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
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
    cap = seq.seqcdc_max_cuts(n, p)
    cuts = torch.empty(cap, dtype=torch.int64, device=dev)
    plan = seq.seqcdc_plan_create()
    torch.cuda.synchronize()

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

    # ---- dominant kernel: mark, timed with HIP events on the stream it is launched on
    groups = (n + 63) // 64
    eo = torch.empty(4 * groups, dtype=torch.int32, device=dev)
    reps = 20
    for _ in range(3):
        seq.seqcdc_mark(d.data_ptr(), n, p, eo.data_ptr(), stream=stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        seq.seqcdc_mark(d.data_ptr(), n, p, eo.data_ptr(), stream=stream)
    ev1.record(stream)
    ev1.synchronize()
    mark_ms = ev0.elapsed_time(ev1) / reps
    alg_bytes = n + 16 * groups  # read every input byte once, write 2 bits per byte
    achieved = alg_bytes / (mark_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            traffic = json.load(open(args.traffic_json)).get("bytes_per_launch_scaled")
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "mark_kernel",
                "kernel_ms": round(mark_ms, 4), "alg_bytes_per_launch": alg_bytes}
    log("mark: %.3f ms, %.1f GB/s algorithmic" % (mark_ms, achieved))

    extra = {}
    # ---- batched
    if not args.no_batch:
        nfiles = 4096
        sizes = synth.lognormal_sizes(nfiles, 256 * 1024, 1.5, 4096, 64 << 20, seed=4).astype(np.int64)
        total = int(sizes.sum())
        log("batched: %d files, %.2f GiB" % (nfiles, total / 2 ** 30))
        buf = torch.empty(total, dtype=torch.uint8, device=dev)
        offs = np.concatenate([[0], np.cumsum(sizes)])
        chunk_host = None
        for f in range(nfiles):
            chunk_host = synth.mixed(int(sizes[f]), seed=100000 + f)
            buf[int(offs[f]):int(offs[f + 1])].copy_(torch.from_numpy(chunk_host))
        pb = seq.seqcdc_params_for_avg(16384)
        cut_offs = [0]
        for s in sizes:
            cut_offs.append(cut_offs[-1] + seq.seqcdc_max_cuts(int(s), pb))
        bcuts = torch.empty(cut_offs[-1], dtype=torch.int64, device=dev)
        bcounts = torch.empty(nfiles, dtype=torch.int64, device=dev)
        files = [(buf.data_ptr() + int(offs[f]), int(sizes[f]), 0) for f in range(nfiles)]

        def bstep():
            seq.seqcdc_chunk_batch(files, [pb], bcuts.data_ptr(), cut_offs, bcounts.data_ptr(), stream=stream,
                                   plan=plan)

        for _ in range(args.warmup):
            bstep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bstep()
        torch.cuda.synchronize()
        bdt = (time.perf_counter() - t0) / args.steps
        # one plain launch per file
        pcap = max(cut_offs[i + 1] - cut_offs[i] for i in range(nfiles))
        t0 = time.perf_counter()
        for f in range(nfiles):
            seq.seqcdc_chunk(files[f][0], files[f][1], pb, bcuts.data_ptr(), pcap, stream=stream, plan=plan)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        extra["batched"] = {"files": nfiles, "bytes": total, "ms_per_step": round(bdt * 1e3, 3),
                            "GBps": round(total / bdt / 1e9, 1), "per_file_launch_GBps": round(total / pdt / 1e9, 2),
                            "speedup_vs_per_file": round(pdt / bdt, 2)}
        log("batched: %s" % extra["batched"])

    # ---- CPU baseline: the oracle on a bounded sample of the same stream
    cpu = None
    if not args.no_cpu:
        import oracle
        sample = host[: min(n, 512 << 20)]
        t0 = time.perf_counter()
        oc = oracle.chunk(sample, mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
                          skip_trigger=p.skip_trigger, skip_size=p.skip_size)
        cdt = time.perf_counter() - t0
        reps_cpu = max(1, int(10.0 / max(cdt, 1e-3)))
        t0 = time.perf_counter()
        for _ in range(min(reps_cpu, 50)):
            oracle.chunk(sample, mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
                         skip_trigger=p.skip_trigger, skip_size=p.skip_size)
        cdt = (time.perf_counter() - t0) / min(reps_cpu, 50)
        cpu = {"value": round(sample.size / cdt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": "first %d MiB of the same stream, %d repetitions, single thread" % (
                   sample.size >> 20, min(reps_cpu, 50))}
        got = cuts[:count].cpu().numpy().astype(np.uint64)
        want_prefix = oc[oc < sample.size - (64 << 10)]
        extra["parity_prefix_ok"] = bool(np.array_equal(got[:want_prefix.size], want_prefix))
        log("cpu oracle: %s" % cpu)

    out = {"metric": "chunking GB/s on 1 MI355X (plain 1 GiB stream; batched in 'batched')", "value": round(value, 2),
           "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "plain 1 GiB mixed stream, Increasing, avg 8 KiB (Table I)", "bytes": n,
                      "cuts": count, "parallelism": "single GPU"},
           "roofline": roofline, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)
    seq.seqcdc_plan_destroy(plan)


if __name__ == "__main__":
    main()
