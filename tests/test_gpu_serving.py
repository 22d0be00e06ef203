"""Serving loop: continuous batching over a device-resident request stream.

Each request's cuts must equal the oracle's and the plain per-request path's, whatever else is in flight and in
whatever order requests arrive; admission never exceeds the memory budget.  One test runs the serving workload at
its full sizes: 256 MiB snapshot versions, log-normal request sizes up to 256 MiB, 8 and 32 KiB averages mixed.
"""
import ctypes
import random
import threading
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2505_21194_amd as seq
    return torch, seq


def _server(seq, params, budget, slots=64, streams=3, max_batch=16):
    arr = (seq.seqcdc_params * len(params))(*params)
    cfg = seq.seqcdc_server_config(0, budget, slots, streams, max_batch, len(params), arr)
    h = ctypes.c_void_p()
    rc = seq.lib.seqcdc_server_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == 0, seq.last_error()
    return h, arr


def _requests(count, seed, base_len, median, hi):
    vers = synth.snapshot_series(base_len, 3, seed=seed, nedits=50, maxlen=4096)
    sizes = synth.lognormal_sizes(count, median, 1.5, 1024, hi, seed=seed)
    picks = synth.uniform_ints(count, len(vers), seed=seed, tag=1)
    reqs = []
    for i in range(count):
        v = vers[int(picks[i])]
        n = int(min(sizes[i], v.size))
        off = int(synth.uniform_ints(1, v.size - n + 1, seed=seed + i, tag=2)[0])
        reqs.append((int(picks[i]), off, n, i % 2))
    return vers, reqs


def _run(seq, h, dev_vers, reqs, order):
    tickets = {}
    for i in order:
        vi, off, n, pi = reqs[i]
        t = ctypes.c_uint64()
        rc = seq.lib.seqcdc_server_submit(h, ctypes.c_void_p(dev_vers[vi].data_ptr() + off), n, pi, ctypes.byref(t))
        assert rc == 0, seq.last_error()
        tickets[i] = t.value
    out = {}
    for i, t in tickets.items():
        res = seq.seqcdc_result()
        rc = seq.lib.seqcdc_server_wait(h, t, 60000.0, ctypes.byref(res))
        assert rc == 0, (rc, seq.last_error())
        out[i] = np.ctypeslib.as_array(res.cuts, shape=(res.count,)).copy() if res.count else np.zeros(0, np.uint64)
        assert res.latency_ms >= res.queue_ms >= 0
        assert seq.lib.seqcdc_server_release(h, t) == 0
    return out


def test_serving_matches_oracle_alone_and_in_mix(env):
    torch, seq = env
    params = [seq.seqcdc_params_for_avg(8192), seq.seqcdc_params_for_avg(32768)]
    pd = [dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
               skip_trigger=p.skip_trigger, skip_size=p.skip_size) for p in params]
    vers, reqs = _requests(160, seed=3, base_len=48 << 20, median=512 << 10, hi=24 << 20)
    dev_vers = [torch.from_numpy(v).cuda() for v in vers]
    budget = 192 << 20
    h, keep = _server(seq, params, budget)
    try:
        mixed = _run(seq, h, dev_vers, reqs, list(range(len(reqs))))
        order = list(range(len(reqs)))
        random.Random(5).shuffle(order)
        shuffled = _run(seq, h, dev_vers, reqs, order)
        adm, passes, peak, peak_n = (ctypes.c_uint64() for _ in range(4))
        seq.lib.seqcdc_server_stats(h, ctypes.byref(adm), ctypes.byref(passes), ctypes.byref(peak),
                                    ctypes.byref(peak_n))
        tl = seq.seqcdc_server_timeline(h)
        assert len(tl) == passes.value and sum(r["requests"] for r in tl) == 2 * len(reqs)
        assert sum(r["bytes"] for r in tl) == 2 * sum(r[2] for r in reqs)
        assert all(r["gpu_ms"] > 0 and r["layout_ms"] >= 0 and r["retire_ms"] >= 0 for r in tl)
        assert adm.value == 2 * len(reqs)
        assert peak.value <= budget
        assert passes.value < adm.value  # requests were batched together
        assert peak_n.value > 1  # and several were in flight at once
    finally:
        seq.lib.seqcdc_server_destroy(h)
    for i, (vi, off, n, pi) in enumerate(reqs):
        data = vers[vi][off:off + n]
        want = oracle.chunk(data, **pd[pi])
        alone = seq.chunk(dev_vers[vi][off:off + n], params[pi]).cpu().numpy().astype(np.uint64)
        assert np.array_equal(alone, want), i
        assert np.array_equal(mixed[i], want), i
        assert np.array_equal(shuffled[i], want), i


def test_serving_concurrent_submitters(env):
    torch, seq = env
    params = [seq.seqcdc_params_for_avg(8192), seq.seqcdc_params_for_avg(32768)]
    vers, reqs = _requests(120, seed=8, base_len=24 << 20, median=256 << 10, hi=8 << 20)
    dev_vers = [torch.from_numpy(v).cuda() for v in vers]
    h, keep = _server(seq, params, 64 << 20, slots=16, streams=2, max_batch=8)
    results = {}
    lock = threading.Lock()

    def worker(idx):
        out = _run(seq, h, dev_vers, reqs, idx)
        with lock:
            results.update(out)

    try:
        ths = [threading.Thread(target=worker, args=(list(range(k, len(reqs), 3)),)) for k in range(3)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
    finally:
        seq.lib.seqcdc_server_destroy(h)
    pd = [dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
               skip_trigger=p.skip_trigger, skip_size=p.skip_size) for p in params]
    for i, (vi, off, n, pi) in enumerate(reqs):
        assert np.array_equal(results[i], oracle.chunk(vers[vi][off:off + n], **pd[pi])), i


def test_serving_errors(env):
    torch, seq = env
    params = [seq.seqcdc_params_for_avg(8192)]
    arr = (seq.seqcdc_params * 1)(*params)
    cfg = seq.seqcdc_server_config(0, 64 << 10, 64, 3, 16, 1, arr)  # too small to hold any pass's workspace
    hh = ctypes.c_void_p()
    assert seq.lib.seqcdc_server_create(ctypes.byref(cfg), ctypes.byref(hh)) == seq.SEQCDC_EINVAL
    # 24 MiB over 3 passes: each holds about 5.6 MiB of requests next to its workspace
    h, keep = _server(seq, params, 24 << 20)
    try:
        t = ctypes.c_uint64()
        buf = torch.zeros(8 << 20, dtype=torch.uint8, device="cuda")
        assert seq.lib.seqcdc_server_submit(h, ctypes.c_void_p(buf.data_ptr()), 8 << 20, 0,
                                            ctypes.byref(t)) == seq.SEQCDC_EBUDGET
        assert seq.lib.seqcdc_server_submit(h, ctypes.c_void_p(buf.data_ptr()), 100, 3,
                                            ctypes.byref(t)) == seq.SEQCDC_EINVAL
        res = seq.seqcdc_result()
        assert seq.lib.seqcdc_server_poll(h, 987654, ctypes.byref(res)) == seq.SEQCDC_ENOENT
        assert seq.lib.seqcdc_server_submit(h, ctypes.c_void_p(buf.data_ptr()), 0, 0, ctypes.byref(t)) == 0
        assert seq.lib.seqcdc_server_wait(h, t.value, 1000.0, ctypes.byref(res)) == 0 and res.count == 0
        assert seq.lib.seqcdc_server_submit(h, ctypes.c_void_p(buf.data_ptr()), 3 << 20, 0, ctypes.byref(t)) == 0
        assert seq.lib.seqcdc_server_wait(h, t.value, 30000.0, ctypes.byref(res)) == 0
        assert res.count == 3 << 20 >> 14  # all-zero bytes: every chunk is cut at the 16 KiB maximum
    finally:
        seq.lib.seqcdc_server_destroy(h)


def test_serving_poll_until_done(env):
    """The non-blocking poll: pending (SEQCDC_EAGAIN) until the pass completes, then the result, then unknown after
    release."""
    torch, seq = env
    params = [seq.seqcdc_params_for_avg(8192)]
    pd = dict(mode=0, seq_length=5, min_size=4096, max_size=16384, skip_trigger=50, skip_size=256)
    host = synth.mixed(40 << 20, seed=81)
    dev = torch.from_numpy(host).cuda()
    h, keep = _server(seq, params, 512 << 20)
    try:
        t = ctypes.c_uint64()
        assert seq.lib.seqcdc_server_submit(h, ctypes.c_void_p(dev.data_ptr()), host.size, 0, ctypes.byref(t)) == 0
        res = seq.seqcdc_result()
        seen_pending = 0
        t0 = time.perf_counter()
        while True:
            rc = seq.lib.seqcdc_server_poll(h, t.value, ctypes.byref(res))
            if rc == 0:
                break
            assert rc == seq.SEQCDC_EAGAIN and res.status == seq.SEQCDC_EAGAIN
            seen_pending += 1
            assert time.perf_counter() - t0 < 60.0
            time.sleep(0.0002)
        assert res.status == 0 and res.latency_ms >= res.queue_ms >= 0
        got = np.ctypeslib.as_array(res.cuts, shape=(res.count,)).copy()
        assert np.array_equal(got, oracle.chunk(host, **pd))
        assert seq.lib.seqcdc_server_release(h, t.value) == 0
        assert seq.lib.seqcdc_server_poll(h, t.value, ctypes.byref(res)) == seq.SEQCDC_ENOENT
    finally:
        seq.lib.seqcdc_server_destroy(h)


def test_serving_full_size_requests(env):
    """The serving workload at its full sizes: slices of 256 MiB snapshot versions with log-normal sizes (median
    1 MiB, sigma 1.5, clamped to 1 KiB..256 MiB, several whole-version requests among them), half at the 8 KiB and
    half at the 32 KiB parameters, all in flight together under a 4 GiB budget; every result equals the oracle's."""
    torch, seq = env
    params = [seq.seqcdc_params_for_avg(8192), seq.seqcdc_params_for_avg(32768)]
    pd = [dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
               skip_trigger=p.skip_trigger, skip_size=p.skip_size) for p in params]
    vers = synth.snapshot_series(256 << 20, 3, seed=11, nedits=200, maxlen=4096)
    sizes = synth.lognormal_sizes(240, 1 << 20, 1.5, 1024, 256 << 20, seed=12)
    picks = synth.uniform_ints(240, len(vers), seed=12, tag=1)
    reqs = []
    for i in range(240):
        v = vers[int(picks[i])]
        n = int(min(sizes[i], v.size))
        off = int(synth.uniform_ints(1, v.size - n + 1, seed=1200 + i, tag=2)[0])
        reqs.append((int(picks[i]), off, n, i % 2))
    for j, vi in enumerate((0, 2)):  # whole versions (the 256 MiB clamp), one at each average
        reqs.append((vi, 0, int(vers[vi].size), j))
    dev_vers = [torch.from_numpy(v).cuda() for v in vers]
    budget = 4 << 30
    h, keep = _server(seq, params, budget, slots=256, streams=4, max_batch=64)
    try:
        print("[case] serving full size:", len(reqs), "requests,", sum(r[2] for r in reqs) >> 20, "MiB", flush=True)
        out = _run(seq, h, dev_vers, reqs, list(range(len(reqs))))
        adm, passes, peak, peak_n = (ctypes.c_uint64() for _ in range(4))
        seq.lib.seqcdc_server_stats(h, ctypes.byref(adm), ctypes.byref(passes), ctypes.byref(peak),
                                    ctypes.byref(peak_n))
        assert adm.value == len(reqs) and peak.value <= budget
    finally:
        seq.lib.seqcdc_server_destroy(h)
    assert max(r[2] for r in reqs) >= 256 << 20
    for i, (vi, off, n, pi) in enumerate(reqs):
        want = oracle.chunk(vers[vi][off:off + n], **pd[pi])
        assert out[i].size == want.size and np.array_equal(out[i], want), i


def test_serving_submit_many_scheduled(env):
    """Requests queued by the library at scheduled arrival offsets: each gets its own ticket and the oracle's cuts;
    a batch with an invalid request queues nothing."""
    torch, seq = env
    params = [seq.seqcdc_params_for_avg(8192), seq.seqcdc_params_for_avg(32768)]
    pd = [dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
               skip_trigger=p.skip_trigger, skip_size=p.skip_size) for p in params]
    vers, reqs = _requests(60, seed=14, base_len=16 << 20, median=256 << 10, hi=8 << 20)
    dev_vers = [torch.from_numpy(v).cuda() for v in vers]
    files = [(dev_vers[vi].data_ptr() + off, n, pi) for vi, off, n, pi in reqs]
    h, keep = _server(seq, params, 256 << 20)
    try:
        bad = files[:3] + [(0, 100, 0)]  # NULL data
        with pytest.raises(seq.SeqCDCError):
            seq.seqcdc_server_submit_many(h, bad)
        at = np.arange(len(files), dtype=np.float64) * 0.05  # one request every 50 us
        tickets, sub = seq.seqcdc_server_submit_many(h, files, at)
        assert len(set(int(t) for t in tickets)) == len(files)
        assert np.all(sub >= at - 1e-6) and np.all(np.diff(sub) >= 0)
        for i, t in enumerate(tickets):
            res = seq.seqcdc_result()
            assert seq.lib.seqcdc_server_wait(h, int(t), 60000.0, ctypes.byref(res)) == 0
            got = np.ctypeslib.as_array(res.cuts, shape=(res.count,)).copy() if res.count else np.zeros(0, np.uint64)
            vi, off, n, pi = reqs[i]
            assert np.array_equal(got, oracle.chunk(vers[vi][off:off + n], **pd[pi])), i
            assert seq.lib.seqcdc_server_release(h, int(t)) == 0
        adm = ctypes.c_uint64()
        seq.lib.seqcdc_server_stats(h, ctypes.byref(adm), None, None, None)
        assert adm.value == sum(1 for r in reqs if r[2] > 0)  # nothing of the rejected batch was queued
    finally:
        seq.lib.seqcdc_server_destroy(h)
