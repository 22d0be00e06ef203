"""Resolve modes, the autotuner and the dedup ratio of a backup-snapshot series.

* Every resolve mode gives the oracle's cuts on many small files and on prepared (graph-replayed) batches.
* Whatever the autotuner picks, the cuts do not change.
* Config 3 at reduced size: a uniform base plus versions made by seeded edits, chunked on the GPU at
  4/8/16/32/64 KiB averages; the cut lists equal the oracle's and the space savings of Eq. 1 computed by
  the library equal the oracle's.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

MODES = [0, 1]  # resolve modes of seqcdc_plan_set_mode: marked, direct


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_21194_amd as seq
    return torch, seq


def _say(*a):
    print("[case]", *a, flush=True)


def P(mode=0, sl=5, mn=4096, mx=16384, trig=50, skip=256):
    return dict(mode=mode, seq_length=sl, min_size=mn, max_size=mx, skip_trigger=trig, skip_size=skip)


def test_autotune_keeps_results(env):
    torch, seq = env
    data = synth.mixed(16 << 20, seed=31)
    d = torch.from_numpy(data).cuda()
    p = seq.seqcdc_params_for_avg(8192)
    pd = dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
              skip_trigger=p.skip_trigger, skip_size=p.skip_size)
    want = oracle.chunk(data, **pd)
    plan = seq.seqcdc_plan_create()
    try:
        _say("autotune 16 MiB")
        ms = seq.seqcdc_autotune(plan, d.data_ptr(), d.numel(), p)
        assert ms > 0
        seg, span, waves = seq.seqcdc_plan_get_tuning(plan, d.numel(), p)
        assert seg > 0 and span in (4, 8, 16, 32, 64) and 0 < waves <= 32
        # a stream of the tuned size uses the tuned segment length as measured (a candidate multiple of min_size)
        assert seg % p.min_size == 0 and seg // p.min_size in (32, 64, 128, 256, 512, 1024)
        # a stream under half the tuned size shrinks it to fill the device: the stream's bytes over the chain
        # waves (CUs x waves per CU), but not below 64 KiB x (min_size / 4 KiB)^2, and at least 64 KiB
        small = 4 << 20
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        m = p.min_size >> 12
        floor = (64 << 10) * min(m * m, 1 << 20) if m > 1 else 64 << 10
        fill = small // (cus * waves)
        expect = max(fill, min(floor, seg)) if fill < seg else seg
        assert seq.seqcdc_plan_get_tuning(plan, small, p)[0] == max(expect, 64 << 10)
        got = seq.chunk(d, p, plan=plan).cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, want)
    finally:
        seq.seqcdc_plan_destroy(plan)


def _pd(p):
    return dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
                skip_trigger=p.skip_trigger, skip_size=p.skip_size)


def test_autotune_batch_keeps_results(env):
    """The batch autotuner times the batched call over these files and sets the plan's settings; the batch and a
    prepared batch with those settings then give the oracle's cuts for every file."""
    torch, seq = env
    sizes = synth.lognormal_sizes(48, 256 * 1024, 1.5, 4096, 8 << 20, seed=33).astype(np.int64)
    datas = [synth.mixed(int(n), seed=500 + i) for i, n in enumerate(sizes)]
    tens = [torch.from_numpy(x).cuda() for x in datas]
    p16, p8 = seq.seqcdc_params_for_avg(16384), seq.seqcdc_params_for_avg(8192)
    params = [p16, p8]
    pidx = [i % 2 for i in range(len(tens))]
    offs = [0]
    for t, k in zip(tens, pidx):
        offs.append(offs[-1] + seq.seqcdc_max_cuts(t.numel(), params[k]))
    cuts = torch.empty(offs[-1], dtype=torch.int64, device="cuda")
    counts = torch.empty(len(tens), dtype=torch.int64, device="cuda")
    files = [(t.data_ptr(), t.numel(), k) for t, k in zip(tens, pidx)]
    wants = [oracle.chunk(x, **_pd(params[k])) for x, k in zip(datas, pidx)]

    def check(label):
        torch.cuda.synchronize()
        c = counts.cpu().numpy()
        allc = cuts.cpu().numpy().astype(np.uint64)
        for i, w in enumerate(wants):
            got = allc[offs[i]:offs[i] + int(c[i])]
            assert got.size == w.size and np.array_equal(got, w), (label, i)

    plan = seq.seqcdc_plan_create()
    try:
        _say("batch autotune, 48 files, two parameter sets")
        ms = seq.seqcdc_autotune_batch(plan, files, params, cuts.data_ptr(), offs, counts.data_ptr())
        assert ms > 0
        check("tuning")
        cuts.fill_(0)
        counts.fill_(0)
        seq.seqcdc_chunk_batch(files, params, cuts.data_ptr(), offs, counts.data_ptr(), plan=plan)
        check("tuned batch")
        cuts.fill_(0)
        counts.fill_(0)
        b = seq.seqcdc_batch_prepare(files, params, cuts.data_ptr(), offs, counts.data_ptr(), settings=plan)
        try:
            seq.seqcdc_batch_launch(b)
            check("tuned prepared batch")
        finally:
            seq.seqcdc_batch_destroy(b)
    finally:
        seq.seqcdc_plan_destroy(plan)


@pytest.mark.parametrize("avg_kib", [4, 8, 16, 32, 64])
def test_snapshot_dedup_matches_oracle(env, avg_kib):
    torch, seq = env
    versions = synth.snapshot_series(16 << 20, 4, seed=21, nedits=200, maxlen=4096)
    p = seq.seqcdc_params_for_avg(avg_kib << 10)
    pd = dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
              skip_trigger=p.skip_trigger, skip_size=p.skip_size)
    _say("snapshot dedup", avg_kib, "KiB,", len(versions), "versions")
    tens = [torch.from_numpy(v).cuda() for v in versions]
    outs = seq.chunk_batch(tens, [p])
    gpu_cuts = [o.cpu().numpy().astype(np.uint64) for o in outs]
    ora_cuts = [oracle.chunk(v, **pd) for v in versions]
    for g, w in zip(gpu_cuts, ora_cuts):
        assert np.array_equal(g, w)
    got = seq.seqcdc_dedup_stats(versions, gpu_cuts)
    want = oracle.dedup_stats(versions, ora_cuts)
    assert got[0] == want[0] and got[1] == want[1]  # original and unique bytes, exactly
    assert got[2] == pytest.approx(want[2], abs=1e-12) and got[3] == pytest.approx(want[3], rel=1e-12)
    assert 0.0 < want[2] < 0.75  # some chunks repeat across the 4 versions; never more than 3 of 4 copies


@pytest.mark.parametrize("groups", [1, 2, 4, 8])
def test_overlapped_batch(env, groups):
    """File groups marked on the caller's stream while side streams run earlier groups' chains: same cuts."""
    torch, seq = env
    rng = np.random.default_rng(40 + groups)
    sizes = [int(x) for x in rng.integers(0, 3 << 20, 36)] + [0, 1, 70000, 8 << 20, 5 << 20]
    params = [P(), P(mode=1, sl=6, mn=8192, mx=32768, skip=512)]
    pidx = [i % 2 for i in range(len(sizes))]
    datas = [synth.mixed(s, seed=900 + i) for i, s in enumerate(sizes)]
    tens = [torch.from_numpy(x).cuda() if x.size else torch.zeros(0, dtype=torch.uint8, device="cuda") for x in datas]
    plan = seq.seqcdc_plan_create()
    try:
        seq.seqcdc_plan_set_tuning(plan, segment_bytes=128 << 10)
        seq.seqcdc_plan_set_overlap(plan, groups)
        seq.seqcdc_plan_set_timing(plan, True)
        for rep in range(2):  # the plan's buffers, streams and events are reused
            _say("overlapped batch", groups, "groups, call", rep)
            outs = seq.chunk_batch(tens, params, params_index=pidx, plan=plan)
            for i, (x, o) in enumerate(zip(datas, outs)):
                assert np.array_equal(o.cpu().numpy().astype(np.uint64), oracle.chunk(x, **params[pidx[i]])), (rep, i)
        ms = seq.seqcdc_plan_phase_ms(plan)
        assert len(ms) == 4 and all(m >= 0 for m in ms)
    finally:
        seq.seqcdc_plan_destroy(plan)


@pytest.mark.parametrize("mode", MODES)
def test_many_small_files(env, mode):
    """Thousands of tiny files, many per 64 mark spans (the span -> file lookup), plus a few large ones."""
    torch, seq = env
    rng = np.random.default_rng(77 + mode)
    sizes = [int(x) for x in rng.integers(0, 12000, 2500)] + [0, 3 << 20, 0, 1, 1 << 20]
    p = P()
    datas = [synth.uniform(s, seed=3000 + i) for i, s in enumerate(sizes)]
    host = np.concatenate([d for d in datas if d.size] + [np.zeros(1, np.uint8)])
    buf = torch.from_numpy(host).cuda()
    offs = np.concatenate([[0], np.cumsum(sizes)])
    tens = [buf[int(offs[i]):int(offs[i + 1])] for i in range(len(sizes))]
    plan = seq.seqcdc_plan_create()
    try:
        seq.seqcdc_plan_set_tuning(plan, segment_bytes=256 << 10, mark_span_blocks=4)
        seq.seqcdc_plan_set_mode(plan, mode)
        _say("many small files, mode", mode)
        outs = seq.chunk_batch(tens, [p], plan=plan)
    finally:
        seq.seqcdc_plan_destroy(plan)
    for i, (x, o) in enumerate(zip(datas, outs)):
        assert np.array_equal(o.cpu().numpy().astype(np.uint64), oracle.chunk(x, **p)), i


@pytest.mark.parametrize("mode", MODES)
def test_prepared_batch_graph_replays(env, mode):
    """A prepared (hipGraph-captured) batch: each replay, with new input contents and eager work in between,
    equals the oracle."""
    torch, seq = env
    rng = np.random.default_rng(123 + mode)
    sizes = [int(x) for x in rng.integers(0, 2 << 20, 20)] + [0, 1, 6 << 20]
    params = [P(), P(mode=1, sl=6, mn=8192, mx=32768, skip=512)]
    pidx = [i % 2 for i in range(len(sizes))]
    bufs = [torch.zeros(max(s, 1), dtype=torch.uint8, device="cuda") for s in sizes]
    ps = [seq.make_params(**p) for p in params]
    offs = [0]
    for s, pi in zip(sizes, pidx):
        offs.append(offs[-1] + max(seq.seqcdc_max_cuts(s, ps[pi]), 1))
    cuts = torch.zeros(offs[-1], dtype=torch.int64, device="cuda")
    counts = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
    ftab = seq.file_table([b.data_ptr() for b in bufs], sizes, pidx)
    settings = seq.seqcdc_plan_create()
    seq.seqcdc_plan_set_tuning(settings, segment_bytes=128 << 10)
    seq.seqcdc_plan_set_mode(settings, mode)
    other = seq.seqcdc_plan_create()
    _say("prepare graph batch, mode", mode)
    batch = seq.seqcdc_batch_prepare(ftab, ps, cuts.data_ptr(), offs, counts.data_ptr(), settings=settings)
    try:
        for rep in range(3):
            datas = [synth.mixed(s, seed=5000 + 100 * rep + i) for i, s in enumerate(sizes)]
            for b, d in zip(bufs, datas):  # new contents, same buffers
                if d.size:
                    b[:d.size].copy_(torch.from_numpy(d))
            cuts.zero_()
            counts.zero_()
            # eager work of the program's own between replays
            eager = seq.chunk_batch([b[:s] for b, s in zip(bufs, sizes)], params, params_index=pidx, plan=other)
            torch.cuda.synchronize()
            _say("replay", rep)
            seq.seqcdc_batch_launch(batch)
            torch.cuda.synchronize()
            cnt = counts.cpu().numpy()
            for i, (d, s) in enumerate(zip(datas, sizes)):
                want = oracle.chunk(d, **params[pidx[i]])
                got = cuts[offs[i]:offs[i] + int(cnt[i])].cpu().numpy().astype(np.uint64)
                assert np.array_equal(got, want), (rep, i)
                assert np.array_equal(eager[i].cpu().numpy().astype(np.uint64), want), (rep, i)
    finally:
        seq.seqcdc_batch_destroy(batch)
        seq.seqcdc_plan_destroy(settings)
        seq.seqcdc_plan_destroy(other)
