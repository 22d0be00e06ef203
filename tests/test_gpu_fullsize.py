"""Parity at the full sizes of the benchmark workloads, whole outputs against the oracle.

* One 1 GiB mixed backup-like stream (1 MiB blocks: uniform, Zipf text, zero / repeated-pattern runs), both
  modes, 8 / 16 / 32 KiB averages (Table I), with the default plan (the configuration bench.py times), and the
  8 KiB parameters at SeqLength 6 in both modes.
* A 256 MiB uniform base plus 9 versions of 200 seeded edits each, chunked in one batch at 4..64 KiB averages:
  every boundary list and the space savings of Eq. 1.
* 512 MiB uniform in 64 KiB segments: more jumps and covered ranges than the stitch keeps in LDS.
* 160 MiB of alternating segment kinds in 64 KiB segments: jumps resolved in LDS, covered ranges beyond it.
* 4096 files with log-normal sizes (median 256 KiB, sigma 1.5, 4 KiB..64 MiB), each a mixed stream of its own
  seed, at a 16 KiB average: the eager batched call and its prepared hipGraph replay.
The plain streams and the 4096-file batch also run in the direct (skip-aware) resolve mode.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import stitch_cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_21194_amd as seq
    return torch, seq


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def direct_plan(env):
    torch, seq = env
    plan = seq.seqcdc_plan_create()
    seq.seqcdc_plan_set_mode(plan, 1)
    yield plan
    seq.seqcdc_plan_destroy(plan)


def _pd(p):
    return dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
                skip_trigger=p.skip_trigger, skip_size=p.skip_size)


@pytest.fixture(scope="module")
def stream_1g(env):
    torch, seq = env
    host = synth.mixed(1 << 30, seed=2)
    return host, torch.from_numpy(host).cuda()


@pytest.mark.parametrize("avg_kib", [8, 16, 32])
@pytest.mark.parametrize("mode", [0, 1])
def test_plain_1gib_mixed(env, stream_1g, direct_plan, avg_kib, mode):
    torch, seq = env
    host, dev = stream_1g
    p = seq.seqcdc_params_for_avg(avg_kib << 10)
    p.mode = mode
    want = oracle.chunk(host, **_pd(p))
    for pl, label in ((None, "marked"), (direct_plan, "direct")):
        _say("plain 1 GiB mixed, avg", avg_kib, "KiB, mode", mode, label)
        got = seq.chunk(dev, p, plan=pl).cpu().numpy().astype(np.uint64)
        assert got.size == want.size and np.array_equal(got, want), label


@pytest.mark.parametrize("mode", [0, 1])
def test_plain_1gib_mixed_seqlength6(env, stream_1g, direct_plan, mode):
    """SeqLength counted as bytes with 6 in place of Table I's 5 (the reading under which Table I's averages hold
    on random data), 8 KiB parameters otherwise: many more skips per chunk and max-size cuts."""
    torch, seq = env
    host, dev = stream_1g
    p = seq.seqcdc_params_for_avg(8192)
    p.seq_length = 6
    p.mode = mode
    want = oracle.chunk(host, **_pd(p))
    for pl, label in ((None, "marked"), (direct_plan, "direct")):
        _say("plain 1 GiB mixed, SeqLength 6, mode", mode, label)
        got = seq.chunk(dev, p, plan=pl).cpu().numpy().astype(np.uint64)
        assert got.size == want.size and np.array_equal(got, want), label


@pytest.mark.parametrize("mode", [0, 1])
def test_many_covered_ranges_512mib(env, mode):
    """512 MiB uniform at an 8 KiB average in the smallest segments (64 KiB): about half the 8192 boundaries
    jump a whole segment, and the active jumps (covered ranges) outnumber the 1024 the stitch keeps in LDS
    (about 1900, counted with oracle paths from every segment start), so its walk spans many 64-jump batches
    and its range search falls back to global memory."""
    torch, seq = env
    host = synth.uniform(512 << 20, seed=3)
    dev = torch.from_numpy(host).cuda()
    p = seq.seqcdc_params_for_avg(8192)
    plan = seq.seqcdc_plan_create()
    try:
        seq.seqcdc_plan_set_tuning(plan, segment_bytes=64 << 10)
        seq.seqcdc_plan_set_mode(plan, mode)
        _say("512 MiB uniform, 64 KiB segments, mode", mode)
        got = seq.chunk(dev, p, plan=plan).cpu().numpy().astype(np.uint64)
    finally:
        seq.seqcdc_plan_destroy(plan)
    want = oracle.chunk(host, **_pd(p))
    assert got.size == want.size and np.array_equal(got, want)


@pytest.mark.parametrize("mode", [0, 1])
def test_lds_jumps_many_ranges_160mib(env, mode):
    """160 MiB alternating fast-resynchronising and never-resynchronising 64 KiB segments: 1280 jumps, at most
    the 2048 the stitch resolves in LDS in parallel, all active, more than the 1024 covered ranges it keeps in
    LDS, so its range search reads the covered ranges from global memory (counts from oracle paths in
    test_stitch_cases.py)."""
    torch, seq = env
    host = stitch_cases.alternating(160 << 20, 64 << 10)
    dev = torch.from_numpy(host).cuda()
    p = seq.seqcdc_params_for_avg(8192)
    plan = seq.seqcdc_plan_create()
    try:
        seq.seqcdc_plan_set_tuning(plan, segment_bytes=64 << 10)
        seq.seqcdc_plan_set_mode(plan, mode)
        _say("160 MiB alternating segments, 64 KiB segments, mode", mode)
        got = seq.chunk(dev, p, plan=plan).cpu().numpy().astype(np.uint64)
    finally:
        seq.seqcdc_plan_destroy(plan)
    want = oracle.chunk(host, **_pd(p))
    assert got.size == want.size and np.array_equal(got, want)


@pytest.fixture(scope="module")
def snapshots(env):
    torch, seq = env
    vers = synth.snapshot_series(256 << 20, 10, seed=0, nedits=200, maxlen=4096)
    return vers, [torch.from_numpy(v).cuda() for v in vers]


@pytest.mark.parametrize("avg_kib", [4, 8, 16, 32, 64])
def test_snapshot_series_full(env, snapshots, avg_kib):
    torch, seq = env
    vers, devs = snapshots
    p = seq.seqcdc_params_for_avg(avg_kib << 10)
    _say("snapshot series 10 x 256 MiB, avg", avg_kib, "KiB")
    outs = [o.cpu().numpy().astype(np.uint64) for o in seq.chunk_batch(devs, [p])]
    want = [oracle.chunk(v, **_pd(p)) for v in vers]
    for i, (g, w) in enumerate(zip(outs, want)):
        assert g.size == w.size and np.array_equal(g, w), i
    got = seq.seqcdc_dedup_stats(vers, outs)
    ref = oracle.dedup_stats(vers, want)
    assert got[0] == ref[0] and got[1] == ref[1]
    assert got[2] == pytest.approx(ref[2], abs=1e-12) and got[3] == pytest.approx(ref[3], rel=1e-12)
    # the same series chunked and deduplicated on the device (fingerprints, table, byte compare)
    plan = seq.seqcdc_plan_create()
    try:
        offs = [0]
        for v in vers:
            offs.append(offs[-1] + seq.seqcdc_max_cuts(v.size, p))
        d_cuts = torch.zeros(offs[-1], dtype=torch.int64, device="cuda")
        d_counts = torch.zeros(len(vers), dtype=torch.int64, device="cuda")
        files = [(d.data_ptr(), d.numel(), 0) for d in devs]
        seq.seqcdc_chunk_batch(files, [p], d_cuts.data_ptr(), offs, d_counts.data_ptr(), plan=plan)
        dev = seq.seqcdc_dedup_batch(plan, files, d_cuts.data_ptr(), offs, d_counts.data_ptr())
    finally:
        seq.seqcdc_plan_destroy(plan)
    assert dev == (ref[0], ref[1])


def test_batched_4096_files(env, direct_plan):
    torch, seq = env
    nfiles = 4096
    sizes = synth.lognormal_sizes(nfiles, 256 * 1024, 1.5, 4096, 64 << 20, seed=4).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    host = np.empty(int(offs[-1]), np.uint8)
    for f in range(nfiles):
        host[int(offs[f]):int(offs[f + 1])] = synth.mixed(int(sizes[f]), seed=100000 + f)
    buf = torch.from_numpy(host).cuda()
    p = seq.seqcdc_params_for_avg(16384)
    cut_offs = [0]
    for s in sizes:
        cut_offs.append(cut_offs[-1] + seq.seqcdc_max_cuts(int(s), p))
    cuts = torch.zeros(cut_offs[-1], dtype=torch.int64, device="cuda")
    counts = torch.zeros(nfiles, dtype=torch.int64, device="cuda")
    ftab = seq.file_table([buf.data_ptr() + int(offs[f]) for f in range(nfiles)], sizes)
    want = [oracle.chunk(host[int(offs[f]):int(offs[f + 1])], **_pd(p)) for f in range(nfiles)]

    def check(label):
        torch.cuda.synchronize()
        cnt = counts.cpu().numpy()
        allc = cuts.cpu().numpy().astype(np.uint64)
        for f in range(nfiles):
            got = allc[cut_offs[f]:cut_offs[f] + int(cnt[f])]
            assert np.array_equal(got, want[f]), (label, f)

    _say("batched 4096 files, eager")
    seq.seqcdc_chunk_batch(ftab, [p], cuts.data_ptr(), cut_offs, counts.data_ptr())
    check("eager")
    cuts.zero_()
    counts.zero_()
    _say("batched 4096 files, eager, direct mode")
    seq.seqcdc_chunk_batch(ftab, [p], cuts.data_ptr(), cut_offs, counts.data_ptr(), plan=direct_plan)
    check("eager-direct")
    cuts.zero_()
    counts.zero_()
    _say("batched 4096 files, prepared graph")
    b = seq.seqcdc_batch_prepare(ftab, [p], cuts.data_ptr(), cut_offs, counts.data_ptr())
    try:
        cuts.zero_()
        counts.zero_()
        seq.seqcdc_batch_launch(b)
        check("graph")
    finally:
        seq.seqcdc_batch_destroy(b)
