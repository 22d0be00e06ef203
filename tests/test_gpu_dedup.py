"""Deduplication on the device (seqcdc_dedup_batch, Sec. II and Eq. 1), through the C ABI.

* Every chunk's SHA-256 equals hashlib's, for chunk lengths around the padding boundaries of FIPS 180-4
  (55/56/63/64/119/120 bytes ...), at every start alignment, including an empty chunk.
* The original and unique bytes equal the oracle's (SHA-256 plus byte compare) on backup-snapshot series chunked by
  the library, at 4..64 KiB averages, on a buffer whose chunks repeat inside it, and on hand-made chunks where a
  prefix of a chunk is not its duplicate and equal contents in different buffers are.
"""
import hashlib

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
    plan = seq.seqcdc_plan_create()
    yield torch, seq, plan
    seq.seqcdc_plan_destroy(plan)


def _pd(p):
    return dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
                skip_trigger=p.skip_trigger, skip_size=p.skip_size)


def _digest_words(d):
    return np.frombuffer(d, dtype=">u4").astype(np.uint32)


def test_sha256_matches_hashlib(env):
    torch, seq, plan = env
    lens = [0, 1, 2, 3, 4, 5, 31, 55, 56, 57, 63, 64, 65, 119, 120, 121, 127, 128, 129, 191, 192, 1000, 4095,
            4096, 4097, 65539]
    host = synth.uniform(sum(lens) * 2 + 64, seed=90)
    files, cut_lists = [], []
    for shift in range(5):  # chunk starts at every alignment: the buffer begins `shift` bytes into its allocation
        cuts = np.cumsum([0] + lens[1:] + [lens[0]]).astype(np.uint64)[1:]  # the empty chunk last
        files.append((shift, cuts))
    dev = torch.from_numpy(host).cuda()
    ptrs = [dev.data_ptr() + shift for shift, _ in files]
    sizes = [int(c[-1]) for _, c in files]
    offs = [0]
    for _, c in files:
        offs.append(offs[-1] + c.size)
    d_cuts = torch.from_numpy(np.concatenate([c for _, c in files]).astype(np.int64)).cuda()
    d_counts = torch.tensor([c.size for _, c in files], dtype=torch.int64, device="cuda")
    dig = torch.zeros(offs[-1] * 8, dtype=torch.int32, device="cuda")
    orig, uniq = seq.seqcdc_dedup_batch(plan, [(p, n, 0) for p, n in zip(ptrs, sizes)], d_cuts.data_ptr(), offs,
                                        d_counts.data_ptr(), d_digests=dig.data_ptr())
    got = dig.cpu().numpy().view(np.uint32).reshape(-1, 8)
    for fi, (shift, cuts) in enumerate(files):
        start = 0
        for j, end in enumerate(cuts):
            piece = host[shift + start:shift + int(end)].tobytes()
            want = _digest_words(hashlib.sha256(piece).digest())
            assert np.array_equal(got[offs[fi] + j], want), (shift, j, int(end) - start)
            start = int(end)
    bufs = [host[s:s + n] for (s, _), n in zip(files, sizes)]
    o2, u2, _, _ = oracle.dedup_stats(bufs, [c for _, c in files])
    assert (orig, uniq) == (o2, u2)


@pytest.mark.parametrize("avg_kib", [4, 8, 16, 32, 64])
def test_snapshot_dedup_on_device(env, avg_kib):
    """Config 3 shape at reduced size: a 24 MiB uniform base and 4 versions of 200 seeded edits each, chunked by
    the batched path, deduplicated on the device; original and unique bytes equal the oracle's exactly."""
    torch, seq, plan = env
    vers = synth.snapshot_series(24 << 20, 5, seed=33, nedits=200, maxlen=4096)
    p = seq.seqcdc_params_for_avg(avg_kib << 10)
    devs = [torch.from_numpy(v).cuda() for v in vers]
    offs = [0]
    for v in vers:
        offs.append(offs[-1] + seq.seqcdc_max_cuts(v.size, p))
    d_cuts = torch.zeros(offs[-1], dtype=torch.int64, device="cuda")
    d_counts = torch.zeros(len(vers), dtype=torch.int64, device="cuda")
    files = [(d.data_ptr(), d.numel(), 0) for d in devs]
    seq.seqcdc_chunk_batch(files, [p], d_cuts.data_ptr(), offs, d_counts.data_ptr(), plan=plan)
    orig, uniq = seq.seqcdc_dedup_batch(plan, files, d_cuts.data_ptr(), offs, d_counts.data_ptr())
    cnt = d_counts.cpu().numpy()
    allc = d_cuts.cpu().numpy().astype(np.uint64)
    cuts = [allc[offs[i]:offs[i] + int(cnt[i])] for i in range(len(vers))]
    for v, c in zip(vers, cuts):
        assert np.array_equal(c, oracle.chunk(v, **_pd(p)))
    o2, u2, s2, r2 = oracle.dedup_stats(vers, cuts)
    assert (orig, uniq) == (o2, u2)
    # some repeats across the versions, fewer than the edits alone would leave: after an edit the boundaries take
    # tens of chunks (hundreds of KB at 8 KiB, megabytes at 32 KiB) to resynchronise, so 200 edits disturb much of
    # a 24 MiB version; at most 4 of 5 copies can be saved
    assert 0.0 < s2 < 0.8


def test_repeats_inside_one_buffer(env):
    """Periodic content: most chunks of a single buffer repeat each other exactly."""
    torch, seq, plan = env
    pat = synth.uniform(5000, seed=3)
    host = np.concatenate([np.resize(pat, 3 << 20), synth.uniform(1 << 20, seed=4), np.resize(pat, 2 << 20)])
    p = seq.make_params(mode=0, seq_length=5, min_size=4096, max_size=16384, skip_trigger=50, skip_size=256)
    dev = torch.from_numpy(host).cuda()
    offs = [0, seq.seqcdc_max_cuts(host.size, p)]
    d_cuts = torch.zeros(offs[-1], dtype=torch.int64, device="cuda")
    d_counts = torch.zeros(1, dtype=torch.int64, device="cuda")
    files = [(dev.data_ptr(), host.size, 0)]
    seq.seqcdc_chunk_batch(files, [p], d_cuts.data_ptr(), offs, d_counts.data_ptr(), plan=plan)
    orig, uniq = seq.seqcdc_dedup_batch(plan, files, d_cuts.data_ptr(), offs, d_counts.data_ptr())
    cuts = d_cuts.cpu().numpy().astype(np.uint64)[:int(d_counts.item())]
    o2, u2, s2, _ = oracle.dedup_stats([host], [cuts])
    assert (orig, uniq) == (o2, u2) and s2 > 0.3


def test_prefix_is_not_a_duplicate(env):
    """The same 64 bytes appear three times and their first 32 bytes twice, across two buffers: a prefix of a chunk
    is not its duplicate, equal contents in different buffers are (Eq. 1: 320 original bytes, 96 unique)."""
    torch, seq, plan = env
    a = synth.uniform(64, seed=8)
    bufs = [np.concatenate([a, a[:32], a]), np.concatenate([a[:32], a, a])]
    cut_lists = [np.array([64, 96, 160], np.uint64), np.array([32, 96, 160], np.uint64)]
    devs = [torch.from_numpy(b).cuda() for b in bufs]
    offs = [0, 3, 6]
    d_cuts = torch.from_numpy(np.concatenate(cut_lists).astype(np.int64)).cuda()
    d_counts = torch.tensor([3, 3], dtype=torch.int64, device="cuda")
    files = [(d.data_ptr(), d.numel(), 0) for d in devs]
    orig, uniq = seq.seqcdc_dedup_batch(plan, files, d_cuts.data_ptr(), offs, d_counts.data_ptr())
    o2, u2, _, _ = oracle.dedup_stats(bufs, cut_lists)
    assert (orig, uniq) == (o2, u2) == (320, 96)  # unique: a (64) and a[:32] (32)
