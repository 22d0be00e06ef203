"""Monte-Carlo calibration on the device (seqcdc_calibrate, Sec. V and Table I), through the C ABI.

* Each candidate's statistics (chunks, chunks cut at the maximum, mean, standard deviation) equal those of the
  oracle's cut list on the same uniform sample, for candidates across SeqLength, SkipTrigger, SkipSize, both modes
  and a binding maximum.
* At 256 MiB, the mean chunk size of the Table I parameter sets (SeqLength counted as bytes, 5 and 6) agrees with the
  exact first-principles expectation of the scan's Markov chain within its sampling error; this settles at scale
  which reading of SeqLength reproduces the averages Table I is said to give.
* The grid search returns the candidate closest to the target average.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_stats import expected_chunk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2505_21194_amd as seq
    plan = seq.seqcdc_plan_create()
    yield torch, seq, plan
    seq.seqcdc_plan_destroy(plan)


def _stats(cuts, n, mx):
    lens = np.diff(np.concatenate([[0], cuts.astype(np.int64)]))
    return dict(chunks=int(lens.size), max_chunks=int((lens[:-1] == mx).sum()), mean=n / lens.size,
                stddev=float(np.sqrt((lens.astype(np.float64) ** 2).mean() - (n / lens.size) ** 2)))


def test_candidates_match_oracle(env):
    torch, seq, plan = env
    n = 16 << 20
    host = synth.uniform(n, seed=17)
    dev = torch.from_numpy(host).cuda()
    cands = [dict(mode=m, seq_length=sl, min_size=mn, max_size=mx, skip_trigger=t, skip_size=k)
             for m, sl, mn, mx, t, k in [(0, 5, 4096, 16384, 50, 256), (1, 5, 4096, 16384, 50, 256),
                                         (0, 6, 4096, 16384, 50, 256), (0, 5, 1024, 8192, 55, 256),
                                         (0, 5, 8192, 32768, 50, 512), (0, 6, 8192, 12288, 40, 128),
                                         (0, 4, 2048, 4096, 0xFFFFFFFF, 0), (0, 3, 64, 1024, 9, 40)]]
    got = seq.seqcdc_calibrate(plan, dev.data_ptr(), n, cands)
    for c, g in zip(cands, got):
        want = _stats(oracle.chunk(host, **c), n, c["max_size"])
        assert g["chunks"] == want["chunks"] and g["max_chunks"] == want["max_chunks"], c
        assert g["mean"] == pytest.approx(want["mean"], rel=1e-12)
        assert g["stddev"] == pytest.approx(want["stddev"], rel=1e-9), c


@pytest.mark.parametrize("sl", [5, 6])
def test_table1_means_at_scale(env, sl):
    """Table I (SkipTrigger, SkipSize) per average with min = avg/2 (1 KiB at 4 KiB) and a maximum that never binds
    here: the measured mean against the exact expectation, within 6 standard errors."""
    torch, seq, plan = env
    n = 256 << 20
    dev = torch.from_numpy(synth.uniform(n, seed=29)).cuda()
    rows = [(1024, 55, 256), (4096, 50, 256), (8192, 50, 512)]  # (min, trigger, skip) at 4 / 8 / 16 KiB
    cands = [dict(mode=0, seq_length=sl, min_size=mn, max_size=1 << 30, skip_trigger=t, skip_size=k)
             for mn, t, k in rows]
    got = seq.seqcdc_calibrate(plan, dev.data_ptr(), n, cands)
    for (mn, t, k), g in zip(rows, got):
        mu = expected_chunk(sl, t, k, mn)
        se = g["stddev"] / math.sqrt(g["chunks"])
        assert abs(g["mean"] - mu) < 6 * se + 1.0, (sl, mn, g["mean"], mu, se)


def test_grid_search_picks_closest(env):
    torch, seq, plan = env
    n = 32 << 20
    dev = torch.from_numpy(synth.uniform(n, seed=5)).cuda()
    best, st, all_ = seq.calibrate_for_avg(plan, dev.data_ptr(), n, 8192, seq_lengths=(5, 6), triggers=(30, 50, 70),
                                           skips=(128, 256, 512))
    assert len(all_) == 18
    assert abs(st["mean"] - 8192) == min(abs(s["mean"] - 8192) for _, s in all_)
