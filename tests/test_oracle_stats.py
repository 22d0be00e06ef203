"""Exact expectations on uniform random bytes, computed from first principles, that the oracle must reproduce.

1. Mark facts (Sec. III-D masks): for iid uniform bytes,
   P(opposing pair) = P(favourable pair) = (1 - 1/256) / 2, and
   P(a strictly increasing run of SL bytes ends at q) = C(256, SL) / 256**SL.
2. Mean chunk length: a scan from a fresh start is a Markov chain on
   (run length, last byte, opposing count); it ends in a boundary (run reaches
   SL) or a trigger (count reaches SkipTrigger).  Chunks are iid, so
   E[chunk] = (min - SL) + E[#triggers] * (E[T | trigger] + 1 + SkipSize) + E[T | boundary] + 1
   with E[#triggers] = P(trigger) / P(boundary) (Sec. III-B, III-C; the maximum
   never binds at these sizes).  The chain is iterated exactly in numpy.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _bit_density(words, n, start):
    bits = np.unpackbits(words.view(np.uint8), bitorder="little")[:n]
    return bits[start:].mean(), n - start


@pytest.mark.parametrize("sl", [2, 3, 5, 6])
def test_mark_densities(sl):
    n = 16 << 20
    data = synth.uniform(n, seed=42)
    E, O = oracle.mark(data, 0, sl)
    p_opp = (1 - 1 / 256) / 2
    p_run = math.comb(256, sl) / 256 ** sl
    d, m = _bit_density(O, n, 1)
    assert abs(d - p_opp) < 5 * math.sqrt(p_opp * (1 - p_opp) / m)
    d, m = _bit_density(E, n, sl - 1)
    # run ends at neighbouring positions are correlated; allow a generous 8 sigma of the iid error
    assert abs(d - p_run) < 8 * math.sqrt(p_run * (1 - p_run) / m), (d, p_run)
    # a wrong comparison (>= for >) would move the opposing density by 1/512 (~ 20 sigma here)


def expected_chunk(sl, trig, skip, mn):
    """Exact mean chunk length on iid uniform bytes with an unbounded maximum."""
    T = trig if trig is not None else 1
    P = np.zeros((sl - 1, T, 256))
    P[0, 0, :] = 1.0 / 256
    p_b = p_t = tb = tt = 0.0
    for t in range(1, 200000):
        cum_lt = np.cumsum(P, axis=2) - P  # mass with v < u
        cum_gt = P.sum(axis=2, keepdims=True) - np.cumsum(P, axis=2)  # mass with v > u
        new = np.zeros_like(P)
        # favourable: run grows
        new[1:, :, :] += cum_lt[:-1, :, :] / 256
        fin = cum_lt[-1].sum() / 256
        p_b += fin
        tb += t * fin
        # equal pair: run restarts
        new[0, :, :] += P.sum(axis=0) / 256
        # opposing pair: run restarts, count grows
        opp = cum_gt.sum(axis=0) / 256  # (T, 256)
        if trig is None:
            new[0, 0, :] += opp[0]
        else:
            new[0, 1:, :] += opp[:-1]
            fin = opp[-1].sum()
            p_t += fin
            tt += t * fin
        P = new
        if P.sum() < 1e-14:
            break
    e_boundary = tb / p_b
    if trig is None:
        return (mn - sl) + e_boundary + 1
    e_trigger = tt / p_t
    return (mn - sl) + (p_t / p_b) * (e_trigger + 1 + skip) + e_boundary + 1


@pytest.mark.parametrize("sl,trig,skip,mn,mx", [
    (5, 50, 256, 4096, 1 << 20),   # Table I, 8 KB row
    (5, 50, 512, 8192, 1 << 20),   # Table I, 16 KB row
    (6, 50, 256, 4096, 1 << 20),   # same with SeqLength read as comparisons
    (4, None, 0, 300, 1 << 20),    # skipping disabled
    (3, 7, 40, 100, 1 << 20),      # dense triggers, short skips
])
@pytest.mark.parametrize("mode", [0, 1])
def test_mean_chunk_matches_markov_expectation(sl, trig, skip, mn, mx, mode):
    n = 48 << 20
    data = synth.uniform(n, seed=7 + sl)
    cuts = oracle.chunk(data, mode=mode, seq_length=sl, min_size=mn, max_size=mx,
                        skip_trigger=trig if trig is not None else oracle.NO_SKIP, skip_size=skip)
    sizes = np.diff(np.concatenate([[0], cuts.astype(np.int64)]))[:-1]
    assert sizes.max() < mx  # the maximum never bound
    want = expected_chunk(sl, trig, skip, mn)
    se = sizes.std() / math.sqrt(sizes.size)
    assert abs(sizes.mean() - want) < 5 * se, (sizes.mean(), want, se)
