"""Pins for the CPU oracle: what the paper and the mathematics fix, independent of the oracle itself.

* hand-worked byte strings (tests/golden/hand_worked.json, each with its passage);
* closed forms (constant data, ramps, data with no candidate run, skipping disabled);
* the mode symmetry dec(b) == inc(255 - b);
* brute force over tiny inputs against a separately written bitmap-level definition (defref);
* invariants (coverage, [min, max], determinism, resynchronisation after an insertion).
"""
import itertools
import json
import os
import random

import numpy as np
import pytest

import oracle
import synth
from tests import defref

HERE = os.path.dirname(os.path.abspath(__file__))
NO_SKIP = 0xFFFFFFFF


def _golden():
    with open(os.path.join(HERE, "golden", "hand_worked.json")) as f:
        return json.load(f)["cases"]


def _materialise(spec):
    if "list" in spec:
        return np.array(spec["list"], dtype=np.uint8)
    if "hex_runs" in spec:
        out = []
        for hx, cnt in spec["hex_runs"]:
            out += [int(hx, 16)] * cnt
        return np.array(out, dtype=np.uint8)
    if "descending_from" in spec:
        top = spec["descending_from"]
        return np.array([top - i for i in range(spec["length"])], dtype=np.uint8)
    raise ValueError(spec)


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["id"])
def test_hand_worked(case):
    data = _materialise(case["data"])
    got = oracle.chunk(data, **case["params"]).tolist()
    assert got == case["cuts"], case["work"]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["id"])
def test_hand_worked_defref(case):
    """The definition-level statement agrees with the hand-worked cuts too."""
    data = _materialise(case["data"])
    assert defref.chunk(data.tolist(), **case["params"]) == case["cuts"]


def test_paper_example_alternative_reading_differs():
    """Under 'SeqLength counts comparisons' the paper's 3-byte run would not be a boundary."""
    case = [c for c in _golden() if c["id"] == "paper_vector_example"][0]
    data = _materialise(case["data"])
    p = dict(case["params"])
    p["seq_length"] = 4  # SL + 1 bytes
    p["min_size"] = 4
    assert oracle.chunk(data, **p).tolist() != case["cuts"]


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n,mx", [(1, 8), (10, 4), (100, 7), (4096, 100), (100000, 16384)])
@pytest.mark.parametrize("value", [0, 77, 255])
def test_constant_data_cuts_every_max(n, mx, value):
    data = np.full(n, value, dtype=np.uint8)
    for mode in (0, 1):
        got = oracle.chunk(data, mode=mode, seq_length=3, min_size=3, max_size=mx, skip_trigger=1, skip_size=5)
        want = list(range(mx, n, mx)) + [n]
        assert got.tolist() == want


@pytest.mark.parametrize("sl,mn,n", [(2, 2, 256), (3, 5, 256), (5, 8, 200), (5, 64, 256), (7, 7, 100)])
def test_ramp_cuts_every_min(sl, mn, n):
    """A strictly increasing ramp: the first run of every chunk starts at its sub-minimum end."""
    inc = np.arange(n, dtype=np.uint8)
    want = list(range(mn, n, mn)) + [n]
    got = oracle.chunk(inc, mode=0, seq_length=sl, min_size=mn, max_size=10 * mn, skip_trigger=1, skip_size=3)
    assert got.tolist() == want
    got = oracle.chunk(inc[::-1].copy(), mode=1, seq_length=sl, min_size=mn, max_size=10 * mn, skip_trigger=1,
                       skip_size=3)
    assert got.tolist() == want


@pytest.mark.parametrize("trig,skip", [(1, 0), (3, 7), (50, 256), (NO_SKIP, 0)])
def test_no_candidate_run_cuts_every_max(trig, skip):
    """Data with no monotone run of SeqLength bytes (a period-2 sawtooth) is cut at the maximum only."""
    n = 50000
    data = np.tile(np.array([10, 200], dtype=np.uint8), n // 2)
    got = oracle.chunk(data, mode=0, seq_length=3, min_size=100, max_size=1000, skip_trigger=trig, skip_size=skip)
    assert got.tolist() == list(range(1000, n, 1000)) + [n]


def test_no_skip_is_first_run_end_capped():
    """Skipping disabled: each cut is one past the first run end at or after c + min - 1, capped at c + max."""
    rng = np.random.default_rng(5)
    data = rng.integers(0, 256, 300000, dtype=np.uint8)
    sl, mn, mx = 4, 700, 3000
    E, _ = oracle.mark(data, 0, sl)  # bitmaps are pinned separately (test_oracle_stats / brute force)
    ends = np.flatnonzero(np.unpackbits(E.view(np.uint8), bitorder="little")[: data.size])
    want, c = [], 0
    while c < data.size:
        i = np.searchsorted(ends, c + mn - 1)
        lim = min(c + mx, data.size)
        cut = int(ends[i]) + 1 if i < ends.size and ends[i] < lim else lim
        want.append(cut)
        c = cut
    got = oracle.chunk(data, mode=0, seq_length=sl, min_size=mn, max_size=mx, skip_trigger=NO_SKIP, skip_size=0)
    assert got.tolist() == want


# ---------------------------------------------------------------- symmetry
@pytest.mark.parametrize("params", [
    dict(seq_length=5, min_size=4096, max_size=65536, skip_trigger=50, skip_size=256),
    dict(seq_length=6, min_size=2048, max_size=8192, skip_trigger=55, skip_size=256),
    dict(seq_length=3, min_size=64, max_size=512, skip_trigger=3, skip_size=9),
])
def test_mode_symmetry(params):
    data = synth.mixed(4 << 20, seed=11)
    a = oracle.chunk(data, mode=1, **params)
    b = oracle.chunk((255 - data).astype(np.uint8), mode=0, **params)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- brute force
def _param_grid():
    for sl in (2, 3, 4):
        for mn in range(sl, 7):
            for mx in (mn, mn + 1, mn + 3, 10):
                if mx < mn:
                    continue
                for trig, skip in ((1, 0), (1, 2), (2, 1), (3, 3), (NO_SKIP, 0)):
                    yield dict(seq_length=sl, min_size=mn, max_size=mx, skip_trigger=trig, skip_size=skip)


def test_brute_force_exhaustive_tiny():
    """All strings over {0,1,2} of length <= 7 (and a fixed sample of length 7..9) under a grid of parameters."""
    grid = list(_param_grid())
    strings = []
    for n in range(0, 8):
        strings += list(itertools.product(range(3), repeat=n))
    rng = random.Random(1234)
    for n in (7, 8, 9):
        strings += [tuple(rng.randrange(4) for _ in range(n)) for _ in range(300)]
    rng2 = random.Random(99)
    checked = 0
    for s in strings:
        data = np.array(s, dtype=np.uint8)
        for p in rng2.sample(grid, 10):
            for mode in (0, 1):
                want = defref.chunk(list(s), mode=mode, **p)
                got = oracle.chunk(data, mode=mode, **p).tolist()
                assert got == want, (s, mode, p)
                checked += 1
    assert checked > 80000


def test_brute_force_random_longer():
    rng = random.Random(7)
    for _ in range(1500):
        n = rng.randrange(0, 400)
        alphabet = rng.choice([2, 3, 4, 16, 256])
        s = [rng.randrange(alphabet) for _ in range(n)]
        sl = rng.randrange(2, 8)
        mn = rng.randrange(sl, sl + 40)
        mx = rng.randrange(mn, mn + 120)
        trig = rng.choice([1, 2, 5, 20, NO_SKIP])
        skip = rng.randrange(0, 50)
        mode = rng.randrange(2)
        p = dict(seq_length=sl, min_size=mn, max_size=mx, skip_trigger=trig, skip_size=skip)
        assert oracle.chunk(np.array(s, dtype=np.uint8), mode=mode, **p).tolist() == defref.chunk(s, mode=mode, **p)


def test_mark_bitmaps_brute_force():
    rng = random.Random(3)
    for _ in range(400):
        n = rng.randrange(0, 300)
        s = [rng.randrange(rng.choice([3, 256])) for _ in range(n)]
        sl = rng.randrange(2, 17)
        mode = rng.randrange(2)
        E, O = oracle.mark(np.array(s, dtype=np.uint8), mode, sl)
        e_int = sum(int(w) << (64 * i) for i, w in enumerate(E))
        o_int = sum(int(w) << (64 * i) for i, w in enumerate(O))
        we, wo = defref.mark_bits(s, mode, sl)
        assert (e_int, o_int) == (we, wo)


def test_invalid_parameters_rejected():
    d = np.zeros(10, dtype=np.uint8)
    for bad in (dict(seq_length=1, min_size=3, max_size=4), dict(seq_length=5, min_size=4, max_size=8),
                dict(seq_length=3, min_size=8, max_size=4), dict(seq_length=3, min_size=3, max_size=4, skip_trigger=0)):
        with pytest.raises(ValueError):
            oracle.chunk(d, **bad)
    with pytest.raises(ValueError):
        oracle.chunk(d, mode=4, seq_length=3, min_size=3, max_size=4)


# ---------------------------------------------------------------- invariants
TABLE_I = {4: (5, 55, 256, 1024, 8192), 8: (5, 50, 256, 4096, 16384), 16: (5, 50, 512, 8192, 32768)}


@pytest.mark.parametrize("gen", ["uniform", "mixed"])
@pytest.mark.parametrize("avg", [4, 8, 16])
@pytest.mark.parametrize("sl_delta", [0, 1])
def test_invariants(gen, avg, sl_delta):
    sl, trig, skip, mn, mx = TABLE_I[avg]
    sl += sl_delta
    data = getattr(synth, gen)(6 << 20, seed=avg)
    for mode in (0, 1):
        cuts = oracle.chunk(data, mode=mode, seq_length=sl, min_size=mn, max_size=mx, skip_trigger=trig, skip_size=skip)
        assert cuts[-1] == data.size
        sizes = np.diff(np.concatenate([[0], cuts.astype(np.int64)]))
        assert (sizes > 0).all()
        assert (sizes[:-1] >= mn).all() and (sizes[:-1] <= mx).all()
        assert sizes[-1] <= mx
        again = oracle.chunk(data, mode=mode, seq_length=sl, min_size=mn, max_size=mx, skip_trigger=trig,
                             skip_size=skip)
        assert np.array_equal(cuts, again)


def test_empty_and_short_streams():
    assert oracle.chunk(np.zeros(0, np.uint8)).tolist() == []
    for n in range(1, 40):
        d = np.arange(n, dtype=np.uint8)
        assert oracle.chunk(d, seq_length=5, min_size=64, max_size=128).tolist() == [n]


@pytest.mark.parametrize("seed", [0, 1])
def test_resync_after_prefix_insertion(seed):
    """Sec. IV: an edit disturbs only nearby chunks; far from it the cut sets coincide again."""
    data = synth.uniform(8 << 20, seed=seed)
    ins = synth.uniform(777, seed=seed + 100)
    pos = 5000
    edited = np.concatenate([data[:pos], ins, data[pos:]])
    p = dict(seq_length=5, min_size=4096, max_size=16384, skip_trigger=50, skip_size=256)
    a = oracle.chunk(data, **p)
    b = oracle.chunk(edited, **p).astype(np.int64) - ins.size
    far = a[a > (2 << 20)]
    shared = np.isin(far, b).mean()
    assert shared > 0.99


# ---------------------------------------------------------------- signed-byte variant
def test_signed_hand_worked():
    """Bytes 0x7E 0x7F 0x80 0x81 increase as unsigned values but fall from 127 to -128 as signed ones (the 8-bit
    signed compares of Sec. III-D's intrinsics): with SeqLength 4 the unsigned reading cuts after the run, the
    signed one finds none and cuts at the maximum; SeqLength 2 finds the signed runs 0x7E 0x7F and 0x80 0x81, and
    the equal bytes after them end at the stream end."""
    b = np.array([0x7E, 0x7F, 0x80, 0x81, 0x00, 0x00, 0x00, 0x00], np.uint8)
    kw = dict(min_size=4, max_size=6, skip_trigger=oracle.NO_SKIP, skip_size=0)
    assert oracle.chunk(b, mode=0, seq_length=4, **kw).tolist() == [4, 8]
    assert oracle.chunk(b, mode=oracle.SIGNED, seq_length=4, **kw).tolist() == [6, 8]
    assert oracle.chunk(b, mode=oracle.SIGNED, seq_length=2, min_size=2, max_size=6, skip_trigger=oracle.NO_SKIP,
                        skip_size=0).tolist() == [2, 4, 8]


@pytest.mark.parametrize("mode", [0, 1])
def test_signed_is_unsigned_of_flipped_bytes(mode):
    """x < y as signed bytes exactly when (x ^ 0x80) < (y ^ 0x80) as unsigned ones (two's complement), so the signed
    variant must equal the unsigned one on the bytes with their top bit flipped."""
    data = synth.mixed(2 << 20, seed=70 + mode)
    for p in (dict(seq_length=5, min_size=4096, max_size=16384, skip_trigger=50, skip_size=256),
              dict(seq_length=3, min_size=64, max_size=1024, skip_trigger=7, skip_size=33)):
        a = oracle.chunk(data, mode=mode | oracle.SIGNED, **p)
        b = oracle.chunk(data ^ np.uint8(0x80), mode=mode, **p)
        assert np.array_equal(a, b)
    E1, O1 = oracle.mark(data, mode | oracle.SIGNED, 5)
    E2, O2 = oracle.mark(data ^ np.uint8(0x80), mode, 5)
    assert np.array_equal(E1, E2) and np.array_equal(O1, O2)


def test_signed_brute_force_around_the_sign_change():
    """All strings over {126, 127, 128, 129} up to length 7, against the definition-level reference reading the
    bytes as two's complement values."""
    for n in range(0, 8):
        for s in itertools.product((126, 127, 128, 129), repeat=n):
            b = np.array(s, np.uint8)
            for mode in (2, 3):
                for sl, mn, mx, trig, skip in ((2, 2, 5, 1, 0), (3, 3, 6, 2, 1), (3, 4, 7, defref.NO_SKIP, 0)):
                    kw = dict(mode=mode, seq_length=sl, min_size=mn, max_size=mx, skip_trigger=trig, skip_size=skip)
                    assert oracle.chunk(b, **kw).tolist() == defref.chunk(b, **kw), (s, kw)
