"""CPU-only checks of the C-ABI library: it loads, exports every symbol the header declares, and its
host-side logic (parameter validation, Table I parameters, bounds, dedup statistics) behaves.
No GPU compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "seqcdc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(seqcdc_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def seq():
    import paper_2505_21194_amd as seq
    return seq


def test_library_exports_every_declared_symbol(seq):
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(seq.lib, name), name
    assert set(names) == set(seq.EXPORTED)


def test_params_for_avg_table_i(seq):
    # Table I: SeqLength 5; SkipTrigger/SkipSize 55/256, 50/256, 50/512; Sec. VI: min avg/2 (1 KiB at 4 KiB), max 2*avg
    want = {4096: (5, 55, 256, 1024, 8192), 8192: (5, 50, 256, 4096, 16384), 16384: (5, 50, 512, 8192, 32768),
            32768: (5, 50, 512, 16384, 65536)}
    for avg, (sl, trig, skip, mn, mx) in want.items():
        p = seq.seqcdc_params_for_avg(avg)
        assert (p.seq_length, p.skip_trigger, p.skip_size, p.min_size, p.max_size, p.mode) == (sl, trig, skip, mn, mx, 0)
    with pytest.raises(seq.SeqCDCError):
        seq.seqcdc_params_for_avg(5000)


def test_validation(seq):
    ok = seq.make_params()
    assert seq.seqcdc_params_validate(ok) == 0
    bad = [dict(seq_length=1), dict(seq_length=17), dict(min_size=3, seq_length=5), dict(min_size=100, max_size=50),
           dict(skip_trigger=0), dict(mode=4)]
    for b in bad:
        p = dict(mode=0, seq_length=5, min_size=4096, max_size=16384, skip_trigger=50, skip_size=256)
        p.update(b)
        assert seq.seqcdc_params_validate(p) == seq.SEQCDC_EINVAL
        assert seq.last_error()
    assert seq.lib.seqcdc_params_validate(None) == seq.SEQCDC_EINVAL


def test_max_cuts(seq):
    p = seq.make_params(min_size=4096)
    assert seq.seqcdc_max_cuts(0, p) == 0
    assert seq.seqcdc_max_cuts(1, p) == 1
    assert seq.seqcdc_max_cuts(4096, p) == 2
    assert seq.seqcdc_max_cuts(1 << 30, p) == (1 << 30) // 4096 + 1


def test_null_arguments_rejected_without_gpu_work(seq):
    cnt = ctypes.c_uint64(123)
    p = seq.make_params()
    assert seq.lib.seqcdc_chunk(None, 0, ctypes.byref(p), None, 0, ctypes.byref(cnt), None) == 0
    assert cnt.value == 0  # empty stream: no cuts, no device work
    assert seq.lib.seqcdc_chunk(None, 10, ctypes.byref(p), None, 0, ctypes.byref(cnt), None) == seq.SEQCDC_EINVAL
    assert seq.lib.seqcdc_chunk(None, 10, None, None, 0, ctypes.byref(cnt), None) == seq.SEQCDC_EINVAL


def test_dedup_stats_matches_oracle(seq):
    """The library's host dedup routine (Eq. 1) against the oracle's, on oracle cut lists."""
    import oracle
    import synth
    vers = synth.snapshot_series(1 << 20, 4, seed=3, nedits=20, maxlen=4096)
    p = dict(seq_length=5, min_size=1024, max_size=8192, skip_trigger=55, skip_size=256)
    cuts = [oracle.chunk(v, **p) for v in vers]
    want = oracle.dedup_stats(vers, cuts)
    got = seq.seqcdc_dedup_stats(vers, cuts)
    assert got[0] == want[0] and got[1] == want[1]
    assert got[2] == pytest.approx(want[2], abs=0, rel=1e-15)
    assert want[2] > 0.5  # four near-identical versions deduplicate well


def test_new_entry_points_reject_bad_arguments_without_gpu_work(seq):
    """Plan knobs, prepared batches and diagnostics check their arguments before touching a device."""
    E = seq.SEQCDC_EINVAL
    assert seq.lib.seqcdc_plan_set_overlap(None, 2) == E
    assert seq.lib.seqcdc_plan_set_mode(None, 0) == E
    assert seq.lib.seqcdc_plan_set_timing(None, 1) == E
    assert seq.lib.seqcdc_plan_phase_ms(None, None) == E
    assert seq.lib.seqcdc_batch_launch(None, None) == E
    assert seq.lib.seqcdc_batch_destroy(None) == E
    out = ctypes.c_void_p(123)
    p = seq.make_params()
    f = (seq.seqcdc_file * 1)(seq.seqcdc_file(None, 0, 0, 0))
    offs = (ctypes.c_uint64 * 2)(0, 1)
    # no output handle; no files
    assert seq.lib.seqcdc_batch_prepare(None, f, 1, ctypes.byref(p), 1, None, offs, None, None) == E
    assert seq.lib.seqcdc_batch_prepare(None, f, 0, ctypes.byref(p), 1, None, offs, None, ctypes.byref(out)) == E
    assert out.value is None  # cleared on failure
    # NULL outputs, bad params index
    assert seq.lib.seqcdc_batch_prepare(None, f, 1, ctypes.byref(p), 1, None, offs, None, ctypes.byref(out)) == E
    f2 = (seq.seqcdc_file * 1)(seq.seqcdc_file(None, 0, 5, 0))
    assert seq.lib.seqcdc_batch_prepare(None, f2, 1, ctypes.byref(p), 1, ctypes.c_void_p(16), offs, ctypes.c_void_p(16),
                                        ctypes.byref(out)) == E
    assert "params_index" in seq.last_error()
