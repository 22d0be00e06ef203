"""Pins for the space-savings measure (Eq. 1) against hand-worked cases.

tests/golden/dedup_hand_worked.json holds small buffers with fixed cut lists whose original size, deduplicated
size, savings and ratio were worked out by hand from Sec. II and Eq. 1 of the paper.  The cases are chosen so that
the plausible mistakes fail: savings computed as unique/original, repeats inside one buffer not counted as
duplicates, chunks matched by length rather than content, a prefix taken for a duplicate.  Both the oracle's
routine and the library's host routine are held to them (CPU only).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _cases():
    with open(os.path.join(HERE, "golden", "dedup_hand_worked.json")) as f:
        return json.load(f)["cases"]


def _inputs(case):
    bufs = [np.frombuffer(s.encode("ascii"), dtype=np.uint8).copy() for s in case["buffers"]]
    cuts = [np.array(c, dtype=np.uint64) for c in case["cuts"]]
    return bufs, cuts


def _expect(case, got):
    orig, uniq, savings, ratio = got
    assert orig == case["orig"], case["work"]
    assert uniq == case["unique"], case["work"]
    # int / int true division is correctly rounded, as is float(Fraction): the two agree exactly
    assert savings == float(Fraction(*case["savings"])), case["work"]
    assert ratio == float(Fraction(*case["ratio"])), case["work"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["id"])
def test_oracle_dedup_hand_worked(case):
    _expect(case, oracle.dedup_stats(*_inputs(case)))


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["id"])
def test_library_dedup_hand_worked(case):
    seq = pytest.importorskip("paper_2505_21194_amd")
    _expect(case, seq.seqcdc_dedup_stats(*_inputs(case)))


def test_golden_cases_are_consistent():
    """The stored fractions follow from the stored sizes (guards the fixture itself)."""
    for c in _cases():
        assert sum(len(s) for s in c["buffers"]) == c["orig"], c["id"]
        for s, cuts in zip(c["buffers"], c["cuts"]):
            assert (not s and not cuts) or (cuts[-1] == len(s) and cuts == sorted(set(cuts))), c["id"]
        assert Fraction(*c["savings"]) == Fraction(c["orig"] - c["unique"], c["orig"]), c["id"]
        assert Fraction(*c["ratio"]) == Fraction(c["orig"], c["unique"]), c["id"]


def test_golden_distinct_chunks_by_set():
    """The stored deduplicated sizes equal the total size of the distinct chunk strings, recounted here from the
    strings themselves (a set of byte strings, independent of either routine's hashing)."""
    for c in _cases():
        distinct = set()
        for s, cuts in zip(c["buffers"], c["cuts"]):
            start = 0
            for e in cuts:
                distinct.add(s[start:e])
                start = e
        assert sum(len(x) for x in distinct) == c["unique"], c["id"]


def test_empty_input_convention():
    """No bytes at all: nothing to save (savings 0) and ratio 1 by convention (Eq. 1 is undefined there)."""
    assert oracle.dedup_stats([np.zeros(0, np.uint8)], [np.zeros(0, np.uint64)]) == (0, 0, 0.0, 1.0)
