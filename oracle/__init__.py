"""SeqCDC CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded reference for what SeqCDC computes (arXiv 2505.21194,
Sec. III-A..III-D, Sec. IV) plus the space-savings measure (Eq. 1).  Only the
tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import it; the GPU library never does, and the two share no code.

``oracle_chunk`` / ``oracle_mark`` live in ``seqcdc_oracle.c`` (plain C, built
with gcc); ``dedup_stats`` is plain Python (hashlib + exact byte comparison).
"""
import ctypes
import hashlib
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "seqcdc_oracle.c")
_LIB = os.path.join(_HERE, "libseqcdc_oracle.so")
_lib = None

INCREASING = 0
DECREASING = 1
SIGNED = 2  # mode flag: compare bytes as signed values
NO_SKIP = 0xFFFFFFFF


def build(force=True):
    """Compile the C oracle with gcc (-O2, nothing else)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, p, u32 = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint
        lib.oracle_chunk.argtypes = [p, u64, u32, u32, u64, u64, u64, u64, p, u64]
        lib.oracle_chunk.restype = ctypes.c_int64
        lib.oracle_mark.argtypes = [p, u64, u32, u32, p, p]
        lib.oracle_mark.restype = ctypes.c_int
        _lib = lib
    return _lib


def _bytes(data):
    if isinstance(data, (bytes, bytearray)):
        data = np.frombuffer(data, dtype=np.uint8)
    return np.ascontiguousarray(data, dtype=np.uint8)


def chunk(data, mode=INCREASING, seq_length=5, min_size=4096, max_size=16384, skip_trigger=50, skip_size=256):
    """Exclusive chunk-end offsets of `data` (uint64 array; last == len(data))."""
    a = _bytes(data)
    n = a.size
    cap = n // max(min_size, 1) + 2
    cuts = np.empty(cap, dtype=np.uint64)
    r = _load().oracle_chunk(ctypes.c_void_p(a.ctypes.data), n, mode, seq_length, min_size, max_size,
                             skip_trigger, skip_size, ctypes.c_void_p(cuts.ctypes.data), cap)
    if r < 0:
        raise ValueError("invalid SeqCDC parameters")
    assert r <= cap
    return cuts[:r].copy()


def mark(data, mode=INCREASING, seq_length=5):
    """(E, O) bitmaps as uint64 arrays of ceil(n/64) words, LSB = lowest offset."""
    a = _bytes(data)
    words = (a.size + 63) // 64
    E = np.zeros(max(words, 1), dtype=np.uint64)
    O = np.zeros(max(words, 1), dtype=np.uint64)
    r = _load().oracle_mark(ctypes.c_void_p(a.ctypes.data), a.size, mode, seq_length,
                            ctypes.c_void_p(E.ctypes.data), ctypes.c_void_p(O.ctypes.data))
    if r < 0:
        raise ValueError("invalid SeqCDC parameters")
    return E[:words], O[:words]


def dedup_stats(buffers, cut_lists):
    """Space savings (Eq. 1) of deduplicating the chunks of `buffers` by exact content.

    Returns (original_bytes, unique_bytes, savings, ratio) with
    savings = (original - deduplicated) / original and ratio = original / deduplicated.
    Chunks are keyed by SHA-256 and confirmed equal byte for byte."""
    seen = {}
    orig = 0
    uniq = 0
    views = [memoryview(_bytes(buf)) for buf in buffers]
    for bi, cuts in enumerate(cut_lists):
        mv = views[bi]
        start = 0
        for end in cuts:
            end = int(end)
            piece = mv[start:end]
            h = hashlib.sha256(piece).digest()
            orig += end - start
            prev = seen.get(h)
            if prev is None:
                seen[h] = [(bi, start, end)]
                uniq += end - start
            elif not any(views[pb][ps:pe] == piece for pb, ps, pe in prev):
                prev.append((bi, start, end))
                uniq += end - start
            start = end
    savings = (orig - uniq) / orig if orig else 0.0
    ratio = orig / uniq if uniq else 1.0
    return orig, uniq, savings, ratio
