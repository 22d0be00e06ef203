"""Seeded synthetic workloads (bytes, sizes, arrivals) shared by tests and benchmarks.

Holds no chunking arithmetic.  The generators live in ``synth.c`` (counter-based
splitmix64 streams, OpenMP-parallel) and are loaded through ctypes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

MIX_BLOCK = 1 << 20


def build(force=True):
    """Compile libsynth.so with gcc (OpenMP)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        lib.synth_uniform.argtypes = [u64, u64, u64, p]
        lib.synth_mixed.argtypes = [u64, u64, u64, p]
        lib.synth_block_kind.argtypes = [u64, u64]
        lib.synth_block_kind.restype = ctypes.c_int
        lib.synth_draw.argtypes = [u64, u64, u64]
        lib.synth_draw.restype = u64
        lib.synth_snapshot_next.argtypes = [p, u64, u64, u64, u64, u64, p, p, u64]
        lib.synth_snapshot_next.restype = u64
        lib.synth_lognormal_sizes.argtypes = [u64, u64, ctypes.c_double, ctypes.c_double, u64, u64, p]
        lib.synth_poisson_arrivals.argtypes = [u64, u64, ctypes.c_double, p]
        lib.synth_uniform_ints.argtypes = [u64, u64, u64, u64, p]
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def uniform(n, seed=0, offset=0):
    """n uniform random bytes (uint8 array) of stream `seed` starting at `offset`."""
    out = np.empty(int(n), dtype=np.uint8)
    if n:
        _load().synth_uniform(seed, offset, int(n), _ptr(out))
    return out


def mixed(n, seed=0, offset=0):
    """n bytes of the mixed backup-like stream (1 MiB blocks: 50% uniform, 30% Zipf text, 20% low-entropy)."""
    out = np.empty(int(n), dtype=np.uint8)
    if n:
        _load().synth_mixed(seed, offset, int(n), _ptr(out))
    return out


def block_kind(seed, block):
    """0 = uniform, 1 = text-like, 2 = low-entropy for 1 MiB block `block` of the mixed stream."""
    return _load().synth_block_kind(seed, block)


def draw(seed, tag, i):
    return _load().synth_draw(seed, tag, i)


def snapshot_series(base_size, nversions, seed=0, nedits=200, maxlen=4096):
    """Backup-snapshot series: a uniform base plus versions derived by seeded edits.

    Returns a list of uint8 arrays (version 0 = base)."""
    lib = _load()
    versions = [uniform(base_size, seed=seed ^ 0x5EED)]
    fresh = np.empty(nedits * maxlen + 16, dtype=np.uint8)
    for v in range(1, nversions):
        prev = versions[-1]
        out = np.empty(prev.size + nedits * maxlen, dtype=np.uint8)
        size = lib.synth_snapshot_next(_ptr(prev), prev.size, seed, v, nedits, maxlen, _ptr(fresh), _ptr(out), out.size)
        assert size > 0
        versions.append(out[:size].copy())
    return versions


def lognormal_sizes(count, median, sigma, lo, hi, seed=0):
    out = np.empty(int(count), dtype=np.uint64)
    if count:
        _load().synth_lognormal_sizes(seed, int(count), float(median), float(sigma), int(lo), int(hi), _ptr(out))
    return out


def poisson_arrivals(count, rate, seed=0):
    out = np.empty(int(count), dtype=np.float64)
    if count:
        _load().synth_poisson_arrivals(seed, int(count), float(rate), _ptr(out))
    return out


def uniform_ints(count, bound, seed=0, tag=0):
    out = np.empty(int(count), dtype=np.uint64)
    if count:
        _load().synth_uniform_ints(seed, tag, int(count), int(bound), _ptr(out))
    return out
