"""Inputs that steer the stitch step onto a chosen path, and the oracle-side count that proves they do.

A stream cut into fixed segments (the plan's forced segment length) alternates two kinds of segment:
 - even segments: constant bytes with an increasing 5-byte marker every 6 KiB.  Every chunk ends just past a
   marker, so chains from any start meet within a cut or two;
 - odd segments: a 7-byte pattern holding a run of 5 increasing bytes, repeated.  Chains that enter it at
   different phases keep different phases (chunk lengths are a fixed multiple of 7) and never meet.
So the continuation of every even chain crosses the odd segment after it and meets the chain of the next even
segment: every even boundary is a jump covering exactly one segment, and every jump is active.
"""
import numpy as np

import oracle

RUN7 = np.array([10, 20, 30, 40, 50, 5, 3], np.uint8)
MARKER = np.array([1, 2, 3, 4, 5], np.uint8)


def alternating(n, seg):
    out = np.full(n, 0x80, np.uint8)
    for k in range((n + seg - 1) // seg):
        s, e = k * seg, min(n, (k + 1) * seg)
        if k % 2:
            out[s:e] = np.resize(RUN7, e - s)
        else:
            for m in range(s + 1000, e - len(MARKER), 6144):
                out[m:m + len(MARKER)] = MARKER
    return out


def jump_counts(b, seg, **params):
    """(jumps, active ranges) of the stitch for stream b in segments of `seg` bytes, from oracle paths.

    A chain starts at each segment start.  The continuation of chain k (its cuts at or past the next segment
    start) converges at its first cut that is also a cut of the chain owning that position (one of that chain's
    cuts inside its own segment, or its segment start).  A jump is a boundary whose continuation converges in a
    chain other than k+1 (or never: the end).  The active jumps are jump 0's successors: in order, the next
    active jump is the first later one whose boundary the previous active one does not cover."""
    n = len(b)
    nseg = (n + seg - 1) // seg
    mx = params["max_size"]
    paths = {}

    def path(k):  # chain k's cuts, from its segment start through a few segments after it
        if k not in paths:
            s = k * seg
            e = min(n, s + 7 * seg)
            c = oracle.chunk(b[s:e], **params).astype(np.int64) + s
            if e < n:
                c = c[c < e - 2 * mx]  # near the slice end the limit would differ from the stream's
            paths[k] = c
        return paths[k]

    conv = []
    for k in range(nseg - 1):
        pk = path(k)
        to = nseg
        for x in pk[pk >= (k + 1) * seg]:
            o = min(int(x) // seg, nseg - 1)
            po = path(o)
            if x == o * seg or x in set(po[po < (o + 1) * seg].tolist()):
                to = o
                break
        conv.append(to)
        paths.pop(k - 1, None)
    jumps = [(k, c) for k, c in enumerate(conv) if c != k + 1]
    active, until = 0, 0
    for k, c in jumps:
        if k >= until:
            active += 1
            until = c
    return len(jumps), active
