"""A second, definition-level statement of SeqCDC used only to pin the oracle.

Written separately from the oracle and in a different shape: instead of a
running byte loop it works from the per-byte facts of the vector formulation
(Sec. III-D): which pairs are favourable / opposing, which bytes end a
monotone run of SeqLength bytes, and which opposing pair is the SkipTrigger-th
one after a scan start.  Pure Python, meant for tiny inputs.
"""

NO_SKIP = 0xFFFFFFFF


def facts(b, mode, seq_length):
    n = len(b)
    if mode & 2:  # signed bytes: two's complement values -128..127
        b = [x - 256 if x >= 128 else x for x in b]
    if mode & 1 == 0:
        fav = [False] + [b[i] > b[i - 1] for i in range(1, n)]
        opp = [False] + [b[i] < b[i - 1] for i in range(1, n)]
    else:
        fav = [False] + [b[i] < b[i - 1] for i in range(1, n)]
        opp = [False] + [b[i] > b[i - 1] for i in range(1, n)]
    # run_end[q]: bytes q-SL+1 .. q strictly monotone, i.e. the SL-1 pairs ending at q are favourable
    run_end = [q >= seq_length - 1 and all(fav[i] for i in range(q - seq_length + 2, q + 1)) for q in range(n)]
    return fav, opp, run_end


def chunk(b, mode=0, seq_length=5, min_size=4096, max_size=16384, skip_trigger=50, skip_size=256):
    b = [int(x) for x in b]
    n = len(b)
    _, opp, run_end = facts(b, mode, seq_length)
    cuts = []
    c = 0
    while c < n:
        limit = min(c + max_size, n)
        start = c + min_size - seq_length  # first byte that may begin a run
        while True:
            # earliest run wholly inside [start, limit)
            candidates = [q for q in range(start + seq_length - 1, limit) if run_end[q]]
            q_end = candidates[0] if candidates else None
            # the SkipTrigger-th opposing pair whose later byte lies in (start, limit)
            q_trig = None
            if skip_trigger != NO_SKIP:
                pairs = [q for q in range(start + 1, limit) if opp[q]]
                if len(pairs) >= skip_trigger:
                    q_trig = pairs[skip_trigger - 1]
            if q_end is not None and (q_trig is None or q_end < q_trig):
                cut = q_end + 1
                break
            if q_trig is None:
                cut = limit
                break
            start = q_trig + 1 + skip_size
        cuts.append(cut)
        c = cut
    return cuts


def mark_bits(b, mode, seq_length):
    """(E, O) as Python ints with bit q set for byte q."""
    _, opp, run_end = facts([int(x) for x in b], mode, seq_length)
    E = sum(1 << q for q, v in enumerate(run_end) if v)
    O = sum(1 << q for q, v in enumerate(opp) if v)
    return E, O
