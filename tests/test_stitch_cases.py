"""The stitch-path inputs do what their GPU tests rely on (oracle paths, CPU only)."""
from tests import stitch_cases


def test_alternating_jumps_160mib():
    """160 MiB in 64 KiB segments: 1280 jumps (at most the 2048 the stitch resolves in LDS), all of them active
    (more than the 1024 covered ranges it keeps in LDS)."""
    b = stitch_cases.alternating(160 << 20, 64 << 10)
    nj, nr = stitch_cases.jump_counts(b, 64 << 10, seq_length=5, min_size=4096, max_size=16384, skip_trigger=50,
                                      skip_size=256)
    assert (nj, nr) == (1280, 1280)
    assert nj <= 2048 and nr > 1024
