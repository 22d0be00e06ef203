"""The allocation-free entry point (seqcdc_chunk_noalloc), called through the C ABI: its cuts equal those of
seqcdc_chunk and of the oracle, on two calls in a row, the second with a smaller input (the scratch array keeps
the first call's contents)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth


def _pd(p):
    return dict(mode=p.mode, seq_length=p.seq_length, min_size=p.min_size, max_size=p.max_size,
                skip_trigger=p.skip_trigger, skip_size=p.skip_size)


def test_noalloc_rejects_streams_beyond_the_scratch_without_gpu_work():
    import paper_2505_21194_amd as seq
    p = seq.seqcdc_params_for_avg(8192)
    rc = seq.lib.seqcdc_chunk_noalloc(ctypes.c_void_p(16), 1 << 30, ctypes.byref(p), ctypes.c_void_p(16), 1 << 20,
                                      ctypes.c_void_p(16), None)
    assert rc == seq.SEQCDC_EINVAL
    assert "scratch" in seq.last_error()
    assert seq.lib.seqcdc_chunk_noalloc(None, 16, ctypes.byref(p), None, 0, ctypes.c_void_p(16), None) == seq.SEQCDC_EINVAL
    assert seq.lib.seqcdc_chunk_noalloc(ctypes.c_void_p(16), 16, ctypes.byref(p), None, 0, None, None) == seq.SEQCDC_EINVAL


@pytest.mark.gpu
@pytest.mark.parametrize("first_mib,second_kib,avg,offset", [(48, 700, 8192, 0), (96, 9000, 16384, 3),
                                                             (20, 64, 4096, 5)])
def test_noalloc_matches_chunk(first_mib, second_kib, avg, offset):
    import torch
    import paper_2505_21194_amd as seq
    assert torch.cuda.is_available()
    p = seq.seqcdc_params_for_avg(avg)
    stream = torch.cuda.current_stream()
    for call, n in enumerate((first_mib << 20, second_kib << 10)):
        host = synth.mixed(n + offset, seed=60 + call + first_mib)[offset:]
        print("[case] noalloc call", call, "n", n, "avg", avg, "offset", offset, flush=True)
        buf = torch.from_numpy(synth.mixed(n + offset, seed=60 + call + first_mib)).cuda()
        d = buf[offset:]
        cap = seq.seqcdc_max_cuts(n, p)
        cuts = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
        count = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        seq.seqcdc_chunk_noalloc(d.data_ptr(), n, p, cuts.data_ptr(), cap, count.data_ptr(), stream=stream)
        torch.cuda.synchronize()
        cnt = int(count.item())
        got = cuts[:cnt].cpu().numpy().astype(np.uint64)
        ref = seq.chunk(d, p).cpu().numpy().astype(np.uint64)
        want = oracle.chunk(host, **_pd(p))
        assert np.array_equal(ref, want)
        assert cnt == want.size and np.array_equal(got, want), (call, cnt, want.size)
        assert bool((cuts[cnt:] == -1).all())  # nothing written past the count


@pytest.mark.gpu
def test_noalloc_short_capacity_and_empty():
    import torch
    import paper_2505_21194_amd as seq
    p = seq.seqcdc_params_for_avg(8192)
    n = 6 << 20
    host = synth.uniform(n, seed=71)
    d = torch.from_numpy(host).cuda()
    want = oracle.chunk(host, **_pd(p))
    cap = want.size // 2
    cuts = torch.full((want.size,), -1, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("[case] noalloc short capacity", flush=True)
    seq.seqcdc_chunk_noalloc(d.data_ptr(), n, p, cuts.data_ptr(), cap, count.data_ptr())
    torch.cuda.synchronize()
    assert int(count.item()) == want.size  # the required count
    assert np.array_equal(cuts[:cap].cpu().numpy().astype(np.uint64), want[:cap])
    assert bool((cuts[cap:] == -1).all())
    print("[case] noalloc empty", flush=True)
    count.fill_(7)
    seq.seqcdc_chunk_noalloc(d.data_ptr(), 0, p, cuts.data_ptr(), cap, count.data_ptr())
    torch.cuda.synchronize()
    assert int(count.item()) == 0
