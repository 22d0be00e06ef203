"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

Covers the mark bitmaps (Sec. III-D masks), the plain chunking path with speculative segments,
stitching and compaction, forced tiny segments and non-converging (periodic / zero-run) data,
ragged and tiny lengths, misaligned inputs, capacity errors and the batched path.  Every chunking
check runs in both resolve modes: marked (the mark kernel's bits) and direct (skip-aware chains over
raw windows).
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
NO_SKIP = 0xFFFFFFFF


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_21194_amd as seq
    return torch, seq


def _say(*a):
    print("[case]", *a, flush=True)


_DIRECT = {}


@pytest.fixture(scope="module", autouse=True)
def _direct_default(env):
    """A plan in the direct resolve mode with default tuning, for the second run of every check."""
    torch, seq = env
    plan = seq.seqcdc_plan_create()
    seq.seqcdc_plan_set_mode(plan, 1)
    _DIRECT["plan"] = plan
    yield
    _DIRECT.clear()
    seq.seqcdc_plan_destroy(plan)


def _dev(torch, a, offset=0):
    """Device copy of a uint8 numpy array, starting `offset` bytes into a larger allocation."""
    if offset == 0:
        return torch.from_numpy(np.ascontiguousarray(a)).cuda(), None
    big = torch.zeros(a.size + offset + 32, dtype=torch.uint8, device="cuda")
    big[offset:offset + a.size] = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return big[offset:offset + a.size], big


def _gpu_cuts(env, data, params, plan=None, offset=0):
    torch, seq = env
    t, keep = _dev(torch, data, offset)
    if data.size == 0:
        t = torch.zeros(1, dtype=torch.uint8, device="cuda")[:0]
    out = seq.chunk(t, params, plan=plan)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.uint64)


def _check(env, data, params, plan=None, offset=0, label=""):
    """The oracle's cuts from the default plan and a direct-mode plan (plan None), from each plan of a list, or
    from one plan."""
    want = oracle.chunk(data, **params)
    plans = list(plan) if isinstance(plan, (list, tuple)) else ([None, _DIRECT["plan"]] if plan is None else [plan])
    for k, pl in enumerate(plans):
        _say(label, "plan", k, "n=%d" % data.size, params, "offset=%d" % offset)
        got = _gpu_cuts(env, data, params, plan=pl, offset=offset)
        assert got.size == want.size and np.array_equal(got, want), \
            (label, k, got.size, want.size,
             np.flatnonzero(got[:min(got.size, want.size)] != want[:min(got.size, want.size)])[:5])


def P(mode=0, sl=5, mn=4096, mx=16384, trig=50, skip=256):
    return dict(mode=mode, seq_length=sl, min_size=mn, max_size=mx, skip_trigger=trig, skip_size=skip)


# ------------------------------------------------------------------ mark bitmaps
@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 63, 64, 65, 100, 1000, 1023, 1024, 1025, 2047, 4113, 24581,
                               (1 << 20) + 333])
def test_mark_bitmaps(env, n):
    torch, seq = env
    data = synth.uniform(n, seed=n)
    low = (synth.uniform(n, seed=n + 1) % 4).astype(np.uint8)  # many equal pairs and short runs
    for d, tag in ((data, "uniform"), (low, "alphabet4")):
        for sl in (2, 3, 5, 6, 9, 16):
            for mode in (0, 1, 2, 3):  # increasing / decreasing, unsigned / signed bytes
                for off in ((0, 5) if n < 5000 else (0, 13)):
                    _say("mark", tag, n, sl, mode, off)
                    t, keep = _dev(torch, d, off)
                    E, O = seq.mark(t, P(mode=mode, sl=sl, mn=16, mx=64))
                    wE, wO = oracle.mark(d, mode, sl)
                    assert np.array_equal(O, wO), ("O", tag, n, sl, mode, off)
                    assert np.array_equal(E, wE), ("E", tag, n, sl, mode, off)


# ------------------------------------------------------------------ plain path
@pytest.mark.parametrize("sl", [5, 6])
@pytest.mark.parametrize("mx", [16384, 65536])
def test_uniform_8mib(env, sl, mx):
    """8 MiB of uniform bytes (seed 0), Increasing, min 4 KiB, trigger 50, skip 256."""
    data = synth.uniform(8 << 20, seed=0)
    _check(env, data, P(sl=sl, mx=mx), label="uniform8MiB")


@pytest.mark.parametrize("avg", [8, 16, 32])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("sl", [5, 6])
def test_mixed_32mib(env, avg, mode, sl):
    data = synth.mixed(32 << 20, seed=avg + mode)
    kb = 1024
    trig, skip = (50, 256) if avg == 8 else (50, 512)
    _check(env, data, P(mode=mode, sl=sl, mn=avg * kb // 2, mx=2 * avg * kb, trig=trig, skip=skip), label="mixed")


@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("offset", [0, 5])
def test_signed_bytes(env, mode, offset):
    """The signed-byte variant (bytes compared as two's complement values), both resolve modes, several parameter
    sets, aligned and misaligned input."""
    data = synth.mixed(8 << 20, seed=60 + mode)
    for params in (P(mode=mode), P(mode=mode, sl=6, mn=8192, mx=32768, skip=512), P(mode=mode, sl=3, mn=64, mx=512,
                                                                                    trig=5, skip=17)):
        _check(env, data, params, offset=offset, label="signed")


@pytest.fixture
def tiny_plan(env):
    """64 KiB segments, in the marked and the direct resolve mode."""
    torch, seq = env
    plans = []
    for mode in (0, 1):
        plan = seq.seqcdc_plan_create()
        seq.seqcdc_plan_set_tuning(plan, segment_bytes=64 * 1024)
        seq.seqcdc_plan_set_mode(plan, mode)
        plans.append(plan)
    yield plans
    for plan in plans:
        seq.seqcdc_plan_destroy(plan)


@pytest.mark.parametrize("gen", ["uniform", "mixed"])
@pytest.mark.parametrize("params", [P(), P(sl=6), P(mode=1, mn=8192, mx=32768, skip=512), P(mn=2048, mx=8192,
                                                                                            trig=55)])
def test_forced_tiny_segments(env, tiny_plan, gen, params):
    """64 KiB segments: most boundaries need a long continuation; results must not change."""
    data = getattr(synth, gen)(12 << 20, seed=5)
    _check(env, data, params, plan=tiny_plan, label="tinyseg-" + gen)


def _periodic(n, period, seed):
    pat = synth.uniform(period, seed=seed)
    return np.resize(pat, n)


@pytest.mark.parametrize("kind", ["zeros", "periodic16", "periodic7", "ramp", "sawtooth", "descending",
                                  "zero_islands"])
def test_adversarial(env, tiny_plan, kind):
    n = 6 << 20
    if kind == "zeros":
        data = np.zeros(n, np.uint8)
    elif kind == "periodic16":
        data = _periodic(n, 16, 1)
    elif kind == "periodic7":
        data = _periodic(n, 7, 2)
    elif kind == "ramp":
        data = (np.arange(n) % 256).astype(np.uint8)
    elif kind == "sawtooth":
        data = (np.arange(n) % 9 * 28).astype(np.uint8)
    elif kind == "descending":
        data = (255 - np.arange(n) % 256).astype(np.uint8)
    else:
        data = synth.uniform(n, seed=9)
        data[(np.arange(n) // 300000) % 2 == 0] = 0
    for params in (P(), P(sl=3, mn=64, mx=4096, trig=7, skip=33), P(sl=6, trig=NO_SKIP)):
        _check(env, data, params, plan=tiny_plan, label=kind)
        _check(env, data, params, label=kind + "-default-seg")


RUN7 = np.array([10, 20, 30, 40, 50, 5, 3], np.uint8)  # a 7-byte pattern holding a run of 5 increasing bytes


def _open_cases():
    """Streams whose continuations fill their buffers (1024 cuts at these parameters) before converging: in RUN7
    repeated, every chunk ends just past a run, at the same phase of the pattern, so chunk lengths are multiples of
    7 (4096 or 4101 bytes at min 4 KiB) that do not divide the segment length, and chains from different starts keep
    different phases for ever."""
    p7 = np.resize(RUN7, 32 << 20)
    mixed = np.concatenate([np.resize(RUN7, 12 << 20), synth.uniform(8 << 20, seed=4), np.resize(RUN7[::-1], 6 << 20),
                            synth.mixed(6 << 20, seed=6)])
    return [("run7", p7), ("run7-then-random", mixed)]


@pytest.mark.parametrize("case", [0, 1])
def test_open_continuations(env, tiny_plan, case):
    """The stitch takes the open continuation on the exact path further (its overflow cuts), once per such chain;
    the result is the oracle's.  64 KiB segments: about 8k cuts (min 4 KiB) and 16k cuts (min 2 KiB, SeqLength 3,
    decreasing) against 1024-cut buffers."""
    name, data = _open_cases()[case]
    _check(env, data, P(), plan=tiny_plan, label="open-" + name)
    _check(env, data, P(mode=1, sl=3, mn=2048, mx=8192, trig=9, skip=40), plan=tiny_plan, label="open2-" + name)


@pytest.mark.parametrize("rmode", [0, 1])
def test_open_continuations_in_a_batch(env, rmode):
    torch, seq = env
    datas = [d for _, d in _open_cases()] + [synth.mixed(3 << 20, seed=7), synth.uniform(70000, seed=8)]
    params = [P()]
    plan = seq.seqcdc_plan_create()
    try:
        seq.seqcdc_plan_set_tuning(plan, segment_bytes=64 << 10)
        seq.seqcdc_plan_set_mode(plan, rmode)
        tens = [torch.from_numpy(d).cuda() for d in datas]
        _say("batch with open continuations, mode", rmode)
        outs = seq.chunk_batch(tens, params, plan=plan)
        for i, (d, o) in enumerate(zip(datas, outs)):
            assert np.array_equal(o.cpu().numpy().astype(np.uint64), oracle.chunk(d, **params[0])), i
    finally:
        seq.seqcdc_plan_destroy(plan)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 17, 63, 64, 65, 100, 1023, 1024, 1025, 4095, 4096, 4097, 65537,
                               (1 << 20) + 7])
def test_small_and_ragged(env, n):
    data = synth.uniform(n, seed=100 + n)
    for params in (P(sl=3, mn=16, mx=64, trig=3, skip=5), P(sl=2, mn=2, mx=2), P(sl=5, mn=5, mx=9, trig=1, skip=0),
                   P()):
        _check(env, data, params, label="ragged")


def test_empty_stream(env):
    torch, seq = env
    t = torch.zeros(1, dtype=torch.uint8, device="cuda")
    assert seq.seqcdc_chunk(t.data_ptr(), 0, P(), t.data_ptr(), 0) == 0


@pytest.mark.parametrize("offset", [1, 3, 8, 15])
def test_misaligned_input(env, offset):
    data = synth.mixed(3 << 20, seed=offset)
    _check(env, data, P(), offset=offset, label="misaligned")
    _check(env, data, P(sl=3, mn=64, mx=512, trig=5, skip=17), offset=offset, label="misaligned-small")


@pytest.mark.parametrize("params", [P(trig=NO_SKIP), P(trig=1, skip=0), P(trig=1, skip=4000), P(mn=5, mx=5),
                                    P(sl=16, mn=16, mx=1 << 20), P(sl=2, mn=2, mx=100, trig=2, skip=1)])
def test_parameter_extremes(env, params):
    data = synth.mixed(4 << 20, seed=77)
    _check(env, data, params, label="extremes")


def test_capacity_error(env):
    torch, seq = env
    data = synth.uniform(1 << 20, seed=4)
    want = oracle.chunk(data, **P())
    t = torch.from_numpy(data).cuda()
    out = torch.zeros(10, dtype=torch.int64, device="cuda")
    with pytest.raises(seq.SeqCDCError) as ei:
        seq.seqcdc_chunk(t.data_ptr(), t.numel(), P(), out.data_ptr(), 10)
    assert ei.value.code == seq.SEQCDC_ECAPACITY and ei.value.count == want.size
    assert np.array_equal(out.cpu().numpy().astype(np.uint64), want[:10])


@pytest.mark.parametrize("n", [0, 1, 5000, 3 << 20])
def test_chunk_host_convenience(env, n):
    """seqcdc_chunk_host: host bytes in, host cuts out (copies over PCIe around the device path)."""
    torch, seq = env
    data = synth.mixed(n, seed=31 + n)
    p = seq.make_params(**P())
    cap = max(seq.seqcdc_max_cuts(n, p), 1)
    out = np.zeros(cap, dtype=np.uint64)
    cnt = ctypes.c_uint64(99)
    src = data if data.size else np.zeros(1, np.uint8)
    rc = seq.lib.seqcdc_chunk_host(ctypes.c_void_p(src.ctypes.data), n, ctypes.byref(p),
                                   ctypes.c_void_p(out.ctypes.data), cap, ctypes.byref(cnt))
    assert rc == 0, seq.last_error()
    want = oracle.chunk(data, **P())
    assert cnt.value == want.size and np.array_equal(out[:cnt.value], want)
    if want.size > 2:  # too small an output: the required count, the first cap cuts
        short = np.zeros(2, dtype=np.uint64)
        rc = seq.lib.seqcdc_chunk_host(ctypes.c_void_p(src.ctypes.data), n, ctypes.byref(p),
                                       ctypes.c_void_p(short.ctypes.data), 2, ctypes.byref(cnt))
        assert rc == seq.SEQCDC_ECAPACITY and cnt.value == want.size
        assert np.array_equal(short, want[:2])


def test_determinism_repeated(env, tiny_plan):
    data = synth.mixed(8 << 20, seed=123)
    first = _gpu_cuts(env, data, P(), plan=tiny_plan[0])
    for _ in range(5):
        for pl in tiny_plan:
            assert np.array_equal(_gpu_cuts(env, data, P(), plan=pl), first)


def test_one_plan_alternating_layouts_and_rewritten_input(env):
    """One plan, one input buffer and one output buffer: calls alternate between two layouts (sizes and
    parameters), and same-layout calls follow a rewrite of the input bytes in place.  A call whose tables
    equal the last upload skips the copy, so every result is checked against the oracle on its own data."""
    torch, seq = env
    plan = seq.seqcdc_plan_create()
    try:
        seq.seqcdc_plan_set_tuning(plan, segment_bytes=64 << 10)
        buf = torch.empty(6 << 20, dtype=torch.uint8, device="cuda")
        layouts = [(6 << 20, P()), (5 << 20, P(mn=2048, mx=8192, trig=55))]
        cap = max(seq.seqcdc_max_cuts(n, seq.seqcdc_params(**p)) for n, p in layouts)
        out = torch.empty(cap, dtype=torch.int64, device="cuda")
        for step, (li, seed) in enumerate([(0, 1), (0, 2), (1, 3), (0, 4), (1, 5), (1, 6)]):
            n, params = layouts[li]
            data = synth.mixed(n, seed=seed)
            buf[:n].copy_(torch.from_numpy(data).cuda())
            _say("alternating layouts, step", step, "layout", li, "seed", seed)
            cnt = seq.seqcdc_chunk(buf.data_ptr(), n, seq.seqcdc_params(**params), out.data_ptr(), cap, plan=plan)
            got = out[:cnt].cpu().numpy().astype(np.uint64)
            want = oracle.chunk(data, **params)
            assert got.size == want.size and np.array_equal(got, want), (step, got.size, want.size)
    finally:
        seq.seqcdc_plan_destroy(plan)


# ------------------------------------------------------------------ batched path
@pytest.mark.parametrize("rmode", [0, 1])
@pytest.mark.parametrize("seed", [0, 1])
def test_batch_matches_oracle(env, seed, rmode):
    torch, seq = env
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in rng.integers(0, 3 << 20, 120)] + [0, 1, 64, 1023, 5000, 9 << 20]
    params = [P(), P(mode=1, sl=6, mn=8192, mx=32768, skip=512), P(sl=3, mn=64, mx=1024, trig=9, skip=40)]
    plan = seq.seqcdc_plan_create()
    seq.seqcdc_plan_set_tuning(plan, segment_bytes=256 * 1024)
    seq.seqcdc_plan_set_mode(plan, rmode)
    try:
        datas = [synth.mixed(s, seed=1000 * seed + i) for i, s in enumerate(sizes)]
        pidx = [i % len(params) for i in range(len(sizes))]
        tens = [torch.from_numpy(d).cuda() if d.size else torch.zeros(0, dtype=torch.uint8, device="cuda")
                for d in datas]
        _say("batch", len(sizes), "files", sum(sizes), "bytes")
        outs = seq.chunk_batch(tens, params, params_index=pidx, plan=plan)
        for i, (d, o) in enumerate(zip(datas, outs)):
            want = oracle.chunk(d, **params[pidx[i]])
            got = o.cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, want), (i, sizes[i])
    finally:
        seq.seqcdc_plan_destroy(plan)


def test_batch_equals_plain_per_file(env):
    torch, seq = env
    sizes = [70000, 1 << 20, 3 << 20, 12345, 2 << 20]
    datas = [synth.mixed(s, seed=40 + i) for i, s in enumerate(sizes)]
    tens = [torch.from_numpy(d).cuda() for d in datas]
    outs = seq.chunk_batch(tens, [P()])
    for t, o in zip(tens, outs):
        assert torch.equal(seq.chunk(t, P()), o)
