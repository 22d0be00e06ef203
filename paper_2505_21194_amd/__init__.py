"""SeqCDC chunk-boundary detection on AMD Instinct MI355X -- Python binding of libseqcdc.

Thin ctypes marshalling over the C ABI declared in ``include/seqcdc.h``; every
step of the chunking runs in the HIP kernels of ``libseqcdc.so``.  PyTorch is
used only for device memory and streams.  There is no CPU fallback: if the
library is missing, importing the binding raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libseqcdc.so")

SEQCDC_OK = 0
SEQCDC_EINVAL = -1
SEQCDC_ECAPACITY = -2
SEQCDC_EHIP = -3
SEQCDC_EBUDGET = -4
SEQCDC_ENOMEM = -5
SEQCDC_EAGAIN = -6
SEQCDC_ENOENT = -7
SEQCDC_INCREASING = 0
SEQCDC_DECREASING = 1
SEQCDC_NO_SKIP = 0xFFFFFFFF
SEQCDC_NOALLOC_SCRATCH_BYTES = 64 << 20

_u32, _u64, _i32, _p = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p


class seqcdc_params(ctypes.Structure):
    _fields_ = [("mode", _u32), ("seq_length", _u32), ("min_size", _u64), ("max_size", _u64),
                ("skip_trigger", _u32), ("skip_size", _u32)]

    def __repr__(self):
        return ("seqcdc_params(mode=%d, seq_length=%d, min_size=%d, max_size=%d, skip_trigger=%d, skip_size=%d)"
                % (self.mode, self.seq_length, self.min_size, self.max_size, self.skip_trigger, self.skip_size))


class seqcdc_file(ctypes.Structure):
    _fields_ = [("d_data", _p), ("n", _u64), ("params_index", _u32), ("reserved", _u32)]


class seqcdc_server_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("budget_bytes", _u64), ("ring_slots", _u32), ("streams", _u32),
                ("max_batch", _u32), ("nparams", _u32), ("params", ctypes.POINTER(seqcdc_params))]


class seqcdc_result(ctypes.Structure):
    _fields_ = [("status", _i32), ("reserved", _u32), ("count", _u64), ("cuts", ctypes.POINTER(_u64)),
                ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double)]


class seqcdc_calib_stats(ctypes.Structure):
    _fields_ = [("chunks", _u64), ("max_chunks", _u64), ("mean", ctypes.c_double), ("stddev", ctypes.c_double)]


class seqcdc_pass_record(ctypes.Structure):
    _fields_ = [("requests", _u32), ("grew", _u32), ("bytes", _u64), ("wait_ms", ctypes.c_double),
                ("layout_ms", ctypes.c_double), ("gpu_ms", ctypes.c_double), ("retire_ms", ctypes.c_double)]


class SeqCDCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("seqcdc error %d: %s" % (code, msg))
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError("libseqcdc.so is not built (run __graft_entry__.build() or paper_2505_21194_amd/build.py)")
# PyTorch ships its own HIP runtime (same soname as the system one).  Loading torch first makes the library bind to
# that copy: loaded the other way round, the process would hold two HIP runtimes, and the second sees no device.
import torch  # noqa: E402,F401
lib = ctypes.CDLL(LIB_PATH)

_SIGS = {
    "seqcdc_params_validate": ([ctypes.POINTER(seqcdc_params)], ctypes.c_int),
    "seqcdc_params_for_avg": ([_u64, ctypes.POINTER(seqcdc_params)], ctypes.c_int),
    "seqcdc_max_cuts": ([_u64, ctypes.POINTER(seqcdc_params)], _u64),
    "seqcdc_plan_create": ([ctypes.c_int, ctypes.POINTER(_p)], ctypes.c_int),
    "seqcdc_plan_destroy": ([_p], ctypes.c_int),
    "seqcdc_plan_set_tuning": ([_p, _u64, _u32, _u32], ctypes.c_int),
    "seqcdc_plan_set_mode": ([_p, ctypes.c_int], ctypes.c_int),
    "seqcdc_plan_set_overlap": ([_p, _u32], ctypes.c_int),
    "seqcdc_plan_set_timing": ([_p, ctypes.c_int], ctypes.c_int),
    "seqcdc_plan_phase_ms": ([_p, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "seqcdc_plan_get_tuning": ([_p, _u64, ctypes.POINTER(seqcdc_params), ctypes.POINTER(_u64),
                                ctypes.POINTER(_u32), ctypes.POINTER(_u32)], ctypes.c_int),
    "seqcdc_autotune": ([_p, _p, _u64, ctypes.POINTER(seqcdc_params), ctypes.POINTER(ctypes.c_double), _p],
                        ctypes.c_int),
    "seqcdc_chunk": ([_p, _u64, ctypes.POINTER(seqcdc_params), _p, _u64, ctypes.POINTER(_u64), _p], ctypes.c_int),
    "seqcdc_chunk_plan": ([_p, _p, _u64, ctypes.POINTER(seqcdc_params), _p, _u64, ctypes.POINTER(_u64), _p],
                          ctypes.c_int),
    "seqcdc_chunk_batch": ([_p, ctypes.POINTER(seqcdc_file), _u32, ctypes.POINTER(seqcdc_params), _u32, _p,
                            ctypes.POINTER(_u64), _p, _p], ctypes.c_int),
    "seqcdc_autotune_batch": ([_p, ctypes.POINTER(seqcdc_file), _u32, ctypes.POINTER(seqcdc_params), _u32, _p,
                               ctypes.POINTER(_u64), _p, ctypes.POINTER(ctypes.c_double), _p], ctypes.c_int),
    "seqcdc_batch_prepare": ([_p, ctypes.POINTER(seqcdc_file), _u32, ctypes.POINTER(seqcdc_params), _u32, _p,
                              ctypes.POINTER(_u64), _p, ctypes.POINTER(_p)], ctypes.c_int),
    "seqcdc_batch_launch": ([_p, _p], ctypes.c_int),
    "seqcdc_batch_destroy": ([_p], ctypes.c_int),
    "seqcdc_mark": ([_p, _u64, ctypes.POINTER(seqcdc_params), _p, _p], ctypes.c_int),
    "seqcdc_chunk_host": ([_p, _u64, ctypes.POINTER(seqcdc_params), _p, _u64, ctypes.POINTER(_u64)], ctypes.c_int),
    "seqcdc_chunk_noalloc": ([_p, _u64, ctypes.POINTER(seqcdc_params), _p, _u64, _p, _p], ctypes.c_int),
    "seqcdc_dedup_stats": ([ctypes.POINTER(_p), ctypes.POINTER(_p), ctypes.POINTER(_u64), _u32,
                            ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "seqcdc_calibrate": ([_p, _p, _u64, ctypes.POINTER(seqcdc_params), _u32, ctypes.POINTER(seqcdc_calib_stats), _p],
                         ctypes.c_int),
    "seqcdc_dedup_batch": ([_p, ctypes.POINTER(seqcdc_file), _u32, _p, ctypes.POINTER(_u64), _p, _p,
                            ctypes.POINTER(_u64), ctypes.POINTER(_u64), _p], ctypes.c_int),
    "seqcdc_server_create": ([ctypes.POINTER(seqcdc_server_config), ctypes.POINTER(_p)], ctypes.c_int),
    "seqcdc_server_submit": ([_p, _p, _u64, _u32, ctypes.POINTER(_u64)], ctypes.c_int),
    "seqcdc_server_submit_many": ([_p, ctypes.POINTER(seqcdc_file), _u32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "seqcdc_server_poll": ([_p, _u64, ctypes.POINTER(seqcdc_result)], ctypes.c_int),
    "seqcdc_server_wait": ([_p, _u64, ctypes.c_double, ctypes.POINTER(seqcdc_result)], ctypes.c_int),
    "seqcdc_server_release": ([_p, _u64], ctypes.c_int),
    "seqcdc_server_stats": ([_p, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                             ctypes.POINTER(_u64)], ctypes.c_int),
    "seqcdc_server_timeline": ([_p, ctypes.POINTER(seqcdc_pass_record), _u32, ctypes.POINTER(_u32)], ctypes.c_int),
    "seqcdc_server_destroy": ([_p], ctypes.c_int),
    "seqcdc_last_error": ([], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTED = tuple(_SIGS)


def last_error():
    return lib.seqcdc_last_error().decode()


def _check(rc, allow=()):
    if rc != SEQCDC_OK and rc not in allow:
        raise SeqCDCError(rc, last_error())
    return rc


def make_params(mode=0, seq_length=5, min_size=4096, max_size=16384, skip_trigger=50, skip_size=256):
    return seqcdc_params(mode, seq_length, min_size, max_size, skip_trigger, skip_size)


def _as_params(p):
    if isinstance(p, seqcdc_params):
        return p
    if isinstance(p, dict):
        return make_params(**p)
    raise TypeError("params must be seqcdc_params or dict")


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ C-named wrappers
def seqcdc_params_for_avg(avg):
    p = seqcdc_params()
    _check(lib.seqcdc_params_for_avg(avg, ctypes.byref(p)))
    return p


def seqcdc_params_validate(params):
    return lib.seqcdc_params_validate(ctypes.byref(_as_params(params)))


def seqcdc_max_cuts(n, params):
    return lib.seqcdc_max_cuts(n, ctypes.byref(_as_params(params)))


def seqcdc_plan_create(device=-1):
    h = _p()
    _check(lib.seqcdc_plan_create(device, ctypes.byref(h)))
    return h


def seqcdc_plan_destroy(plan):
    _check(lib.seqcdc_plan_destroy(plan))


def seqcdc_plan_set_tuning(plan, segment_bytes=0, mark_span_blocks=0, waves_per_cu=0):
    _check(lib.seqcdc_plan_set_tuning(plan, segment_bytes, mark_span_blocks, waves_per_cu))


def seqcdc_plan_set_mode(plan, mode):
    """Resolve mode: 0 = marked (the mark kernel, then pass A, pass B, stitch and compaction; default); 1 = direct
    (skip-aware chains that read only the raw windows they scan; no mark kernel)."""
    _check(lib.seqcdc_plan_set_mode(plan, mode))


def seqcdc_plan_set_overlap(plan, groups):
    """Overlapped batches: 0 = default, 1 = off, 2..8 file groups whose marking overlaps earlier groups' chains."""
    _check(lib.seqcdc_plan_set_overlap(plan, groups))


def seqcdc_plan_set_timing(plan, on=True):
    _check(lib.seqcdc_plan_set_timing(plan, 1 if on else 0))


def seqcdc_plan_phase_ms(plan):
    """Durations (ms) of the last timed call: mark, pass A, pass B, stitch + compaction."""
    ms = (ctypes.c_float * 4)()
    _check(lib.seqcdc_plan_phase_ms(plan, ms))
    return tuple(ms)


def seqcdc_plan_get_tuning(plan, n, params):
    seg, span, waves = _u64(), _u32(), _u32()
    _check(lib.seqcdc_plan_get_tuning(plan, n, ctypes.byref(_as_params(params)), ctypes.byref(seg),
                                      ctypes.byref(span), ctypes.byref(waves)))
    return seg.value, span.value, waves.value


def seqcdc_autotune(plan, d_sample, n, params, stream=None):
    ms = ctypes.c_double()
    _check(lib.seqcdc_autotune(plan, d_sample, n, ctypes.byref(_as_params(params)), ctypes.byref(ms),
                               _stream_handle(stream)))
    return ms.value


def seqcdc_autotune_batch(plan, files, params_list, d_cuts, cut_offsets, d_counts, stream=None):
    """Tunes `plan` for this batch (arguments as for seqcdc_chunk_batch); returns the best time in ms."""
    if isinstance(files, ctypes.Array):
        farr, nf = files, getattr(files, "_len", len(files))
    else:
        farr = file_table([f[0] for f in files], [f[1] for f in files], [f[2] for f in files])
        nf = len(files)
    parr = (seqcdc_params * max(len(params_list), 1))(*[_as_params(p) for p in params_list])
    offs = cut_offsets if isinstance(cut_offsets, ctypes.Array) else offsets_table(cut_offsets)
    if len(offs) < nf + 1:
        raise ValueError("cut_offsets needs nfiles + 1 entries")
    ms = ctypes.c_double()
    _check(lib.seqcdc_autotune_batch(plan, farr, nf, parr, len(params_list), d_cuts, offs, d_counts,
                                     ctypes.byref(ms), _stream_handle(stream)))
    return ms.value


def seqcdc_chunk(d_stream, n, params, d_cuts, cap, stream=None, plan=None):
    """Raw call on device pointers; returns the cut count (raises on error, SEQCDC_ECAPACITY included)."""
    cnt = _u64()
    rc = lib.seqcdc_chunk_plan(plan, d_stream, n, ctypes.byref(_as_params(params)), d_cuts, cap,
                               ctypes.byref(cnt), _stream_handle(stream))
    if rc == SEQCDC_ECAPACITY:
        err = SeqCDCError(rc, last_error())
        err.count = cnt.value
        raise err
    _check(rc)
    return cnt.value


def seqcdc_chunk_noalloc(d_stream, n, params, d_cuts, cap, d_count, stream=None):
    """Raw allocation-free call on device pointers: enqueues the chunking of n bytes on `stream`; the count goes to
    the device uint64 at d_count (raises on argument errors, a stream too large for the fixed scratch included)."""
    _check(lib.seqcdc_chunk_noalloc(d_stream, n, ctypes.byref(_as_params(params)), d_cuts, cap, d_count,
                                    _stream_handle(stream)))


_FILE_DTYPE = None


def file_table(ptrs, sizes, params_index=None):
    """A seqcdc_file array built from sequences (or numpy arrays) of device pointers, lengths and params indices.

    Building it once and passing it to seqcdc_chunk_batch keeps per-call marshalling out of a hot loop."""
    import numpy as np
    global _FILE_DTYPE
    if _FILE_DTYPE is None:
        _FILE_DTYPE = np.dtype([("d_data", "<u8"), ("n", "<u8"), ("params_index", "<u4"), ("reserved", "<u4")])
        assert _FILE_DTYPE.itemsize == ctypes.sizeof(seqcdc_file)
    nf = len(sizes)
    a = np.zeros(max(nf, 1), dtype=_FILE_DTYPE)
    a["d_data"][:nf] = np.asarray(ptrs, dtype=np.uint64)
    a["n"][:nf] = np.asarray(sizes, dtype=np.uint64)
    if params_index is not None:
        a["params_index"][:nf] = np.asarray(params_index, dtype=np.uint32)
    arr = (seqcdc_file * max(nf, 1)).from_buffer(a)
    arr._keep = a
    arr._len = nf
    return arr


def offsets_table(offsets):
    """A uint64 array of cut offsets (nfiles + 1 entries) for seqcdc_chunk_batch."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    arr = (_u64 * a.size).from_buffer(a)
    arr._keep = a
    return arr


def seqcdc_chunk_batch(files, params_list, d_cuts, cut_offsets, d_counts, stream=None, plan=None):
    """files: list of (device_ptr, n, params_index) or a file_table(); cut_offsets: nfiles+1 host offsets
    (a sequence or an offsets_table())."""
    if isinstance(files, ctypes.Array):
        farr, nf = files, getattr(files, "_len", len(files))
    else:
        farr = file_table([f[0] for f in files], [f[1] for f in files], [f[2] for f in files])
        nf = len(files)
    parr = (seqcdc_params * max(len(params_list), 1))(*[_as_params(p) for p in params_list])
    offs = cut_offsets if isinstance(cut_offsets, ctypes.Array) else offsets_table(cut_offsets)
    if len(offs) < nf + 1:
        raise ValueError("cut_offsets needs nfiles + 1 entries")
    _check(lib.seqcdc_chunk_batch(plan, farr, nf, parr, len(params_list), d_cuts, offs, d_counts,
                                  _stream_handle(stream)))


def seqcdc_batch_prepare(files, params_list, d_cuts, cut_offsets, d_counts, settings=None):
    """A prepared (hipGraph-captured) batch; arguments as for seqcdc_chunk_batch.  Returns the handle."""
    if isinstance(files, ctypes.Array):
        farr, nf = files, getattr(files, "_len", len(files))
    else:
        farr = file_table([f[0] for f in files], [f[1] for f in files], [f[2] for f in files])
        nf = len(files)
    parr = (seqcdc_params * max(len(params_list), 1))(*[_as_params(p) for p in params_list])
    offs = cut_offsets if isinstance(cut_offsets, ctypes.Array) else offsets_table(cut_offsets)
    h = _p()
    _check(lib.seqcdc_batch_prepare(settings, farr, nf, parr, len(params_list), d_cuts, offs, d_counts,
                                    ctypes.byref(h)))
    return h


def seqcdc_batch_launch(batch, stream=None):
    _check(lib.seqcdc_batch_launch(batch, _stream_handle(stream)))


def seqcdc_batch_destroy(batch):
    _check(lib.seqcdc_batch_destroy(batch))


def seqcdc_mark(d_stream, n, params, d_eo, stream=None):
    _check(lib.seqcdc_mark(d_stream, n, ctypes.byref(_as_params(params)), d_eo, _stream_handle(stream)))


def seqcdc_server_submit_many(server, files, at_ms=None):
    """Queue requests (a file_table() or a list of (device_ptr, n, params_index)), optionally at arrival offsets in
    ms from the call; returns (tickets, submitted_ms) as numpy arrays."""
    import numpy as np
    if isinstance(files, ctypes.Array):
        farr, nf = files, getattr(files, "_len", len(files))
    else:
        farr = file_table([f[0] for f in files], [f[1] for f in files], [f[2] for f in files])
        nf = len(files)
    tickets = np.zeros(max(nf, 1), dtype=np.uint64)
    sub = np.zeros(max(nf, 1), dtype=np.float64)
    at = None
    if at_ms is not None:
        at_arr = np.ascontiguousarray(at_ms, dtype=np.float64)
        at = at_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib.seqcdc_server_submit_many(server, farr, nf, at, tickets.ctypes.data_as(ctypes.POINTER(_u64)),
                                         sub.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return tickets[:nf], sub[:nf]


def seqcdc_server_timeline(server, cap=4096):
    """The server's most recent pass records (oldest first) as a list of dicts."""
    recs = (seqcdc_pass_record * cap)()
    n = _u32()
    _check(lib.seqcdc_server_timeline(server, recs, cap, ctypes.byref(n)))
    return [{k: getattr(recs[i], k) for k, _ in seqcdc_pass_record._fields_} for i in range(n.value)]


def seqcdc_dedup_stats(buffers, cut_lists):
    """buffers: list of uint8 numpy arrays; cut_lists: list of uint64 numpy arrays (host)."""
    import numpy as np
    nb = len(buffers)
    bufs = [np.ascontiguousarray(b, dtype=np.uint8) for b in buffers]
    cuts = [np.ascontiguousarray(c, dtype=np.uint64) for c in cut_lists]
    bp = (_p * max(nb, 1))(*[b.ctypes.data for b in bufs])
    cp = (_p * max(nb, 1))(*[c.ctypes.data for c in cuts])
    cnt = (_u64 * max(nb, 1))(*[c.size for c in cuts])
    o, u, s, r = _u64(), _u64(), ctypes.c_double(), ctypes.c_double()
    _check(lib.seqcdc_dedup_stats(bp, cp, cnt, nb, ctypes.byref(o), ctypes.byref(u), ctypes.byref(s),
                                  ctypes.byref(r)))
    return o.value, u.value, s.value, r.value


def seqcdc_calibrate(plan, d_sample, n, candidates, stream=None):
    """Chunk statistics of each candidate parameter set on a device-resident sample: a list of dicts (chunks,
    max_chunks, mean, stddev)."""
    cands = [_as_params(p) for p in candidates]
    arr = (seqcdc_params * max(len(cands), 1))(*cands)
    out = (seqcdc_calib_stats * max(len(cands), 1))()
    _check(lib.seqcdc_calibrate(plan, d_sample, n, arr, len(cands), out, _stream_handle(stream)))
    return [{k: getattr(out[i], k) for k, _ in seqcdc_calib_stats._fields_} for i in range(len(cands))]


def calibrate_for_avg(plan, d_sample, n, target_avg, seq_lengths=(5, 6), triggers=(25, 35, 45, 50, 55, 65, 80),
                      skips=(128, 256, 384, 512, 768), stream=None):
    """The candidate closest to a target average chunk size on the sample (Sec. V): a grid over SeqLength,
    SkipTrigger and SkipSize with min = target/2 and max = 2 x target (Sec. VI), evaluated in one call.  Returns
    (best params, its stats, all (params, stats) pairs)."""
    grid = [make_params(0, sl, max(target_avg // 2, sl), 2 * target_avg, t, k)
            for sl in seq_lengths for t in triggers for k in skips]
    stats = seqcdc_calibrate(plan, d_sample, n, grid, stream=stream)
    best = min(range(len(grid)), key=lambda i: abs(stats[i]["mean"] - target_avg))
    return grid[best], stats[best], list(zip(grid, stats))


def seqcdc_dedup_batch(plan, files, d_cuts, cut_offsets, d_counts, d_digests=None, stream=None):
    """Device deduplication of chunked files (Eq. 1): returns (original bytes, unique bytes).  files: a
    file_table() or a list of (device_ptr, n, params_index)."""
    if isinstance(files, ctypes.Array):
        farr, nf = files, getattr(files, "_len", len(files))
    else:
        farr = file_table([f[0] for f in files], [f[1] for f in files], [f[2] for f in files])
        nf = len(files)
    offs = cut_offsets if isinstance(cut_offsets, ctypes.Array) else offsets_table(cut_offsets)
    o, u = _u64(), _u64()
    _check(lib.seqcdc_dedup_batch(plan, farr, nf, d_cuts, offs, d_counts, d_digests, ctypes.byref(o),
                                  ctypes.byref(u), _stream_handle(stream)))
    return o.value, u.value


# ------------------------------------------------------------------ torch conveniences
def chunk(data, params, stream=None, plan=None):
    """Cut offsets of a uint8 CUDA tensor as an int64 CUDA tensor (exclusive chunk ends; last == len)."""
    import torch
    assert data.is_cuda and data.dtype == torch.uint8 and data.is_contiguous()
    p = _as_params(params)
    n = data.numel()
    cap = max(seqcdc_max_cuts(n, p), 1)
    out = torch.empty(cap, dtype=torch.int64, device=data.device)
    cnt = seqcdc_chunk(data.data_ptr(), n, p, out.data_ptr(), cap, stream=stream, plan=plan)
    return out[:cnt]


def chunk_batch(tensors, params_list, params_index=None, stream=None, plan=None):
    """Chunk a list of uint8 CUDA tensors in one batched pass; returns a list of int64 CUDA tensors."""
    import torch
    ps = [_as_params(p) for p in params_list]
    if params_index is None:
        params_index = [0] * len(tensors)
    offs = [0]
    for t, pi in zip(tensors, params_index):
        offs.append(offs[-1] + max(seqcdc_max_cuts(t.numel(), ps[pi]), 1))
    dev = tensors[0].device if tensors else torch.device("cuda")
    cuts = torch.empty(max(offs[-1], 1), dtype=torch.int64, device=dev)
    counts = torch.empty(max(len(tensors), 1), dtype=torch.int64, device=dev)
    files = [(t.data_ptr(), t.numel(), pi) for t, pi in zip(tensors, params_index)]
    seqcdc_chunk_batch(files, ps, cuts.data_ptr(), offs, counts.data_ptr(), stream=stream, plan=plan)
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    cnt = counts[:len(tensors)].cpu().tolist()
    return [cuts[offs[i]:offs[i] + cnt[i]] for i in range(len(tensors))]


def mark(data, params, stream=None):
    """(E, O) bitmaps of a uint8 CUDA tensor as uint64-word numpy arrays (LSB = lowest offset)."""
    import numpy as np
    import torch
    p = _as_params(params)
    n = data.numel()
    groups = (n + 63) // 64
    eo = torch.zeros(max(4 * groups, 4), dtype=torch.int32, device=data.device)
    seqcdc_mark(data.data_ptr(), n, p, eo.data_ptr(), stream=stream)
    torch.cuda.synchronize()
    w = eo[:4 * groups].cpu().numpy().view(np.uint32).reshape(groups, 4).astype(np.uint64)
    e16 = w & 0xFFFF
    o16 = w >> 16
    E = e16[:, 0] | (e16[:, 1] << 16) | (e16[:, 2] << 32) | (e16[:, 3] << 48)
    O = o16[:, 0] | (o16[:, 1] << 16) | (o16[:, 2] << 32) | (o16[:, 3] << 48)
    return E.astype(np.uint64), O.astype(np.uint64)
