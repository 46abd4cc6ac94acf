"""ctypes binding of ``libraduls.so`` (argument marshalling only).

Every operation runs in the library's HIP kernels; torch tensors only carry
device memory and the current stream.  If the library is not built, loading
raises ``RuntimeError`` -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import struct

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libraduls.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, EMODEL, EDEVICE = 0, -1, -2, -3, -4, -5, -6
PROC_RADIX, PROC_LSD, PROC_BITONIC, PROC_RANK, PROC_BIG = 0, 1, 2, 3, 4
SCHED_HEURISTIC, SCHED_LEARNED, SCHED_FORCED = 0, 1, 2
MLP_F, MLP_H, MLP_P = 9, 32, 3
MLP_PARAMS = MLP_F * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_P * MLP_H + MLP_P

_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int
_f32 = ctypes.c_float


class Tuning(ctypes.Structure):
    _fields_ = [
        ("big_digit_bits", _u32),
        ("block_digit_bits", _u32),
        ("tile_records", _u32),
        ("lds_finish_max", _u32),
        ("bitonic_max", _u32),
        ("workgroups_per_cu", _u32),
        ("big_min", _u64),
        ("nontemporal", _u32),
        ("big_rule", _u32),
        ("job_records", _u32),
        ("reg_finish", _u32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TraceRow(ctypes.Structure):
    _fields_ = [
        ("features", ctypes.c_float * 9),
        ("chosen", _u32),
        ("count", _u32),
        ("observed", _u32),
        ("time_ticks", _u32 * 3),
        ("flags", _u32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("last_ms", ctypes.c_double),
        ("last_records", _u64),
        ("last_levels", _u32),
        ("sched_mode", _u32),
        ("workspace_bytes", _u64),
        ("model_params", _u64),
        ("graph_cache_entries", _u64),
    ]


TRACE_ROW_BYTES = ctypes.sizeof(TraceRow)

_SIGS = {
    "raduls_sort": (_i32, [_vp, _vp, _u64, _u32, _u32, _vp]),
    "raduls_sort_noalloc": (_i32, [_vp, _vp, _u64, _u32, _u32, _vp]),
    "raduls_tune": (_i32, [_u32, _u32, _u64, _vp]),
    "raduls_sort_segmented": (_i32, [_vp, _vp, _vp, _u32, _u64, _u32, _u32, _vp]),
    "raduls_partition": (_i32, [_vp, _vp, _u64, _u32, _u32, _u32, _u32, _vp, _vp]),
    "raduls_count_runs": (_i32, [_vp, _u64, _u32, _u32, _vp, _vp, _vp, _vp]),
    "raduls_sort_count": (_i32, [_vp, _vp, _u64, _u32, _u32, _vp, _vp, _vp, _vp]),
    "raduls_prefix_search": (_i32, [_vp, _u64, _vp, _vp, _u64, _u32, _u32, _vp, _vp, _u32, _vp]),
    "raduls_sort_search": (_i32, [_vp, _vp, _u64, _u32, _u32, _vp, _u64, _vp, _vp, _vp, _vp]),
    "raduls_sync_check": (_i32, [_vp]),
    "raduls_set_scheduler": (_i32, [_i32, _i32]),
    "raduls_get_scheduler": (_i32, [ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "raduls_load_model": (_i32, [_vp, ctypes.c_size_t]),
    "raduls_unload_model": (_i32, []),
    "raduls_set_tuning": (_i32, [ctypes.POINTER(Tuning)]),
    "raduls_get_tuning": (_i32, [ctypes.POINTER(Tuning)]),
    "raduls_default_tuning": (_i32, [_u32, _u32, _u64, ctypes.POINTER(Tuning)]),
    "raduls_effective_tuning": (_i32, [_u32, _u32, _u64, ctypes.POINTER(Tuning)]),
    "raduls_set_trace": (_i32, [_vp, _u64, _u32]),
    "raduls_trace_count": (_i32, [ctypes.POINTER(_u64), _vp]),
    "raduls_get_stats": (_i32, [ctypes.POINTER(Stats)]),
    "raduls_set_timing": (_i32, [_i32]),
    "raduls_phase_times": (_i32, [ctypes.POINTER(ctypes.c_double), _u32]),
    "raduls_last_work": (_i32, [ctypes.POINTER(_u64), _u32]),
    "raduls_workspace_bytes": (ctypes.c_size_t, [_u64, _u32, _u32]),
    "raduls_sort_inplace": (_i32, [_vp, _u64, _u32, _u32, _vp]),
    "raduls_inplace_workspace_bytes": (ctypes.c_size_t, [_u64, _u32, _u32]),
    "raduls_status_string": (ctypes.c_char_p, [_i32]),
    "raduls_last_error_message": (ctypes.c_char_p, []),
    "raduls_release": (None, []),
    "raduls_mlp_forward": (_i32, [_vp, _vp, _vp, _u32, _vp]),
    "raduls_mlp_loss_grad": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _u32, _vp]),
    "raduls_mlp_adam": (_i32, [_vp, _vp, _vp, _vp, _u32, _f32, _f32, _f32, _f32, _vp]),
}

EXPORTS = tuple(_SIGS)

_lib = None


class RadulsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def lib():
    """The loaded library (raises RuntimeError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # Device memory and streams come from PyTorch, so the library must bind
        # to the HIP runtime PyTorch loads: load that one first.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        msg = lib().raduls_last_error_message().decode(errors="replace")
        raise RadulsError(rc, msg or lib().raduls_status_string(rc).decode())


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _torch_stream(stream):
    """The torch stream object for ``stream`` (None: the current stream)."""
    import torch
    if stream is None:
        return torch.cuda.current_stream()
    if isinstance(stream, int):
        return torch.cuda.ExternalStream(stream)
    return stream


def _scratch_like(records, stream):
    """tmp for one call, allocated on the stream the call runs on, so that
    the caching allocator does not hand the block out again while the sort
    still writes to it."""
    import torch
    with torch.cuda.stream(_torch_stream(stream)):
        return torch.empty_like(records)


def _records(t):
    import torch
    if t.dtype != torch.uint8 or t.dim() != 2 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("records must be a contiguous CUDA uint8 tensor of shape (n, rec_bytes)")
    return t


def sort(records, key_bytes: int, tmp=None, stream=None, check: bool = False):
    """Sort ``records`` (uint8 [n, rec_bytes] on the GPU) in place by key.

    With ``check`` the call waits for the stream and raises if a device-side
    check failed (``raduls_sync_check``: look-back wait limit, queue
    overflow)."""
    records = _records(records)
    n, r = records.shape
    if tmp is None:
        tmp = _scratch_like(records, stream)
    _check(lib().raduls_sort(records.data_ptr(), tmp.data_ptr(), n, r, key_bytes, _stream(stream)))
    if check:
        sync_check(stream)
    return records


def sort_inplace(records, key_bytes: int, stream=None, check: bool = False):
    """Sort ``records`` by key within their own memory (``raduls_sort_inplace``):
    no ``tmp``; NOT stable -- records with equal keys end in an unspecified
    order.  ``check`` as for ``sort``."""
    records = _records(records)
    n, r = records.shape
    _check(lib().raduls_sort_inplace(records.data_ptr(), n, r, key_bytes, _stream(stream)))
    if check:
        sync_check(stream)
    return records


def sort_inplace_ptr(records_ptr: int, n: int, rec_bytes: int, key_bytes: int, stream: int) -> int:
    """Raw call returning the status code (for argument-error tests)."""
    return lib().raduls_sort_inplace(records_ptr, n, rec_bytes, key_bytes, stream)


def inplace_workspace_bytes(n: int, rec_bytes: int, key_bytes: int) -> int:
    return int(lib().raduls_inplace_workspace_bytes(n, rec_bytes, key_bytes))


NOALLOC_SCRATCH_BYTES = 64 << 20


def sort_noalloc(records, key_bytes: int, tmp, stream=None, check: bool = False):
    """``sort`` through ``raduls_sort_noalloc``: the library allocates no
    device memory (its workspace is a fixed array of NOALLOC_SCRATCH_BYTES
    per GPU), so ``tmp`` must be given."""
    records = _records(records)
    tmp = _records(tmp)
    n, r = records.shape
    if tmp.shape[0] < n or tmp.shape[1] != r:
        raise ValueError("tmp must hold at least as many records of the same size")
    _check(lib().raduls_sort_noalloc(records.data_ptr(), tmp.data_ptr(), n, r, key_bytes, _stream(stream)))
    if check:
        sync_check(stream)
    return records


def sort_ptr(records_ptr: int, tmp_ptr: int, n: int, rec_bytes: int, key_bytes: int, stream: int) -> int:
    """Raw call returning the status code (for argument-error tests)."""
    return lib().raduls_sort(records_ptr, tmp_ptr, n, rec_bytes, key_bytes, stream)


def sort_segmented(records, offsets, key_bytes: int, tmp=None, stream=None, check: bool = False):
    """Sort each segment [offsets[s], offsets[s+1]) of ``records`` independently.

    ``offsets`` is a CUDA int64/uint64 tensor of num_segs + 1 entries.  With
    ``check`` the call waits and raises on a device-side failure (invalid
    offsets included).
    """
    records = _records(records)
    n, r = records.shape
    if tmp is None:
        tmp = _scratch_like(records, stream)
    if not offsets.is_cuda or offsets.element_size() != 8 or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous 8-byte CUDA tensor")
    S = offsets.numel() - 1
    _check(lib().raduls_sort_segmented(records.data_ptr(), tmp.data_ptr(), offsets.data_ptr(), S, n, r,
                                       key_bytes, _stream(stream)))
    if check:
        sync_check(stream)
    return records


def partition(inp, out, key_bytes: int, shift: int, bits: int, counts=None, stream=None):
    """One stable counting pass on the digit (shift, bits); ``counts`` (CUDA int64 [2**bits]) optional."""
    inp = _records(inp)
    out = _records(out)
    n, r = inp.shape
    cp = counts.data_ptr() if counts is not None else None
    _check(lib().raduls_partition(inp.data_ptr(), out.data_ptr(), n, r, key_bytes, shift, bits, cp,
                                  _stream(stream)))
    return out


def _runs_outputs(records, uniq, counts, stream):
    import torch
    n = records.shape[0]
    with torch.cuda.stream(_torch_stream(stream)):
        if uniq is None:
            uniq = torch.empty_like(records)
        if counts is None:
            counts = torch.empty(n, dtype=torch.int64, device=records.device)
        num = torch.empty(1, dtype=torch.int64, device=records.device)
    uniq = _records(uniq)
    if uniq.shape[0] < n or uniq.shape[1] != records.shape[1]:
        raise ValueError("uniq must hold as many records of the same size")
    if not counts.is_cuda or counts.element_size() != 8 or not counts.is_contiguous() or counts.numel() < n:
        raise ValueError("counts must be a contiguous 8-byte CUDA tensor of at least n entries")
    return uniq, counts, num


def _runs_result(uniq, counts, num, stream, check):
    _torch_stream(stream).synchronize()
    if check:
        sync_check(stream)
    u = int(num.item())
    return uniq[:u], counts[:u]


def count_runs(sorted_records, key_bytes: int, uniq=None, counts=None, stream=None, check: bool = False):
    """Runs of equal keys in key-ordered records (``raduls_count_runs``):
    returns (first record of each run, run lengths) as views of ``uniq`` and
    ``counts`` (allocated when not given; ``uniq`` may be the input)."""
    rec = _records(sorted_records)
    n, r = rec.shape
    uniq, counts, num = _runs_outputs(rec, uniq, counts, stream)
    _check(lib().raduls_count_runs(rec.data_ptr(), n, r, key_bytes, uniq.data_ptr(), counts.data_ptr(),
                                   num.data_ptr(), _stream(stream)))
    return _runs_result(uniq, counts, num, stream, check)


def sort_count(records, key_bytes: int, tmp=None, uniq=None, counts=None, stream=None, check: bool = False):
    """Sort ``records`` in place, then count its runs (``raduls_sort_count``):
    the distinct keys in ascending order with their multiplicities.  ``uniq``
    may be ``records`` or ``tmp``."""
    rec = _records(records)
    n, r = rec.shape
    if tmp is None:
        tmp = _scratch_like(rec, stream)
    uniq, counts, num = _runs_outputs(rec, uniq, counts, stream)
    _check(lib().raduls_sort_count(rec.data_ptr(), tmp.data_ptr(), n, r, key_bytes, uniq.data_ptr(),
                                   counts.data_ptr(), num.data_ptr(), _stream(stream)))
    return _runs_result(uniq, counts, num, stream, check)


def count_runs_ptr(sorted_ptr: int, n: int, rec_bytes: int, key_bytes: int, uniq_ptr: int, counts_ptr: int,
                   num_ptr: int, stream: int) -> int:
    """Raw call returning the status code (for argument-error tests)."""
    return lib().raduls_count_runs(sorted_ptr, n, rec_bytes, key_bytes, uniq_ptr, counts_ptr, num_ptr, stream)


SEARCH_NO_NARROWING = 1


def _search_outputs(nq, device, lo, hi, stream):
    import torch
    with torch.cuda.stream(_torch_stream(stream)):
        if lo is None:
            lo = torch.empty(nq, dtype=torch.int64, device=device)
        if hi is None:
            hi = torch.empty(nq, dtype=torch.int64, device=device)
    for t in (lo, hi):
        if not t.is_cuda or t.element_size() != 8 or not t.is_contiguous() or t.numel() < nq:
            raise ValueError("lo and hi must be contiguous 8-byte CUDA tensors of at least nq entries")
    return lo, hi


def _text_sa(text, sa):
    import torch
    if text.dtype != torch.uint8 or text.dim() != 1 or not text.is_contiguous() or not text.is_cuda:
        raise ValueError("text must be a contiguous 1-D CUDA uint8 tensor")
    if sa.element_size() != 4 or sa.dim() != 1 or not sa.is_contiguous() or not sa.is_cuda or sa.numel() != text.numel():
        raise ValueError("sa must be a contiguous 1-D CUDA int32/uint32 tensor of the text's length")


def prefix_search(text, sa, queries, key_bytes: int, lo=None, hi=None, narrow: bool = True, stream=None):
    """Suffix-array range [lo, hi) of each query's key_bytes characters
    (``raduls_prefix_search``); returns (lo, hi) int64 tensors."""
    _text_sa(text, sa)
    q = _records(queries)
    nq, r = q.shape
    lo, hi = _search_outputs(nq, q.device, lo, hi, stream)
    _check(lib().raduls_prefix_search(text.data_ptr(), text.numel(), sa.data_ptr(), q.data_ptr(), nq, r, key_bytes,
                                      lo.data_ptr(), hi.data_ptr(), 0 if narrow else SEARCH_NO_NARROWING,
                                      _stream(stream)))
    return lo[:nq], hi[:nq]


def sort_search(text, sa, queries, key_bytes: int, tmp=None, lo=None, hi=None, stream=None):
    """Sort the query records in place, then search them (``raduls_sort_search``)."""
    _text_sa(text, sa)
    q = _records(queries)
    nq, r = q.shape
    if tmp is None:
        tmp = _scratch_like(q, stream)
    lo, hi = _search_outputs(nq, q.device, lo, hi, stream)
    _check(lib().raduls_sort_search(q.data_ptr(), tmp.data_ptr(), nq, r, key_bytes, text.data_ptr(), text.numel(),
                                    sa.data_ptr(), lo.data_ptr(), hi.data_ptr(), _stream(stream)))
    return lo[:nq], hi[:nq]


def prefix_search_ptr(text_ptr, text_len, sa_ptr, q_ptr, nq, rec_bytes, key_bytes, lo_ptr, hi_ptr, flags, stream) -> int:
    """Raw call returning the status code (for argument-error tests)."""
    return lib().raduls_prefix_search(text_ptr, text_len, sa_ptr, q_ptr, nq, rec_bytes, key_bytes, lo_ptr, hi_ptr,
                                      flags, stream)


def sync_check(stream=None):
    _check(lib().raduls_sync_check(_stream(stream)))


def set_scheduler(mode: int, forced_proc: int = 0):
    _check(lib().raduls_set_scheduler(mode, forced_proc))


def get_scheduler():
    m, f = _i32(), _i32()
    _check(lib().raduls_get_scheduler(ctypes.byref(m), ctypes.byref(f)))
    return m.value, f.value


def model_blob(theta, mean, scale) -> bytes:
    """Serialise a network (flat parameters, feature means and scales)."""
    import numpy as np
    theta = np.asarray(theta, dtype=np.float32).ravel()
    mean = np.asarray(mean, dtype=np.float32).ravel()
    scale = np.asarray(scale, dtype=np.float32).ravel()
    if theta.size != MLP_PARAMS or mean.size != MLP_F or scale.size != MLP_F:
        raise ValueError("wrong parameter or feature-normalisation size")
    body = b"RDLSMLP1" + struct.pack("<3I", MLP_F, MLP_H, MLP_P) + theta.tobytes() + mean.tobytes() + scale.tobytes()
    return body + struct.pack("<I", fnv1a(body))


def fnv1a(b: bytes) -> int:
    h = 2166136261
    for x in b:
        h ^= x
        h = (h * 16777619) & 0xFFFFFFFF
    return h


def load_model(blob: bytes):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(lib().raduls_load_model(ctypes.cast(buf, _vp), len(blob)))


def load_model_raw(blob: bytes) -> int:
    buf = ctypes.create_string_buffer(blob, len(blob))
    return lib().raduls_load_model(ctypes.cast(buf, _vp), len(blob))


def unload_model():
    _check(lib().raduls_unload_model())


def default_tuning(rec_bytes: int, key_bytes: int, n: int) -> Tuning:
    t = Tuning()
    _check(lib().raduls_default_tuning(rec_bytes, key_bytes, n, ctypes.byref(t)))
    return t


def set_tuning(t: Tuning | None):
    _check(lib().raduls_set_tuning(ctypes.byref(t) if t is not None else None))


def tune(rec_bytes: int, key_bytes: int, n_hint: int, stream=None) -> Tuning:
    """Run the library's autotuner for this shape and size class; returns the
    tuning later sorts of that shape and size class use."""
    _check(lib().raduls_tune(rec_bytes, key_bytes, n_hint, _stream(stream)))
    return effective_tuning(rec_bytes, key_bytes, n_hint)


def effective_tuning(rec_bytes: int, key_bytes: int, n: int) -> Tuning:
    """The tuning a sort of n records of this shape would use now."""
    t = Tuning()
    _check(lib().raduls_effective_tuning(rec_bytes, key_bytes, n, ctypes.byref(t)))
    return t


def get_tuning() -> Tuning | None:
    t = Tuning()
    rc = lib().raduls_get_tuning(ctypes.byref(t))
    return t if rc == OK else None


def set_trace(rows_tensor=None, sample_period: int = 0):
    """Trace into a CUDA uint8 tensor of capacity * 64 bytes (None: off)."""
    if rows_tensor is None:
        _check(lib().raduls_set_trace(None, 0, 0))
        return
    cap = rows_tensor.numel() * rows_tensor.element_size() // TRACE_ROW_BYTES
    _check(lib().raduls_set_trace(rows_tensor.data_ptr(), cap, sample_period))


def trace_count(stream=None) -> int:
    c = _u64()
    _check(lib().raduls_trace_count(ctypes.byref(c), _stream(stream)))
    return c.value


def get_stats() -> Stats:
    s = Stats()
    _check(lib().raduls_get_stats(ctypes.byref(s)))
    return s


def set_timing(mode):
    """0 off, 1 whole sort (Stats.last_ms), 2 whole sort and per-phase times."""
    _check(lib().raduls_set_timing(int(mode)))


PHASES = 85


def phase_names(lmax: int = 20):
    names = ["setup"]
    for l in range(20):
        names += [f"L{l}.prep", f"L{l}.hist", f"L{l}.scan", f"L{l}.scatter"]
    return names + ["order_small", "small", "small_jobs", "copy"]


def phase_times():
    """{phase name: ms} of the last sort run with timing mode 2 (zero phases dropped)."""
    arr = (ctypes.c_double * PHASES)()
    _check(lib().raduls_phase_times(arr, PHASES))
    return {n: arr[i] for i, n in enumerate(phase_names()) if arr[i] > 0}


def last_work():
    """Records handled per stage by the last sort.

    {'levels': [(in, moved), ...], 'small', 'tiny', 'copy', 'block_pass',
    'wave_jobs', 'wg_jobs', 'tiny_done', 'fin_max'}; 'fin_max' > 0 means the
    workgroup jobs were finished in registers (k_fin_jobs), else in LDS
    (k_small_jobs).
    """
    arr = (_u64 * 48)()
    _check(lib().raduls_last_work(arr, 48))
    levels = [(arr[2 * l], arr[2 * l + 1]) for l in range(20)]
    while levels and levels[-1] == (0, 0):
        levels.pop()
    return {"levels": levels, "small": arr[40], "tiny": arr[41], "copy": arr[42], "block_pass": arr[43],
            "wave_jobs": arr[44], "wg_jobs": arr[45], "tiny_done": arr[46], "fin_max": arr[47]}


def workspace_bytes(n: int, rec_bytes: int, key_bytes: int) -> int:
    return lib().raduls_workspace_bytes(n, rec_bytes, key_bytes)


def status_string(code: int) -> str:
    return lib().raduls_status_string(code).decode()


def release():
    lib().raduls_release()


def mlp_forward(X, theta, Y, stream=None):
    _check(lib().raduls_mlp_forward(X.data_ptr(), theta.data_ptr(), Y.data_ptr(), X.shape[0], _stream(stream)))


def mlp_loss_grad(X, T, M, theta, grad, loss, stream=None):
    _check(lib().raduls_mlp_loss_grad(X.data_ptr(), T.data_ptr(), M.data_ptr(), theta.data_ptr(), grad.data_ptr(),
                                      loss.data_ptr(), X.shape[0], _stream(stream)))


def mlp_adam(theta, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().raduls_mlp_adam(theta.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), t, lr, beta1, beta2,
                                 eps, _stream(stream)))
