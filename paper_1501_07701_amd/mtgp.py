"""ctypes binding of the C ABI in ``include/mtgp.h``.

Argument marshalling only: every step of generation runs in the HIP library
(``_build/libmtgp.so``).  Device buffers are passed as raw addresses; torch
tensors are accepted wherever a device buffer is expected and only their
``data_ptr()`` is used.  Streams are ``torch.cuda.Stream`` objects, raw
``hipStream_t`` integers, or None (the current torch stream).

If the library has not been built, the first call raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# The in-tree build; MTGP_LIBRARY may name another build of the same sources.
LIB_PATH = os.environ.get("MTGP_LIBRARY") or os.path.join(_HERE, "_build", "libmtgp.so")
PARAM_WORDS = 53
DEVICE_PARAM_BYTES = 4096
NOALLOC_SCRATCH_BYTES = 64 << 20
U32, F32 = 0, 1
PENDING, DONE, FAILED = 0, 1, 2

OK, EINVAL, ENOMEM, EDEVICE, ETOOBIG, EAGAIN, ENOENT, ECANCELED, ETIMEDOUT = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)


class MTGPError(RuntimeError):
    def __init__(self, code: int, func: str, detail: str):
        super().__init__("%s failed: %s (%d): %s" % (func, _strerror(code), code, detail))
        self.code = code


class Work(ctypes.Structure):
    _fields_ = [("stream_id", ctypes.c_int32), ("dtype", ctypes.c_uint32),
                ("count", ctypes.c_uint64), ("d_out", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("threads_per_stream", ctypes.c_int), ("outputs_per_lane", ctypes.c_int),
                ("workgroup_size", ctypes.c_int), ("jump_target_steps", ctypes.c_int),
                ("window_below_w", ctypes.c_int)]

    def as_tuple(self):
        return (self.threads_per_stream, self.outputs_per_lane, self.workgroup_size,
                self.jump_target_steps, self.window_below_w)

    def __repr__(self):
        return "Tuning(tps=%d, k=%d, wg=%d, jump=%d, window_below=%d)" % self.as_tuple()


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_inflight_batches", ctypes.c_int), ("max_batch_items", ctypes.c_int),
                ("max_queue", ctypes.c_int), ("batch_window_ns", ctypes.c_uint64),
                ("workspace_bytes_per_batch", ctypes.c_uint64)]


_lib = None
_lock = threading.Lock()

_VP, _U32P, _U64P, _INTP = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                            ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int))
_SIGS = {
    "mtgp_state_words": ([ctypes.c_uint32], ctypes.c_int),
    "mtgp_check_params": ([_VP, ctypes.c_int], ctypes.c_int),
    "mtgp_init_states": ([_VP, _VP, ctypes.c_int, _VP, _VP, ctypes.c_int, _VP], ctypes.c_int),
    "mtgp_load_params": ([_VP, ctypes.c_int, _VP, _VP], ctypes.c_int),
    "mtgp_seed_states": ([_VP, _VP, ctypes.c_int, ctypes.c_int, _VP], ctypes.c_int),
    "mtgp_release_params": ([_VP], ctypes.c_int),
    "mtgp_generate_u32": ([_VP, _VP, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _VP, _VP],
                          ctypes.c_int),
    "mtgp_generate_f32": ([_VP, _VP, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _VP, _VP],
                          ctypes.c_int),
    "mtgp_batch_workspace_bytes": ([ctypes.c_int], ctypes.c_size_t),
    "mtgp_batch_workspace_query": ([_VP, ctypes.POINTER(Work), ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "mtgp_generate_batch": ([_VP, _VP, ctypes.c_int, ctypes.POINTER(Work), ctypes.c_int, _VP,
                             ctypes.c_size_t, _VP], ctypes.c_int),
    "mtgp_batch_errors": ([_VP, _VP, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
    "mtgp_generate_batch_noalloc": ([_VP, _VP, ctypes.c_int, ctypes.POINTER(Work), ctypes.c_int,
                                     _VP], ctypes.c_int),
    "mtgp_get_tuning": ([ctypes.c_uint32, ctypes.POINTER(Tuning)], ctypes.c_int),
    "mtgp_set_tuning": ([ctypes.c_uint32, ctypes.POINTER(Tuning)], ctypes.c_int),
    "mtgp_tuning_candidates": ([ctypes.c_uint32, ctypes.POINTER(Tuning), ctypes.c_int],
                               ctypes.c_int),
    "mtgp_autotune": ([_VP, _VP, ctypes.c_int, ctypes.POINTER(Work), ctypes.c_int, _VP,
                       ctypes.c_size_t, ctypes.c_int, _VP, ctypes.POINTER(Tuning),
                       ctypes.POINTER(ctypes.c_float), ctypes.c_int], ctypes.c_int),
    "mtgp_state_export": ([_VP, _VP, ctypes.c_int, ctypes.c_int, _VP, _VP], ctypes.c_int),
    "mtgp_state_import": ([_VP, _VP, ctypes.c_int, ctypes.c_int, _VP, _VP], ctypes.c_int),
    "mtgp_generate_workgroup": ([_VP, _VP, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_int, ctypes.c_int, _VP, _VP], ctypes.c_int),
    "mtgp_stream_polynomials": ([_VP, ctypes.c_int, _VP, ctypes.c_int, _VP, _VP],
                                ctypes.c_int),
    "mtgp_screen": ([_VP, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                     ctypes.c_int, _VP, _VP], ctypes.c_int),
    "mtgp_fill_u32": ([_VP, ctypes.c_uint64, ctypes.c_uint32, _VP], ctypes.c_int),
    "mtgp_server_create": ([_VP, _VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_uint64,
                            ctypes.POINTER(ServerOpts), ctypes.POINTER(ctypes.c_void_p)],
                           ctypes.c_int),
    "mtgp_submit": ([_VP, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int, _U64P], ctypes.c_int),
    "mtgp_submit_many": ([_VP, _VP, _VP, _VP, ctypes.c_int, _VP], ctypes.c_int),
    "mtgp_server_replay": ([_VP, _VP, _VP, _VP, _VP, ctypes.c_int, _VP, _VP, _VP],
                           ctypes.c_int),
    "mtgp_server_repaired": ([_VP, _U64P], ctypes.c_int),
    "mtgp_poll": ([_VP, ctypes.c_uint64, _INTP, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "mtgp_wait": ([_VP, ctypes.c_uint64, ctypes.c_uint64], ctypes.c_int),
    "mtgp_release": ([_VP, ctypes.c_uint64], ctypes.c_int),
    "mtgp_request_times": ([_VP, ctypes.c_uint64, _U64P, _U64P, _U64P, _U64P], ctypes.c_int),
    "mtgp_server_destroy": ([_VP], ctypes.c_int),
    "mtgp_set_phase_timing": ([ctypes.c_int], ctypes.c_int),
    "mtgp_batch_phase_times": ([_VP, _VP, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "mtgp_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "mtgp_last_error_detail": ([], ctypes.c_char_p),
}


def lib():
    """The loaded HIP library; raises if it was never built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "MTGP HIP library not built (%s missing); run "
                    "`python -m paper_1501_07701_amd.build` or __graft_entry__.build()" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            for name, (args, res) in _SIGS.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = res
            _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().mtgp_strerror(code).decode()
    except Exception:  # library missing while formatting an error
        return "error"


def _check(rc: int, func: str) -> int:
    if rc < 0:
        raise MTGPError(rc, func, lib().mtgp_last_error_detail().decode())
    return rc


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    raise TypeError("cannot take the address of %r" % type(x))


def _stream(s) -> int:
    if s is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def _host_params(params: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(params, dtype=np.uint32)
    if p.ndim != 2 or p.shape[1] != PARAM_WORDS:
        raise ValueError("params must be (n, %d) uint32" % PARAM_WORDS)
    return p


# ----------------------------------------------------------------- core ---

def state_words(mexp: int) -> int:
    return _check(lib().mtgp_state_words(mexp), "mtgp_state_words")


def check_params(params: np.ndarray) -> None:
    p = _host_params(params)
    _check(lib().mtgp_check_params(_ptr(p), p.shape[0]), "mtgp_check_params")


def init_states(params: np.ndarray, seeds: np.ndarray, d_params, d_states, stride: int,
                stream=None) -> None:
    p = _host_params(params)
    s = np.ascontiguousarray(seeds, dtype=np.uint32)
    if s.shape != (p.shape[0],):
        raise ValueError("one seed per stream")
    _check(lib().mtgp_init_states(_ptr(p), _ptr(s), p.shape[0], _ptr(d_params), _ptr(d_states),
                                  stride, _stream(stream)), "mtgp_init_states")


def seed_states(d_params, d_states, stride: int, n_streams: int, stream=None) -> None:
    _check(lib().mtgp_seed_states(_ptr(d_params), _ptr(d_states), stride, n_streams,
                                  _stream(stream)), "mtgp_seed_states")


def load_params(params: np.ndarray, d_params, stream=None) -> None:
    p = _host_params(params)
    _check(lib().mtgp_load_params(_ptr(p), p.shape[0], _ptr(d_params), _stream(stream)),
           "mtgp_load_params")


def release_params(d_params) -> None:
    _check(lib().mtgp_release_params(_ptr(d_params)), "mtgp_release_params")


def generate(d_params, d_states, stride: int, n_streams: int, count: int, d_out,
             dtype: int = U32, stream=None) -> None:
    fn = lib().mtgp_generate_f32 if dtype == F32 else lib().mtgp_generate_u32
    _check(fn(_ptr(d_params), _ptr(d_states), stride, n_streams, count, _ptr(d_out),
              _stream(stream)), "mtgp_generate_%s" % ("f32" if dtype == F32 else "u32"))


def batch_workspace_bytes(n_items: int) -> int:
    return int(lib().mtgp_batch_workspace_bytes(n_items))


def make_work(items) -> ctypes.Array:
    """items: iterable of (stream_id, dtype, count, d_out)."""
    items = list(items)
    arr = (Work * max(len(items), 1))()
    for i, (sid, dt, cnt, out) in enumerate(items):
        arr[i] = Work(int(sid), int(dt), int(cnt), _ptr(out))
    return arr, len(items)


def _nbytes(t) -> int:
    if hasattr(t, "numel"):
        return int(t.numel() * t.element_size())
    raise TypeError("pass workspace_bytes for a raw workspace address")


def batch_workspace_query(d_params, items) -> int:
    arr, n = items if isinstance(items, tuple) else make_work(items)
    out = ctypes.c_size_t()
    _check(lib().mtgp_batch_workspace_query(_ptr(d_params), arr, n, ctypes.byref(out)),
           "mtgp_batch_workspace_query")
    return int(out.value)


def generate_batch(d_params, d_states, stride: int, items, d_workspace, stream=None,
                   workspace_bytes=None) -> None:
    arr, n = items if isinstance(items, tuple) else make_work(items)
    wsb = _nbytes(d_workspace) if workspace_bytes is None else int(workspace_bytes)
    _check(lib().mtgp_generate_batch(_ptr(d_params), _ptr(d_states), stride, arr, n,
                                     _ptr(d_workspace), wsb, _stream(stream)),
           "mtgp_generate_batch")


def generate_batch_noalloc(d_params, d_states, stride: int, items, stream=None) -> None:
    """mtgp_generate_batch with the library's static device scratch as the
    workspace (no allocation)."""
    arr, n = items if isinstance(items, tuple) else make_work(items)
    _check(lib().mtgp_generate_batch_noalloc(_ptr(d_params), _ptr(d_states), stride, arr, n,
                                             _stream(stream)),
           "mtgp_generate_batch_noalloc")


def batch_errors(d_workspace, stream=None) -> int:
    n = ctypes.c_uint32()
    _check(lib().mtgp_batch_errors(_ptr(d_workspace), _stream(stream), ctypes.byref(n)),
           "mtgp_batch_errors")
    return int(n.value)


def set_phase_timing(enable: bool) -> None:
    _check(lib().mtgp_set_phase_timing(1 if enable else 0), "mtgp_set_phase_timing")


def batch_phase_times(d_workspace, stream=None):
    """(prefix-and-jump launch, segments, request checks) durations in
    microseconds of the last batch call on the workspace that ran with phase
    timing enabled."""
    us = (ctypes.c_double * 3)()
    _check(lib().mtgp_batch_phase_times(_ptr(d_workspace), _stream(stream), us),
           "mtgp_batch_phase_times")
    return tuple(us)


def get_tuning(mexp: int) -> Tuning:
    t = Tuning()
    _check(lib().mtgp_get_tuning(mexp, ctypes.byref(t)), "mtgp_get_tuning")
    return t


def set_tuning(mexp: int, tps: int, k: int, wg: int, jump_target_steps=None,
               window_below_w=None) -> None:
    """Sets the launch tuning of an exponent; the jump target and the window
    threshold keep their current values unless given."""
    cur = get_tuning(mexp)
    if jump_target_steps is None:
        jump_target_steps = cur.jump_target_steps
    if window_below_w is None:
        window_below_w = cur.window_below_w
    t = Tuning(tps, k, wg, jump_target_steps, window_below_w)
    _check(lib().mtgp_set_tuning(mexp, ctypes.byref(t)), "mtgp_set_tuning")


def tuning_candidates(mexp: int):
    n = _check(lib().mtgp_tuning_candidates(mexp, None, 0), "mtgp_tuning_candidates")
    arr = (Tuning * n)()
    _check(lib().mtgp_tuning_candidates(mexp, arr, n), "mtgp_tuning_candidates")
    return [arr[i] for i in range(n)]


def autotune(d_params, d_states, stride: int, items, d_scratch, reps: int = 2, stream=None,
             scratch_bytes=None):
    """Times every compiled candidate (then jump targets) on this batch;
    returns (best, per-candidate ms)."""
    arr, n = items if isinstance(items, tuple) else make_work(items)
    best = Tuning()
    ms = (ctypes.c_float * 64)()
    sb = _nbytes(d_scratch) if scratch_bytes is None else int(scratch_bytes)
    _check(lib().mtgp_autotune(_ptr(d_params), _ptr(d_states), stride, arr, n, _ptr(d_scratch),
                               sb, reps, _stream(stream), ctypes.byref(best), ms, 64),
           "mtgp_autotune")
    return best, list(ms)


def state_export(d_params, d_states, stride: int, n_streams: int, n_words: int,
                 stream=None) -> np.ndarray:
    out = np.zeros((n_streams, n_words), dtype=np.uint32)
    _check(lib().mtgp_state_export(_ptr(d_params), _ptr(d_states), stride, n_streams, _ptr(out),
                                   _stream(stream)), "mtgp_state_export")
    return out


def state_import(d_params, d_states, stride: int, host_states: np.ndarray, stream=None) -> None:
    h = np.ascontiguousarray(host_states, dtype=np.uint32)
    _check(lib().mtgp_state_import(_ptr(d_params), _ptr(d_states), stride, h.shape[0], _ptr(h),
                                   _stream(stream)), "mtgp_state_import")


def generate_workgroup(d_params, d_states, stride: int, n_streams: int, count: int, d_out,
                       dtype: int = U32, threads: int = 256, stream=None) -> None:
    """Generation through the device-side draw API (one workgroup per
    stream); out[k * count + j] as for generate()."""
    _check(lib().mtgp_generate_workgroup(_ptr(d_params), _ptr(d_states), stride, n_streams,
                                         count, dtype, threads, _ptr(d_out), _stream(stream)),
           "mtgp_generate_workgroup")


def stream_polynomials(d_params, n_streams: int, mexp: int, stream=None):
    """(degrees (n,) int32, coefficients (n, mexp//32+1) uint32): the
    minimal polynomial of each stream's output sequence from its seed."""
    words = mexp // 32 + 1
    coeffs = np.zeros((n_streams, words), dtype=np.uint32)
    degrees = np.zeros(n_streams, dtype=np.int32)
    _check(lib().mtgp_stream_polynomials(_ptr(d_params), n_streams, coeffs.ctypes.data, words,
                                         degrees.ctypes.data, _stream(stream)),
           "mtgp_stream_polynomials")
    return degrees, coeffs


def screen(d_outputs, n_streams: int, count: int, gap_lo: int, gap_hi: int, gap_bins: int,
           d_counts, stream=None) -> None:
    """Gap-test and Hamming-weight-dependency counts per stream into
    d_counts (n_streams x (gap_bins + 9) uint64 on the device)."""
    _check(lib().mtgp_screen(_ptr(d_outputs), n_streams, count, gap_lo, gap_hi, gap_bins,
                             _ptr(d_counts), _stream(stream)), "mtgp_screen")


def fill_u32(d_out, n_words: int, value: int, stream=None) -> None:
    _check(lib().mtgp_fill_u32(_ptr(d_out), n_words, value & 0xFFFFFFFF, _stream(stream)),
           "mtgp_fill_u32")


# ------------------------------------------------------------- helpers ---

class Generators:
    """A parameter set with its device-resident states, allocated with torch.

    params: (n, 53) uint32 host array; seeds: (n,) uint32."""

    def __init__(self, params: np.ndarray, seeds: np.ndarray, device="cuda", stride=None):
        import torch
        self.params = _host_params(params)
        self.n = self.params.shape[0]
        self.mexp = int(self.params[0, 0])
        self.N = state_words(self.mexp)
        self.stride = int(stride) if stride else self.N
        self.device = torch.device(device)
        self.d_params = torch.empty(self.n * DEVICE_PARAM_BYTES, dtype=torch.uint8,
                                    device=self.device)
        self.d_states = torch.empty(self.n * self.stride, dtype=torch.int32, device=self.device)
        init_states(self.params, seeds, self.d_params, self.d_states, self.stride)

    def generate(self, count: int, dtype: int = U32, out=None, n_streams=None, stream=None):
        import torch
        n = self.n if n_streams is None else n_streams
        if out is None:
            out = torch.empty(n * count, dtype=torch.float32 if dtype == F32 else torch.int32,
                              device=self.device)
        generate(self.d_params, self.d_states, self.stride, n, count, out, dtype, stream)
        return out

    def reseed(self, stream=None) -> None:
        seed_states(self.d_params, self.d_states, self.stride, self.n, stream)

    def states_host(self) -> np.ndarray:
        return state_export(self.d_params, self.d_states, self.stride, self.n, self.N)

    def load_states(self, host_states: np.ndarray) -> None:
        state_import(self.d_params, self.d_states, self.stride, host_states)

    def workspace(self, items):
        """Device workspace sized for `items` (a list, or a count for the
        minimum without jump-ahead splitting)."""
        import torch
        if isinstance(items, int):
            nbytes = batch_workspace_bytes(items)
        else:
            nbytes = batch_workspace_query(self.d_params, list(items))
        return torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def batch(self, items, workspace=None, stream=None):
        items = list(items)
        ws = self.workspace(items) if workspace is None else workspace
        generate_batch(self.d_params, self.d_states, self.stride, items, ws, stream)
        return ws

    def close(self):
        try:
            release_params(self.d_params)
        except MTGPError:
            pass


class Server:
    """Serving loop over the resident states of `gens` (a Generators).

    pool_bytes of device memory are allocated with torch for outputs and
    launch workspaces; requests are admitted while their outputs fit."""

    def __init__(self, gens: Generators, pool_bytes: int, inflight: int = 4,
                 max_batch_items: int = 256, max_queue: int = 1 << 20,
                 batch_window_ns: int = 20000, workspace_bytes_per_batch: int = 64 << 20):
        import torch
        self.gens = gens
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=gens.device)
        opts = ServerOpts(inflight, max_batch_items, max_queue, batch_window_ns,
                          workspace_bytes_per_batch)
        h = ctypes.c_void_p()
        _check(lib().mtgp_server_create(_ptr(gens.d_params), _ptr(gens.d_states), gens.stride,
                                        gens.n, _ptr(self.pool), int(pool_bytes),
                                        ctypes.byref(opts), ctypes.byref(h)),
               "mtgp_server_create")
        self.h = h

    def submit(self, stream_id: int, count: int, dtype: int = U32) -> int:
        t = ctypes.c_uint64()
        _check(lib().mtgp_submit(self.h, int(stream_id), int(count), int(dtype),
                                 ctypes.byref(t)), "mtgp_submit")
        return int(t.value)

    def submit_many(self, stream_ids, counts, dtypes) -> np.ndarray:
        """Queues all requests in one call; returns their tickets."""
        st = np.ascontiguousarray(stream_ids, dtype=np.int32)
        ct = np.ascontiguousarray(counts, dtype=np.uint64)
        dt = np.ascontiguousarray(dtypes, dtype=np.int32)
        tk = np.zeros(st.shape[0], dtype=np.uint64)
        _check(lib().mtgp_submit_many(self.h, st.ctypes.data, ct.ctypes.data, dt.ctypes.data,
                                      int(st.shape[0]), tk.ctypes.data), "mtgp_submit_many")
        return tk

    def replay(self, t_arrival_ns, stream_ids, counts, dtypes, keep=None):
        """Replays a request trace (native submission at the arrival times);
        returns (latency ns (n,), stages ns (n, 3): queued, admitted, running).
        keep: optional sequence of n device addresses (0 = drop) where the
        results of chosen requests are copied."""
        ta = np.ascontiguousarray(t_arrival_ns, dtype=np.uint64)
        st = np.ascontiguousarray(stream_ids, dtype=np.int32)
        ct = np.ascontiguousarray(counts, dtype=np.uint64)
        dt = np.ascontiguousarray(dtypes, dtype=np.int32)
        n = int(ta.shape[0])
        lat = np.zeros(n, dtype=np.uint64)
        stg = np.zeros((n, 3), dtype=np.uint64)
        kp = None
        if keep is not None:
            kp = np.ascontiguousarray([_ptr(x) for x in keep], dtype=np.uint64)
            if kp.shape[0] != n:
                raise ValueError("keep needs one entry per request")
        _check(lib().mtgp_server_replay(self.h, ta.ctypes.data, st.ctypes.data, ct.ctypes.data,
                                        dt.ctypes.data, n, lat.ctypes.data, stg.ctypes.data,
                                        kp.ctypes.data if kp is not None else None),
               "mtgp_server_replay")
        return lat, stg

    def repaired(self) -> int:
        """Requests regenerated after a failed jump-ahead segment check."""
        v = ctypes.c_uint64()
        _check(lib().mtgp_server_repaired(self.h, ctypes.byref(v)), "mtgp_server_repaired")
        return int(v.value)

    def poll(self, ticket: int):
        st = ctypes.c_int()
        ptr = ctypes.c_void_p()
        _check(lib().mtgp_poll(self.h, ticket, ctypes.byref(st), ctypes.byref(ptr)), "mtgp_poll")
        return int(st.value), (int(ptr.value) if ptr.value else 0)

    def wait(self, ticket: int, timeout_ns: int = 0) -> None:
        _check(lib().mtgp_wait(self.h, ticket, int(timeout_ns)), "mtgp_wait")

    def release(self, ticket: int) -> None:
        _check(lib().mtgp_release(self.h, ticket), "mtgp_release")

    def times(self, ticket: int):
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(lib().mtgp_request_times(self.h, ticket, *[ctypes.byref(x) for x in v]),
               "mtgp_request_times")
        return tuple(int(x.value) for x in v)

    def result(self, ticket: int, count: int, dtype: int = U32):
        """Copy of a finished request's outputs as a torch tensor."""
        import torch
        state, ptr = self.poll(ticket)
        if state != DONE:
            raise RuntimeError("ticket %d not done" % ticket)
        off = ptr - self.pool.data_ptr()
        raw = self.pool[off:off + 4 * count].clone()
        return raw.view(torch.float32 if dtype == F32 else torch.int32)

    def close(self) -> None:
        if self.h:
            h, self.h = self.h, None
            _check(lib().mtgp_server_destroy(h), "mtgp_server_destroy")
        self.pool = None  # the output pool's device memory goes back to torch
