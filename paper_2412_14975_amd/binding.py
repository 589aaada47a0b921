"""ctypes binding of libri.so (include/ri.h), with the C names.

Argument marshalling only: every step of recognition runs in the library's
HIP kernels.  Texts are torch uint8 tensors on the GPU; streams are
``torch.cuda.Stream`` objects (default: torch's current stream).  There is no
CPU path: without the built library or without a GPU tensor these functions
raise.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime that libri.so binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libri.so")

RI_OK, RI_ERR_PARSE, RI_ERR_LIMIT, RI_ERR_NOMEM, RI_ERR_DEVICE, RI_ERR_ARG = 0, -1, -2, -3, -4, -5
RI_ALGO_RID, RI_ALGO_DFA, RI_ALGO_SUBSET, RI_ALGO_NFA = 0, 1, 2, 3
RI_NUM_ALGOS = 4
ALGOS = {"rid": RI_ALGO_RID, "dfa": RI_ALGO_DFA, "subset": RI_ALGO_SUBSET, "nfa": RI_ALGO_NFA}

SYMBOLS = ("ri_build", "ri_free", "ri_info", "ri_recognize", "ri_recognize_ex",
           "ri_recognize_async", "ri_chunk_maps", "ri_state_content", "ri_set_profiling", "ri_last_timings",
           "ri_set_option", "ri_get_option", "ri_autotune", "ri_last_error",
           "ri_batch_create", "ri_batch_free", "ri_batch_run", "ri_batch_capture",
           "ri_batch_launch", "ri_batch_get_info", "ri_batch_get_group", "ri_batch_autotune",
           "ri_batch_create_ex", "ri_batch_update", "ri_request_footprint", "ri_recognize_noalloc")
RI_BATCH_AUTO, RI_BATCH_GROUPED, RI_BATCH_FUSED, RI_BATCH_QUEUE = 0, 1, 2, 3
BATCH_MODES = {"auto": RI_BATCH_AUTO, "grouped": RI_BATCH_GROUPED, "fused": RI_BATCH_FUSED,
               "queue": RI_BATCH_QUEUE}
RI_OPT_CONVERGE, RI_OPT_WARMUP_BYTES, RI_OPT_RUNS_PER_LANE, RI_OPT_CHUNK_TARGET, RI_OPT_JOIN = 1, 2, 3, 4, 5
RI_OPT_PREFIX = 6
OPTIONS = {"converge": RI_OPT_CONVERGE, "warmup_bytes": RI_OPT_WARMUP_BYTES,
           "runs_per_lane": RI_OPT_RUNS_PER_LANE, "chunk_target": RI_OPT_CHUNK_TARGET,
           "join": RI_OPT_JOIN, "prefix": RI_OPT_PREFIX}


class RIError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class ri_build_opts(ctypes.Structure):
    _fields_ = [("max_states", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class ri_result(ctypes.Structure):
    _fields_ = [("accept", ctypes.c_int32), ("final_state", ctypes.c_int32),
                ("n", ctypes.c_uint64), ("chunks", ctypes.c_uint32),
                ("chunk_size", ctypes.c_uint32)]


class ri_tuning(ctypes.Structure):
    _fields_ = [("chunk_target", ctypes.c_uint32), ("warmup_bytes", ctypes.c_uint32),
                ("runs_per_lane", ctypes.c_uint32), ("trials", ctypes.c_uint32),
                ("best_ms", ctypes.c_float), ("converge", ctypes.c_uint32)]


class ri_info_t(ctypes.Structure):
    _fields_ = [("nfa_states", ctypes.c_uint32), ("interface_states", ctypes.c_uint32),
                ("ridfa_states", ctypes.c_uint32), ("ridfa_full_states", ctypes.c_uint32),
                ("min_dfa_states", ctypes.c_uint32), ("subset_dfa_states", ctypes.c_uint32),
                ("classes", ctypes.c_uint32), ("accepts_empty", ctypes.c_uint32),
                ("starts", ctypes.c_uint32 * RI_NUM_ALGOS),
                ("entry_bytes", ctypes.c_uint32 * RI_NUM_ALGOS),
                ("table_bytes", ctypes.c_uint64 * RI_NUM_ALGOS),
                ("prefix_depth", ctypes.c_uint32 * RI_NUM_ALGOS),
                ("prefix_states", ctypes.c_uint32 * RI_NUM_ALGOS)]


class ri_request(ctypes.Structure):
    _fields_ = [("h", ctypes.c_void_p), ("text_dev", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("algo", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


class ri_batch_info(ctypes.Structure):
    _fields_ = [("texts", ctypes.c_uint32), ("groups", ctypes.c_uint32), ("slots", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("kernels", ctypes.c_uint32), ("captured", ctypes.c_uint32), ("fused", ctypes.c_uint32),
                ("queue", ctypes.c_uint32)]


class ri_batch_opts(ctypes.Structure):
    _fields_ = [("chunk_bytes", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("warmup_bytes", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ri_batch_group(ctypes.Structure):
    _fields_ = [("h", ctypes.c_void_p), ("algo", ctypes.c_int32), ("texts", ctypes.c_uint32),
                ("slots", ctypes.c_uint32), ("bytes", ctypes.c_uint64),
                ("chunk_bytes", ctypes.c_uint32), ("warmup_bytes", ctypes.c_uint32),
                ("runs_per_lane", ctypes.c_uint32), ("join_levels", ctypes.c_uint32),
                ("tuned_ms", ctypes.c_float)]


class ri_batch_tuning(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_uint32), ("best_ms", ctypes.c_float)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libri.so (built by ``__graft_entry__.build()``); raise if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, u32, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_int
    L.ri_build.argtypes = [ctypes.c_char_p, sz, ctypes.POINTER(ri_build_opts), ctypes.POINTER(vp)]
    L.ri_free.argtypes = [vp]
    L.ri_free.restype = None
    L.ri_info.argtypes = [vp, ctypes.POINTER(ri_info_t)]
    L.ri_recognize.argtypes = [vp, vp, sz, vp, ctypes.POINTER(ri_result)]
    L.ri_recognize_ex.argtypes = [vp, vp, sz, vp, i32, u32, ctypes.POINTER(ri_result)]
    L.ri_recognize_async.argtypes = [vp, vp, sz, vp, i32, u32, vp]
    L.ri_recognize_noalloc.argtypes = [vp, vp, sz, vp, i32, u32, vp]
    L.ri_chunk_maps.argtypes = [vp, vp, sz, vp, i32, u32, vp, sz, ctypes.POINTER(ri_result)]
    L.ri_state_content.argtypes = [vp, i32, u32, ctypes.POINTER(u32), u32, ctypes.POINTER(u32)]
    L.ri_set_profiling.argtypes = [vp, i32]
    L.ri_last_timings.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    L.ri_set_option.argtypes = [vp, i32, ctypes.c_int64]
    L.ri_get_option.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64)]
    L.ri_autotune.argtypes = [vp, vp, sz, vp, i32, ctypes.POINTER(ri_tuning)]
    L.ri_batch_create.argtypes = [ctypes.POINTER(ri_request), u32, u32, ctypes.POINTER(vp)]
    L.ri_batch_create_ex.argtypes = [ctypes.POINTER(ri_request), u32, ctypes.POINTER(ri_batch_opts), ctypes.POINTER(vp)]
    L.ri_batch_update.argtypes = [vp, ctypes.POINTER(ri_request), u32]
    L.ri_request_footprint.argtypes = [vp, i32, ctypes.c_uint64, u32, ctypes.POINTER(ctypes.c_uint64)]
    L.ri_batch_free.argtypes = [vp]
    L.ri_batch_free.restype = None
    L.ri_batch_run.argtypes = [vp, vp, vp]
    L.ri_batch_capture.argtypes = [vp, vp]
    L.ri_batch_launch.argtypes = [vp, vp]
    L.ri_batch_get_info.argtypes = [vp, ctypes.POINTER(ri_batch_info)]
    L.ri_batch_get_group.argtypes = [vp, u32, ctypes.POINTER(ri_batch_group)]
    L.ri_batch_autotune.argtypes = [vp, vp, ctypes.POINTER(ri_batch_tuning)]
    L.ri_last_error.argtypes = []
    L.ri_last_error.restype = ctypes.c_char_p
    for name in SYMBOLS:
        if name not in ("ri_free", "ri_last_error", "ri_batch_free"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != RI_OK:
        raise RIError(rc, lib().ri_last_error().decode(errors="replace"))


def _algo(a) -> int:
    return ALGOS[a] if isinstance(a, str) else int(a)


def _text_ptr(text: torch.Tensor) -> tuple:
    if not isinstance(text, torch.Tensor) or text.dtype != torch.uint8 or text.dim() != 1:
        raise TypeError("text must be a 1-D torch.uint8 tensor")
    if not text.is_cuda:
        raise TypeError("text must be on the GPU (no CPU path)")
    if not text.is_contiguous():
        raise TypeError("text must be contiguous")
    return text.data_ptr(), text.numel()


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if isinstance(stream, torch.cuda.Stream) else int(stream)


# ---------------------------------------------------------------------------
# the C functions
# ---------------------------------------------------------------------------

def ri_build(regex, max_states: int = 0) -> int:
    if isinstance(regex, str):
        regex = regex.encode("latin-1")
    regex = bytes(regex)
    h = ctypes.c_void_p()
    opts = ri_build_opts(max_states, 0)
    _check(lib().ri_build(regex, len(regex), ctypes.byref(opts), ctypes.byref(h)))
    return h.value


def ri_free(h: int) -> None:
    lib().ri_free(h)


def ri_info(h: int) -> dict:
    info = ri_info_t()
    _check(lib().ri_info(h, ctypes.byref(info)))
    out = {name: getattr(info, name) for name, _ in ri_info_t._fields_}
    for k in ("starts", "entry_bytes", "table_bytes", "prefix_depth", "prefix_states"):
        out[k] = list(out[k])
    return out


def _result(r: ri_result) -> dict:
    return dict(accept=bool(r.accept), final_state=int(r.final_state), n=int(r.n),
                chunks=int(r.chunks), chunk_size=int(r.chunk_size))


def ri_recognize(h: int, text: torch.Tensor, stream=None) -> dict:
    ptr, n = _text_ptr(text)
    r = ri_result()
    _check(lib().ri_recognize(h, ptr, n, _stream_ptr(stream), ctypes.byref(r)))
    return _result(r)


def ri_recognize_ex(h: int, text: torch.Tensor, stream=None, algo="rid", chunks: int = 0) -> dict:
    ptr, n = _text_ptr(text)
    r = ri_result()
    _check(lib().ri_recognize_ex(h, ptr, n, _stream_ptr(stream), _algo(algo), int(chunks),
                                 ctypes.byref(r)))
    return _result(r)


def ri_recognize_async(h: int, text: torch.Tensor, result: torch.Tensor, stream=None, algo="rid",
                       chunks: int = 0) -> None:
    """Enqueues the recognition on the stream; result (int32 GPU tensor of at
    least 2 entries) receives [accept, final_state] in stream order."""
    ptr, n = _text_ptr(text)
    _check(lib().ri_recognize_async(h, ptr, n, _stream_ptr(stream), _algo(algo), int(chunks),
                                    _results_ptr(result, 1)))


def ri_recognize_noalloc(h: int, text: torch.Tensor, result: torch.Tensor, stream=None, algo="rid",
                         chunks: int = 0) -> None:
    """ri_recognize_async with the library's fixed scratch array (no device
    allocation); the handle's tables must already be on the device."""
    ptr, n = _text_ptr(text)
    _check(lib().ri_recognize_noalloc(h, ptr, n, _stream_ptr(stream), _algo(algo), int(chunks),
                                      _results_ptr(result, 1)))


def ri_chunk_maps(h: int, text: torch.Tensor, stream=None, algo="rid", chunks: int = 0):
    """Returns (result dict, int32 numpy array [chunks, starts]) of the chunk
    maps.  A first call sizes the output from the chunk count actually used."""
    import numpy as np
    ptr, n = _text_ptr(text)
    L = ri_info(h)["starts"][_algo(algo)]
    first = ri_recognize_ex(h, text, stream, algo, chunks)
    cap = max(1, first["chunks"] * L)
    maps = np.full(cap, -1, dtype=np.int32)
    r = ri_result()
    _check(lib().ri_chunk_maps(h, ptr, n, _stream_ptr(stream), _algo(algo), int(chunks),
                               maps.ctypes.data, cap, ctypes.byref(r)))
    res = _result(r)
    c = res["chunks"]
    return res, maps[: c * L].reshape(c, L)


def ri_state_content(h: int, algo, state: int) -> list:
    cap = 1 << 16
    buf = (ctypes.c_uint32 * cap)()
    cnt = ctypes.c_uint32(0)
    _check(lib().ri_state_content(h, _algo(algo), int(state), buf, cap, ctypes.byref(cnt)))
    return list(buf[: cnt.value])


def ri_set_profiling(h: int, enable: bool) -> None:
    _check(lib().ri_set_profiling(h, 1 if enable else 0))


def ri_set_option(h: int, option, value: int) -> None:
    opt = OPTIONS[option] if isinstance(option, str) else int(option)
    _check(lib().ri_set_option(h, opt, int(value)))


def ri_get_option(h: int, option) -> int:
    opt = OPTIONS[option] if isinstance(option, str) else int(option)
    v = ctypes.c_int64(0)
    _check(lib().ri_get_option(h, opt, ctypes.byref(v)))
    return int(v.value)


def ri_autotune(h: int, text: torch.Tensor, stream=None, algo="rid") -> dict:
    ptr, n = _text_ptr(text)
    t = ri_tuning()
    _check(lib().ri_autotune(h, ptr, n, _stream_ptr(stream), _algo(algo), ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in ri_tuning._fields_}


def ri_last_timings(h: int) -> list:
    """[reach phase, join + finalize, whole call, dominant reach kernel, warm-up kernel] in ms."""
    ms = (ctypes.c_float * 5)()
    _check(lib().ri_last_timings(h, ms))
    return [float(x) for x in ms]


def ri_last_error() -> str:
    return lib().ri_last_error().decode(errors="replace")


def _results_ptr(results: torch.Tensor, count: int) -> int:
    if (not isinstance(results, torch.Tensor) or results.dtype != torch.int32 or not results.is_cuda
            or not results.is_contiguous() or results.numel() < 2 * count):
        raise TypeError("results must be a contiguous int32 GPU tensor of at least 2 * count entries")
    return results.data_ptr()


def _requests(requests):
    arr = (ri_request * max(1, len(requests)))()
    for i, (h, text, algo) in enumerate(requests):
        ptr, n = _text_ptr(text)
        arr[i] = ri_request(h, ptr if n else None, n, _algo(algo), 0)
    return arr


def ri_batch_create(requests, chunk_bytes: int = 0) -> int:
    """requests: sequence of (handle, text tensor, algo).  The texts must stay
    alive and unchanged while the batch is used."""
    b = ctypes.c_void_p()
    _check(lib().ri_batch_create(_requests(requests), len(requests), int(chunk_bytes), ctypes.byref(b)))
    return b.value


def ri_batch_create_ex(requests, chunk_bytes: int = 0, mode="auto", warmup_bytes: int = 0) -> int:
    opts = ri_batch_opts(int(chunk_bytes), BATCH_MODES[mode] if isinstance(mode, str) else int(mode),
                         int(warmup_bytes), 0)
    b = ctypes.c_void_p()
    _check(lib().ri_batch_create_ex(_requests(requests), len(requests), ctypes.byref(opts), ctypes.byref(b)))
    return b.value


def ri_batch_update(b: int, requests) -> None:
    _check(lib().ri_batch_update(b, _requests(requests), len(requests)))


def ri_request_footprint(h: int, algo, n: int, chunk_bytes: int = 0) -> int:
    v = ctypes.c_uint64(0)
    _check(lib().ri_request_footprint(h, _algo(algo), int(n), int(chunk_bytes), ctypes.byref(v)))
    return int(v.value)


def ri_batch_free(b: int) -> None:
    lib().ri_batch_free(b)


def ri_batch_run(b: int, results: torch.Tensor, stream=None) -> None:
    info = ri_batch_get_info(b)
    _check(lib().ri_batch_run(b, _stream_ptr(stream), _results_ptr(results, info["texts"])))


def ri_batch_capture(b: int, results: torch.Tensor) -> None:
    info = ri_batch_get_info(b)
    _check(lib().ri_batch_capture(b, _results_ptr(results, info["texts"])))


def ri_batch_launch(b: int, stream=None) -> None:
    _check(lib().ri_batch_launch(b, _stream_ptr(stream)))


def ri_batch_get_info(b: int) -> dict:
    i = ri_batch_info()
    _check(lib().ri_batch_get_info(b, ctypes.byref(i)))
    return {name: getattr(i, name) for name, _ in ri_batch_info._fields_}


def ri_batch_get_group(b: int, index: int) -> dict:
    g = ri_batch_group()
    _check(lib().ri_batch_get_group(b, int(index), ctypes.byref(g)))
    return {name: getattr(g, name) for name, _ in ri_batch_group._fields_}


def ri_batch_autotune(b: int, stream=None) -> dict:
    t = ri_batch_tuning()
    _check(lib().ri_batch_autotune(b, _stream_ptr(stream), ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in ri_batch_tuning._fields_}


# ---------------------------------------------------------------------------
# convenience wrappers
# ---------------------------------------------------------------------------

class Batch:
    """Owns one batch: ``Batch([(recognizer, text, "rid"), ...]).run()`` returns
    an int32 GPU tensor [count, 2] of (accept, final state)."""

    def __init__(self, requests, chunk_bytes: int = 0, mode="auto", warmup_bytes: int = 0):
        reqs = [(r.handle if isinstance(r, Recognizer) else r, t, a) for r, t, a in requests]
        self._texts = [t for _, t, _ in reqs]     # keep the texts alive
        self.count = len(reqs)
        self.handle = ri_batch_create_ex(reqs, chunk_bytes, mode, warmup_bytes)
        dev = self._texts[0].device if self._texts else torch.device("cuda")
        self.results = torch.zeros(max(1, self.count) * 2, dtype=torch.int32, device=dev)

    def run(self, stream=None) -> torch.Tensor:
        ri_batch_run(self.handle, self.results, stream)
        return self.results[: 2 * self.count].view(self.count, 2)

    def capture(self) -> None:
        ri_batch_capture(self.handle, self.results)

    def launch(self, stream=None) -> torch.Tensor:
        ri_batch_launch(self.handle, stream)
        return self.results[: 2 * self.count].view(self.count, 2)

    def info(self) -> dict:
        return ri_batch_get_info(self.handle)

    def group(self, index: int) -> dict:
        return ri_batch_get_group(self.handle, index)

    def autotune(self, stream=None) -> dict:
        return ri_batch_autotune(self.handle, stream)

    def close(self) -> None:
        if self.handle:
            ri_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Recognizer:
    """Owns one handle: ``Recognizer(regex).recognize(text_tensor)``."""

    def __init__(self, regex, max_states: int = 0):
        self.handle = ri_build(regex, max_states)

    def info(self) -> dict:
        return ri_info(self.handle)

    def recognize(self, text, algo="rid", chunks: int = 0, stream=None) -> dict:
        return ri_recognize_ex(self.handle, text, stream, algo, chunks)

    def recognize_async(self, text, result, algo="rid", chunks: int = 0, stream=None) -> None:
        ri_recognize_async(self.handle, text, result, stream, algo, chunks)

    def chunk_maps(self, text, algo="rid", chunks: int = 0, stream=None):
        return ri_chunk_maps(self.handle, text, stream, algo, chunks)

    def state_content(self, algo, state: int) -> list:
        return ri_state_content(self.handle, algo, state)

    def set_profiling(self, enable: bool = True) -> None:
        ri_set_profiling(self.handle, enable)

    def last_timings(self) -> list:
        return ri_last_timings(self.handle)

    def set_option(self, option, value: int) -> None:
        ri_set_option(self.handle, option, value)

    def get_option(self, option) -> int:
        return ri_get_option(self.handle, option)

    def autotune(self, text, algo="rid", stream=None) -> dict:
        return ri_autotune(self.handle, text, stream, algo)

    def close(self) -> None:
        if self.handle:
            ri_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
