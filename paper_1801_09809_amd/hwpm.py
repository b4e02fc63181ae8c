"""Python binding of libhwpm.so (include/hwpm.h): argument marshalling only.

Every function here has the name of the C entry point it calls and passes
plain pointers and sizes; all matching work runs in the library's HIP
kernels.  PyTorch supplies device memory (the CSC, the matchings, the
workspace) and the stream.  There is no CPU fallback: if the library is
missing or the GPU is absent, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first: libhwpm.so then binds to torch's HIP runtime

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhwpm.so")

HWPM_OK = 0
HWPM_EINVAL = -1
HWPM_ESINGULAR = -2
HWPM_EBADCSC = -3
HWPM_EBADMATCH = -4
HWPM_ENOMEM = -5
HWPM_ETOOBIG = -6
HWPM_EDEVICE = -7
HWPM_EINTERNAL = -8
HWPM_PENDING = 1
MAX_ROUND_STATS = 512
STATIC_SCRATCH_BYTES = 128 << 20  # HWPM_STATIC_SCRATCH_BYTES
TUNE_CANDIDATES = 12
TUNE_CONFIGS = ((1, 4), (1, 8), (1, 16), (1, 32), (1, 64), (3, 4), (3, 8), (3, 16), (3, 32), (4, 4),
                (5, 4), (5, 8))

EXPORTED = (
    "hwpm_default_options", "hwpm_strerror", "hwpm_create", "hwpm_destroy",
    "hwpm_workspace_bytes", "hwpm_check_csc", "hwpm_improve", "hwpm_improve_static", "hwpm_match",
    "hwpm_autotune", "hwpm_batch_workspace_bytes", "hwpm_improve_batch", "hwpm_match_batch",
    "hwpm_server_default_options", "hwpm_server_create", "hwpm_server_destroy",
    "hwpm_submit", "hwpm_poll", "hwpm_server_get_stats", "hwpm_server_get_tune_table",
    "hwpm_default_tune_table", "hwpm_tune_bin", "hwpm_set_tune_table", "hwpm_autotune_table",
)


class HwpmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {hwpm_strerror(status)} (status {status})")


class hwpm_csc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("col_ptr", ctypes.c_void_p),
        ("row_idx", ctypes.c_void_p),
        ("weight", ctypes.c_void_p),
    ]


class hwpm_options(ctypes.Structure):
    _fields_ = [
        ("max_rounds", ctypes.c_int32),
        ("check_csc", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("tile_width", ctypes.c_int32),
        ("probe", ctypes.c_int32),
        ("mcm_plain", ctypes.c_int32),
        ("full_search", ctypes.c_int32),
        ("graph", ctypes.c_int32),
    ]


class hwpm_stats(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int32),
        ("hit_round_cap", ctypes.c_int32),
        ("cycles_applied", ctypes.c_int64),
        ("long_columns", ctypes.c_int32),
        ("greedy_rounds", ctypes.c_int32),
        ("greedy_cardinality", ctypes.c_int32),
        ("mcm_cardinality", ctypes.c_int32),
        ("mcm_phases", ctypes.c_int32),
        ("mcm_levels", ctypes.c_int32),
        ("init_weight", ctypes.c_double),
        ("final_weight", ctypes.c_double),
        ("ms_check", ctypes.c_float),
        ("ms_greedy", ctypes.c_float),
        ("ms_mcm", ctypes.c_float),
        ("ms_setup", ctypes.c_float),
        ("ms_transpose", ctypes.c_float),
        ("ms_search", ctypes.c_float),
        ("ms_resolve", ctypes.c_float),
        ("ms_apply", ctypes.c_float),
        ("ms_final", ctypes.c_float),
        ("ms_total", ctypes.c_float),
        ("ms_search_first", ctypes.c_float),
        ("graph_launches", ctypes.c_int32),
        ("probe_used", ctypes.c_int32),
        ("tile_used", ctypes.c_int32),
        ("round_candidates", ctypes.c_int32 * MAX_ROUND_STATS),
        ("round_applied", ctypes.c_int32 * MAX_ROUND_STATS),
        ("round_ms_search", ctypes.c_float * MAX_ROUND_STATS),
        ("round_roots", ctypes.c_int32 * MAX_ROUND_STATS),
    ]

    def as_dict(self) -> dict:
        nr = min(self.rounds, MAX_ROUND_STATS)
        d = {name: getattr(self, name) for name, _ in self._fields_
             if not name.startswith("round_")}
        d["round_candidates"] = list(self.round_candidates[:nr])
        d["round_applied"] = list(self.round_applied[:nr])
        d["round_ms_search"] = list(self.round_ms_search[:nr])
        d["round_roots"] = list(self.round_roots[:nr])
        return d


class hwpm_item_stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("hit_round_cap", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("cycles_applied", ctypes.c_int64),
        ("init_weight", ctypes.c_double),
        ("final_weight", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


TUNE_BINS = 6  # HWPM_TUNE_BINS


class hwpm_tune_table(ctypes.Structure):
    _fields_ = [
        ("max_degree", ctypes.c_float * TUNE_BINS),
        ("probe", ctypes.c_int32 * TUNE_BINS),
        ("tile_width", ctypes.c_int32 * TUNE_BINS),
        ("ms_per_mentry", ctypes.c_float * TUNE_BINS),
    ]

    def as_list(self) -> list:
        return [{"max_degree": float(self.max_degree[b]), "probe": int(self.probe[b]),
                 "tile_width": int(self.tile_width[b]), "ms_per_mentry": float(self.ms_per_mentry[b])}
                for b in range(TUNE_BINS)]


class hwpm_server_options(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("workers", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("tune", ctypes.c_int32),
        ("arena_bytes", ctypes.c_size_t),
        ("solve", hwpm_options),
        ("rounds_per_step", ctypes.c_int32),
        ("copy_inputs", ctypes.c_int32),
    ]


class hwpm_request_info(ctypes.Structure):
    _fields_ = [
        ("item", hwpm_item_stats),
        ("queue_ms", ctypes.c_double),
        ("latency_ms", ctypes.c_double),
        ("batch_size", ctypes.c_int32),
        ("worker", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = self.item.as_dict()
        d.update(queue_ms=self.queue_ms, latency_ms=self.latency_ms, batch_size=self.batch_size,
                 worker=self.worker, steps=self.steps)
        return d


class hwpm_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "submitted", "completed", "batches", "max_batch_seen", "max_running", "pending", "running",
        "arena_in_use", "arena_peak", "joined")]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhwpm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_1801_09809_amd/build.py")
        lib = ctypes.CDLL(path)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.hwpm_default_options.restype = None
        lib.hwpm_default_options.argtypes = [ctypes.POINTER(hwpm_options)]
        lib.hwpm_strerror.restype = ctypes.c_char_p
        lib.hwpm_strerror.argtypes = [ctypes.c_int]
        lib.hwpm_create.restype = ctypes.c_int
        lib.hwpm_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
        lib.hwpm_destroy.restype = ctypes.c_int
        lib.hwpm_destroy.argtypes = [vp]
        lib.hwpm_workspace_bytes.restype = ctypes.c_int
        lib.hwpm_workspace_bytes.argtypes = [i32, i64, ctypes.POINTER(ctypes.c_size_t)]
        lib.hwpm_check_csc.restype = ctypes.c_int
        lib.hwpm_check_csc.argtypes = [vp, ctypes.POINTER(hwpm_csc), vp, ctypes.c_size_t]
        lib.hwpm_match.restype = ctypes.c_int
        lib.hwpm_match.argtypes = [vp, ctypes.POINTER(hwpm_csc), vp, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(hwpm_options), ctypes.POINTER(hwpm_stats), vp,
                                   ctypes.c_size_t]
        lib.hwpm_batch_workspace_bytes.restype = ctypes.c_int
        lib.hwpm_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(hwpm_csc), ctypes.POINTER(ctypes.c_size_t)]
        batch_args = [vp, i32, ctypes.POINTER(hwpm_csc)]
        tail = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(hwpm_options),
                ctypes.POINTER(hwpm_item_stats), ctypes.POINTER(hwpm_stats), vp, ctypes.c_size_t]
        lib.hwpm_improve_batch.restype = ctypes.c_int
        lib.hwpm_improve_batch.argtypes = batch_args + [ctypes.POINTER(vp), ctypes.POINTER(vp)] + tail
        lib.hwpm_match_batch.restype = ctypes.c_int
        lib.hwpm_match_batch.argtypes = batch_args + [ctypes.POINTER(vp)] + tail
        lib.hwpm_improve.restype = ctypes.c_int
        lib.hwpm_improve.argtypes = [vp, ctypes.POINTER(hwpm_csc), vp, vp,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(hwpm_options),
                                     ctypes.POINTER(hwpm_stats), vp, ctypes.c_size_t]
        lib.hwpm_improve_static.restype = ctypes.c_int
        lib.hwpm_improve_static.argtypes = [vp, ctypes.POINTER(hwpm_csc), vp, vp,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(hwpm_options),
                                            ctypes.POINTER(hwpm_stats)]
        lib.hwpm_autotune.restype = ctypes.c_int
        lib.hwpm_autotune.argtypes = [vp, ctypes.POINTER(hwpm_csc), vp, vp, ctypes.POINTER(hwpm_options),
                                      ctypes.POINTER(ctypes.c_float), vp, ctypes.c_size_t]
        lib.hwpm_server_default_options.restype = None
        lib.hwpm_server_default_options.argtypes = [ctypes.POINTER(hwpm_server_options)]
        lib.hwpm_server_create.restype = ctypes.c_int
        lib.hwpm_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(hwpm_server_options)]
        lib.hwpm_server_destroy.restype = ctypes.c_int
        lib.hwpm_server_destroy.argtypes = [vp]
        lib.hwpm_submit.restype = ctypes.c_int
        lib.hwpm_submit.argtypes = [vp, ctypes.POINTER(hwpm_csc), ctypes.POINTER(ctypes.c_uint64)]
        lib.hwpm_poll.restype = ctypes.c_int
        lib.hwpm_poll.argtypes = [vp, ctypes.c_uint64, i32, vp, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(hwpm_request_info)]
        lib.hwpm_server_get_stats.restype = ctypes.c_int
        lib.hwpm_server_get_stats.argtypes = [vp, ctypes.POINTER(hwpm_server_stats)]
        lib.hwpm_server_get_tune_table.restype = ctypes.c_int
        lib.hwpm_server_get_tune_table.argtypes = [vp, ctypes.POINTER(hwpm_tune_table)]
        lib.hwpm_default_tune_table.restype = None
        lib.hwpm_default_tune_table.argtypes = [ctypes.POINTER(hwpm_tune_table)]
        lib.hwpm_tune_bin.restype = ctypes.c_int
        lib.hwpm_tune_bin.argtypes = [ctypes.POINTER(hwpm_tune_table), i32, i64]
        lib.hwpm_set_tune_table.restype = ctypes.c_int
        lib.hwpm_set_tune_table.argtypes = [vp, ctypes.POINTER(hwpm_tune_table)]
        lib.hwpm_autotune_table.restype = ctypes.c_int
        lib.hwpm_autotune_table.argtypes = [vp, ctypes.POINTER(hwpm_csc), vp, vp, ctypes.POINTER(hwpm_tune_table),
                                            vp, ctypes.c_size_t]
        _lib = lib
    return _lib


# ---------------------------------------------------------------------------
# one function per C entry point

def hwpm_default_options() -> hwpm_options:
    o = hwpm_options()
    load_library().hwpm_default_options(ctypes.byref(o))
    return o


def hwpm_strerror(status: int) -> str:
    return load_library().hwpm_strerror(int(status)).decode()


def hwpm_create(device: int = 0, stream: int | None = None) -> int:
    """Returns the handle (an integer address); `stream` is a hipStream_t address."""
    h = ctypes.c_void_p()
    st = load_library().hwpm_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream or 0))
    if st != HWPM_OK:
        raise HwpmError(st, "hwpm_create")
    return h.value


def hwpm_destroy(handle: int) -> int:
    return load_library().hwpm_destroy(ctypes.c_void_p(handle))


def hwpm_workspace_bytes(n: int, nnz: int) -> int:
    b = ctypes.c_size_t(0)
    st = load_library().hwpm_workspace_bytes(int(n), int(nnz), ctypes.byref(b))
    if st != HWPM_OK:
        raise HwpmError(st, "hwpm_workspace_bytes")
    return int(b.value)


def _csc(n, nnz, col_ptr_ptr, row_idx_ptr, weight_ptr) -> hwpm_csc:
    return hwpm_csc(int(n), int(nnz), ctypes.c_void_p(col_ptr_ptr), ctypes.c_void_p(row_idx_ptr),
                    ctypes.c_void_p(weight_ptr))


def hwpm_check_csc(handle: int, n: int, nnz: int, col_ptr_ptr: int, row_idx_ptr: int,
                   weight_ptr: int, ws_ptr: int, ws_bytes: int) -> int:
    A = _csc(n, nnz, col_ptr_ptr, row_idx_ptr, weight_ptr)
    return load_library().hwpm_check_csc(ctypes.c_void_p(handle), ctypes.byref(A),
                                         ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes))


def hwpm_improve(handle: int, n: int, nnz: int, col_ptr_ptr: int, row_idx_ptr: int,
                 weight_ptr: int, mate_in_ptr: int, perm_out_ptr: int, ws_ptr: int,
                 ws_bytes: int, options: hwpm_options | None = None, want_stats: bool = True):
    """Returns (status, total, stats or None)."""
    A = _csc(n, nnz, col_ptr_ptr, row_idx_ptr, weight_ptr)
    total = ctypes.c_double(0.0)
    stats = hwpm_stats() if want_stats else None
    st = load_library().hwpm_improve(
        ctypes.c_void_p(handle), ctypes.byref(A), ctypes.c_void_p(mate_in_ptr),
        ctypes.c_void_p(perm_out_ptr), ctypes.byref(total),
        ctypes.byref(options) if options is not None else None,
        ctypes.byref(stats) if stats is not None else None,
        ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes))
    return st, total.value, stats


def hwpm_improve_static(handle: int, n: int, nnz: int, col_ptr_ptr: int, row_idx_ptr: int,
                        weight_ptr: int, mate_in_ptr: int, perm_out_ptr: int,
                        options: hwpm_options | None = None, want_stats: bool = True):
    """hwpm_improve on the library's static workspace.  Returns (status, total, stats or None)."""
    A = _csc(n, nnz, col_ptr_ptr, row_idx_ptr, weight_ptr)
    total = ctypes.c_double(0.0)
    stats = hwpm_stats() if want_stats else None
    st = load_library().hwpm_improve_static(
        ctypes.c_void_p(handle), ctypes.byref(A), ctypes.c_void_p(mate_in_ptr),
        ctypes.c_void_p(perm_out_ptr), ctypes.byref(total),
        ctypes.byref(options) if options is not None else None,
        ctypes.byref(stats) if stats is not None else None)
    return st, total.value, stats


def hwpm_match(handle: int, n: int, nnz: int, col_ptr_ptr: int, row_idx_ptr: int, weight_ptr: int,
               perm_out_ptr: int, ws_ptr: int, ws_bytes: int, options: hwpm_options | None = None,
               want_stats: bool = True):
    """Returns (status, total, stats or None)."""
    A = _csc(n, nnz, col_ptr_ptr, row_idx_ptr, weight_ptr)
    total = ctypes.c_double(0.0)
    stats = hwpm_stats() if want_stats else None
    st = load_library().hwpm_match(
        ctypes.c_void_p(handle), ctypes.byref(A), ctypes.c_void_p(perm_out_ptr), ctypes.byref(total),
        ctypes.byref(options) if options is not None else None,
        ctypes.byref(stats) if stats is not None else None,
        ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes))
    return st, total.value, stats


def hwpm_autotune(handle: int, n: int, nnz: int, col_ptr_ptr: int, row_idx_ptr: int, weight_ptr: int,
                  mate_ptr: int, perm_ptr: int, ws_ptr: int, ws_bytes: int,
                  options: hwpm_options | None = None):
    """Returns (status, tuned options, per-candidate best ms list)."""
    A = _csc(n, nnz, col_ptr_ptr, row_idx_ptr, weight_ptr)
    opt = options if options is not None else hwpm_default_options()
    ms = (ctypes.c_float * TUNE_CANDIDATES)()
    st = load_library().hwpm_autotune(ctypes.c_void_p(handle), ctypes.byref(A), ctypes.c_void_p(mate_ptr),
                                      ctypes.c_void_p(perm_ptr), ctypes.byref(opt), ms,
                                      ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes))
    return st, opt, list(ms)


def _csc_array(mats):
    """mats: sequence of (n, nnz, col_ptr_ptr, row_idx_ptr, weight_ptr)."""
    arr = (hwpm_csc * max(len(mats), 1))()
    for b, m in enumerate(mats):
        arr[b] = _csc(*m)
    return arr


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * max(len(ptrs), 1))()
    for b, p in enumerate(ptrs):
        arr[b] = p
    return arr


def hwpm_batch_workspace_bytes(mats) -> int:
    arr = _csc_array(mats)
    b = ctypes.c_size_t(0)
    st = load_library().hwpm_batch_workspace_bytes(len(mats), arr, ctypes.byref(b))
    if st != HWPM_OK:
        raise HwpmError(st, "hwpm_batch_workspace_bytes")
    return int(b.value)


def hwpm_improve_batch(handle: int, mats, mate_ptrs, perm_ptrs, ws_ptr: int, ws_bytes: int,
                       options: hwpm_options | None = None):
    """Returns (status, totals list, item stats array, batch stats)."""
    count = len(mats)
    totals = (ctypes.c_double * max(count, 1))()
    items = (hwpm_item_stats * max(count, 1))()
    stats = hwpm_stats()
    st = load_library().hwpm_improve_batch(
        ctypes.c_void_p(handle), count, _csc_array(mats), _ptr_array(mate_ptrs), _ptr_array(perm_ptrs),
        totals, ctypes.byref(options) if options is not None else None, items, ctypes.byref(stats),
        ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes))
    return st, list(totals[:count]), items, stats


def hwpm_match_batch(handle: int, mats, perm_ptrs, ws_ptr: int, ws_bytes: int,
                     options: hwpm_options | None = None):
    """Returns (status, totals list, item stats array, batch stats)."""
    count = len(mats)
    totals = (ctypes.c_double * max(count, 1))()
    items = (hwpm_item_stats * max(count, 1))()
    stats = hwpm_stats()
    st = load_library().hwpm_match_batch(
        ctypes.c_void_p(handle), count, _csc_array(mats), _ptr_array(perm_ptrs), totals,
        ctypes.byref(options) if options is not None else None, items, ctypes.byref(stats),
        ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes))
    return st, list(totals[:count]), items, stats


def hwpm_server_default_options() -> hwpm_server_options:
    o = hwpm_server_options()
    load_library().hwpm_server_default_options(ctypes.byref(o))
    return o


def hwpm_server_create(options: hwpm_server_options | None = None) -> int:
    s = ctypes.c_void_p()
    st = load_library().hwpm_server_create(ctypes.byref(s),
                                           ctypes.byref(options) if options is not None else None)
    if st != HWPM_OK:
        raise HwpmError(st, "hwpm_server_create")
    return s.value


def hwpm_server_destroy(server: int) -> int:
    return load_library().hwpm_server_destroy(ctypes.c_void_p(server))


def hwpm_submit(server: int, n: int, nnz: int, col_ptr_ptr: int, row_idx_ptr: int,
                weight_ptr: int) -> tuple[int, int]:
    """HOST pointers.  Returns (status, ticket)."""
    t = ctypes.c_uint64(0)
    A = _csc(n, nnz, col_ptr_ptr, row_idx_ptr, weight_ptr)
    st = load_library().hwpm_submit(ctypes.c_void_p(server), ctypes.byref(A), ctypes.byref(t))
    return st, int(t.value)


def hwpm_poll(server: int, ticket: int, wait: bool, perm_ptr: int | None):
    """perm_ptr: HOST int32[n] or None.  Returns (status, total, request info)."""
    total = ctypes.c_double(0.0)
    info = hwpm_request_info()
    st = load_library().hwpm_poll(ctypes.c_void_p(server), ctypes.c_uint64(ticket), int(bool(wait)),
                                  ctypes.c_void_p(perm_ptr or 0), ctypes.byref(total), ctypes.byref(info))
    return st, total.value, info


def hwpm_default_tune_table() -> hwpm_tune_table:
    t = hwpm_tune_table()
    load_library().hwpm_default_tune_table(ctypes.byref(t))
    return t


def hwpm_tune_bin(table: hwpm_tune_table, n: int, nnz: int) -> int:
    return load_library().hwpm_tune_bin(ctypes.byref(table), int(n), int(nnz))


def hwpm_set_tune_table(handle: int, table: hwpm_tune_table | None) -> int:
    return load_library().hwpm_set_tune_table(ctypes.c_void_p(handle),
                                              ctypes.byref(table) if table is not None else None)


def hwpm_autotune_table(handle: int, n: int, nnz: int, col_ptr_ptr: int, row_idx_ptr: int, weight_ptr: int,
                        mate_in_ptr: int, perm_out_ptr: int, table: hwpm_tune_table, ws_ptr: int,
                        ws_bytes: int) -> int:
    A = _csc(n, nnz, col_ptr_ptr, row_idx_ptr, weight_ptr)
    return load_library().hwpm_autotune_table(ctypes.c_void_p(handle), ctypes.byref(A), ctypes.c_void_p(mate_in_ptr),
                                              ctypes.c_void_p(perm_out_ptr), ctypes.byref(table),
                                              ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes))


def hwpm_server_get_tune_table(server: int) -> hwpm_tune_table:
    t = hwpm_tune_table()
    st = load_library().hwpm_server_get_tune_table(ctypes.c_void_p(server), ctypes.byref(t))
    if st != HWPM_OK:
        raise HwpmError(st, "hwpm_server_get_tune_table")
    return t


def hwpm_server_get_stats(server: int) -> hwpm_server_stats:
    s = hwpm_server_stats()
    st = load_library().hwpm_server_get_stats(ctypes.c_void_p(server), ctypes.byref(s))
    if st != HWPM_OK:
        raise HwpmError(st, "hwpm_server_get_stats")
    return s


# ---------------------------------------------------------------------------
# convenience wrappers

class ImproveResult:
    """perm: int32 on the device; total: the matched weight; stats: a dict of
    the call's hwpm_stats, converted on first access (the conversion costs
    more host time than the rest of the binding's work per call)."""
    __slots__ = ("perm", "total", "_raw", "_stats")

    def __init__(self, perm: torch.Tensor, total: float, raw: hwpm_stats):
        self.perm = perm
        self.total = total
        self._raw = raw
        self._stats = None

    @property
    def stats(self) -> dict:
        if self._stats is None:
            self._stats = self._raw.as_dict()
        return self._stats


class Solver:
    """Owns a handle (bound to a device and stream) and a workspace tensor."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HWPM library runs on the device only")
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = hwpm_create(device, self.stream.cuda_stream)
        self.ws = torch.empty(0, dtype=torch.uint8, device=self.device)
        self._ws_need = {}  # workspace bytes per (n, nnz)

    def close(self):
        if self.handle:
            hwpm_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _workspace(self, n: int, nnz: int) -> torch.Tensor:
        need = self._ws_need.get((n, nnz))
        if need is None:
            need = self._ws_need[(n, nnz)] = hwpm_workspace_bytes(n, nnz)
        if self.ws.numel() < need:
            self.ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self.ws

    @staticmethod
    def _check(t: torch.Tensor, dtype, name: str, numel: int | None = None):
        if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
        if numel is not None and t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")

    def check_csc(self, col_ptr, row_idx, w) -> int:
        n = col_ptr.numel() - 1
        nnz = row_idx.numel()
        ws = self._workspace(n, nnz)
        with torch.cuda.stream(self.stream):
            return hwpm_check_csc(self.handle, n, nnz, col_ptr.data_ptr(), row_idx.data_ptr(),
                                  w.data_ptr(), ws.data_ptr(), ws.numel())

    @staticmethod
    def options(max_rounds=0, check_csc=True, timing=False, tile_width=0, probe=0,
                mcm_plain=False, full_search=False, graph=True) -> hwpm_options:
        opt = hwpm_default_options()
        opt.max_rounds = int(max_rounds)
        opt.check_csc = int(bool(check_csc))
        opt.timing = int(timing)  # False/True -> 0/1; 2: search stage only
        opt.tile_width = int(tile_width)
        opt.probe = int(probe)
        opt.mcm_plain = int(bool(mcm_plain))
        opt.full_search = int(bool(full_search))
        opt.graph = int(bool(graph))
        return opt

    def match(self, col_ptr: torch.Tensor, row_idx: torch.Tensor, w: torch.Tensor,
              perm_out: torch.Tensor | None = None, **kw) -> ImproveResult:
        n = col_ptr.numel() - 1
        nnz = row_idx.numel()
        self._check(col_ptr, torch.int64, "col_ptr")
        self._check(row_idx, torch.int32, "row_idx")
        self._check(w, torch.float64, "w", nnz)
        if perm_out is None:
            perm_out = torch.empty(n, dtype=torch.int32, device=self.device)
        self._check(perm_out, torch.int32, "perm_out", n)
        ws = self._workspace(n, nnz)
        st, total, stats = hwpm_match(self.handle, n, nnz, col_ptr.data_ptr(), row_idx.data_ptr(),
                                      w.data_ptr(), perm_out.data_ptr(), ws.data_ptr(), ws.numel(),
                                      self.options(**kw))
        if st != HWPM_OK:
            raise HwpmError(st, "hwpm_match")
        return ImproveResult(perm_out, total, stats)

    def _batch(self, mats, mates, perms, match: bool, **kw):
        desc = []
        for (cp, ri, w) in mats:
            self._check(cp, torch.int64, "col_ptr")
            self._check(ri, torch.int32, "row_idx")
            self._check(w, torch.float64, "w", ri.numel())
            desc.append((cp.numel() - 1, ri.numel(), cp.data_ptr(), ri.data_ptr(), w.data_ptr()))
        if perms is None:
            perms = [torch.empty(d[0], dtype=torch.int32, device=self.device) for d in desc]
        need = hwpm_batch_workspace_bytes(desc)
        if self.ws.numel() < need:
            self.ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        opt = self.options(**kw)
        if match:
            st, totals, items, stats = hwpm_match_batch(
                self.handle, desc, [p.data_ptr() for p in perms], self.ws.data_ptr(), self.ws.numel(), opt)
        else:
            st, totals, items, stats = hwpm_improve_batch(
                self.handle, desc, [m.data_ptr() for m in mates], [p.data_ptr() for p in perms],
                self.ws.data_ptr(), self.ws.numel(), opt)
        if st != HWPM_OK:
            raise HwpmError(st, "hwpm_match_batch" if match else "hwpm_improve_batch")
        return perms, totals, [items[b].as_dict() for b in range(len(desc))], stats.as_dict()

    def improve_batch(self, mats, mates, perms=None, **kw):
        """mats: list of (col_ptr, row_idx, w) device tensors; mates: starting matchings."""
        return self._batch(mats, mates, perms, False, **kw)

    def match_batch(self, mats, perms=None, **kw):
        return self._batch(mats, None, perms, True, **kw)

    def set_tune_table(self, table: hwpm_tune_table | None):
        """Batches with default launch options take their configuration from
        this table by degree bin (None: library defaults)."""
        st = hwpm_set_tune_table(self.handle, table)
        if st != HWPM_OK:
            raise HwpmError(st, "hwpm_set_tune_table")

    def autotune_table(self, col_ptr: torch.Tensor, row_idx: torch.Tensor, w: torch.Tensor,
                       mate_in: torch.Tensor, table: hwpm_tune_table | None = None) -> hwpm_tune_table:
        """Tune the degree bin of this matrix; returns the table (a new default
        one when none is given) with that bin's entry filled."""
        n = col_ptr.numel() - 1
        nnz = row_idx.numel()
        self._check(col_ptr, torch.int64, "col_ptr")
        self._check(row_idx, torch.int32, "row_idx")
        self._check(w, torch.float64, "w", nnz)
        self._check(mate_in, torch.int32, "mate_in", n)
        table = table if table is not None else hwpm_default_tune_table()
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        ws = self._workspace(n, nnz)
        st = hwpm_autotune_table(self.handle, n, nnz, col_ptr.data_ptr(), row_idx.data_ptr(), w.data_ptr(),
                                 mate_in.data_ptr(), perm.data_ptr(), table, ws.data_ptr(), ws.numel())
        if st != HWPM_OK:
            raise HwpmError(st, "hwpm_autotune_table")
        return table

    def autotune(self, col_ptr: torch.Tensor, row_idx: torch.Tensor, w: torch.Tensor,
                 mate_in: torch.Tensor, perm_out: torch.Tensor | None = None, **kw):
        """Returns (probe, tile_width, {(probe, tile): best ms}, perm_out)."""
        n = col_ptr.numel() - 1
        nnz = row_idx.numel()
        self._check(col_ptr, torch.int64, "col_ptr")
        self._check(row_idx, torch.int32, "row_idx")
        self._check(w, torch.float64, "w", nnz)
        self._check(mate_in, torch.int32, "mate_in", n)
        if perm_out is None:
            perm_out = torch.empty(n, dtype=torch.int32, device=self.device)
        ws = self._workspace(n, nnz)
        st, opt, ms = hwpm_autotune(self.handle, n, nnz, col_ptr.data_ptr(), row_idx.data_ptr(), w.data_ptr(),
                                    mate_in.data_ptr(), perm_out.data_ptr(), ws.data_ptr(), ws.numel(),
                                    self.options(**kw))
        if st != HWPM_OK:
            raise HwpmError(st, "hwpm_autotune")
        return opt.probe, opt.tile_width, dict(zip(TUNE_CONFIGS, ms)), perm_out

    def improve(self, col_ptr: torch.Tensor, row_idx: torch.Tensor, w: torch.Tensor,
                mate_in: torch.Tensor, perm_out: torch.Tensor | None = None, max_rounds: int = 0,
                check_csc: bool = True, timing: int = 0, tile_width: int = 0,
                probe: int = 0, full_search: bool = False, graph: bool = True) -> ImproveResult:
        n = col_ptr.numel() - 1
        nnz = row_idx.numel()
        self._check(col_ptr, torch.int64, "col_ptr")
        self._check(row_idx, torch.int32, "row_idx")
        self._check(w, torch.float64, "w", nnz)
        self._check(mate_in, torch.int32, "mate_in", n)
        if perm_out is None:
            perm_out = torch.empty(n, dtype=torch.int32, device=self.device)
        self._check(perm_out, torch.int32, "perm_out", n)
        ws = self._workspace(n, nnz)
        opt = self.options(max_rounds, check_csc, timing, tile_width, probe, False, full_search, graph)
        st, total, stats = hwpm_improve(self.handle, n, nnz, col_ptr.data_ptr(), row_idx.data_ptr(),
                                        w.data_ptr(), mate_in.data_ptr(), perm_out.data_ptr(),
                                        ws.data_ptr(), ws.numel(), opt)
        if st != HWPM_OK:
            raise HwpmError(st, "hwpm_improve")
        return ImproveResult(perm_out, total, stats)


class Server:
    """Request loop over host matrices (numpy arrays): submit, then poll.  With
    copy_inputs=False the server reads the caller's arrays until the result is
    polled, and they are kept alive here until then."""

    def __init__(self, device: int = 0, workers: int = 2, max_batch: int = 64,
                 arena_bytes: int = 8 << 30, tune: bool = True, rounds_per_step: int = 8,
                 copy_inputs: bool = True, **solve_kw):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HWPM library runs on the device only")
        opt = hwpm_server_default_options()
        opt.device = int(device)
        opt.workers = int(workers)
        opt.max_batch = int(max_batch)
        opt.arena_bytes = int(arena_bytes)
        opt.tune = int(bool(tune))
        opt.rounds_per_step = int(rounds_per_step)
        opt.copy_inputs = int(bool(copy_inputs))
        if solve_kw:
            opt.solve = Solver.options(**solve_kw)
        self.server = hwpm_server_create(opt)
        self._copy = bool(copy_inputs)
        self._n = {}
        self._keep = {}  # the host arrays of each queued request, until polled (by reference only)

    def close(self):
        if self.server:
            hwpm_server_destroy(self.server)
            self.server = 0
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, col_ptr, row_idx, w) -> int:
        import numpy as np
        cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
        ri = np.ascontiguousarray(row_idx, dtype=np.int32)
        ww = np.ascontiguousarray(w, dtype=np.float64)
        n = cp.size - 1
        if ww.size != ri.size:
            raise ValueError("row_idx and w differ in length")
        st, ticket = hwpm_submit(self.server, n, ri.size, cp.ctypes.data, ri.ctypes.data, ww.ctypes.data)
        if st != HWPM_OK:
            raise HwpmError(st, "hwpm_submit")
        self._n[ticket] = n
        if not self._copy:
            self._keep[ticket] = (cp, ri, ww)  # the server reads them until the result is polled
        return ticket

    def poll(self, ticket: int, wait: bool = True):
        """Returns None while pending, else (status, perm numpy int32 or None, total, info dict)."""
        import numpy as np
        n = self._n[ticket]
        perm = np.empty(max(n, 1), dtype=np.int32)
        st, total, info = hwpm_poll(self.server, ticket, wait, perm.ctypes.data)
        if st == HWPM_PENDING:
            return None
        del self._n[ticket]
        self._keep.pop(ticket, None)
        return st, (perm[:n] if st == HWPM_OK else None), total, info.as_dict()

    def stats(self) -> dict:
        return hwpm_server_get_stats(self.server).as_dict()

    def tune_table(self) -> list:
        """The online tuning table: per degree bin its bound and the tuned
        (probe, tile_width), probe 0 while untuned."""
        return hwpm_server_get_tune_table(self.server).as_list()
