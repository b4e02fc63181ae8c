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
from dataclasses import dataclass

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
MAX_ROUND_STATS = 512

EXPORTED = (
    "hwpm_default_options", "hwpm_strerror", "hwpm_create", "hwpm_destroy",
    "hwpm_workspace_bytes", "hwpm_check_csc", "hwpm_improve", "hwpm_match",
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
        ("ms_reserved", ctypes.c_float),
        ("round_candidates", ctypes.c_int32 * MAX_ROUND_STATS),
        ("round_applied", ctypes.c_int32 * MAX_ROUND_STATS),
        ("round_ms_search", ctypes.c_float * MAX_ROUND_STATS),
        ("round_roots", ctypes.c_int32 * MAX_ROUND_STATS),
    ]

    def as_dict(self) -> dict:
        nr = min(self.rounds, MAX_ROUND_STATS)
        d = {name: getattr(self, name) for name, _ in self._fields_
             if not name.startswith("round_") and name != "ms_reserved"}
        d["round_candidates"] = list(self.round_candidates[:nr])
        d["round_applied"] = list(self.round_applied[:nr])
        d["round_ms_search"] = list(self.round_ms_search[:nr])
        d["round_roots"] = list(self.round_roots[:nr])
        return d


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
        lib.hwpm_improve.restype = ctypes.c_int
        lib.hwpm_improve.argtypes = [vp, ctypes.POINTER(hwpm_csc), vp, vp,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(hwpm_options),
                                     ctypes.POINTER(hwpm_stats), vp, ctypes.c_size_t]
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


# ---------------------------------------------------------------------------
# convenience wrapper over torch tensors

@dataclass
class ImproveResult:
    perm: torch.Tensor      # int32 on the device
    total: float
    stats: dict


class Solver:
    """Owns a handle (bound to a device and stream) and a workspace tensor."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HWPM library runs on the device only")
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = hwpm_create(device, self.stream.cuda_stream)
        self.ws = torch.empty(0, dtype=torch.uint8, device=self.device)

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
        need = hwpm_workspace_bytes(n, nnz)
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
                mcm_plain=False, full_search=False) -> hwpm_options:
        opt = hwpm_default_options()
        opt.max_rounds = int(max_rounds)
        opt.check_csc = int(bool(check_csc))
        opt.timing = int(bool(timing))
        opt.tile_width = int(tile_width)
        opt.probe = int(probe)
        opt.mcm_plain = int(bool(mcm_plain))
        opt.full_search = int(bool(full_search))
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
        return ImproveResult(perm_out, total, stats.as_dict())

    def improve(self, col_ptr: torch.Tensor, row_idx: torch.Tensor, w: torch.Tensor,
                mate_in: torch.Tensor, perm_out: torch.Tensor | None = None, max_rounds: int = 0,
                check_csc: bool = True, timing: bool = False, tile_width: int = 0,
                probe: int = 0, full_search: bool = False) -> ImproveResult:
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
        opt = self.options(max_rounds, check_csc, timing, tile_width, probe, False, full_search)
        st, total, stats = hwpm_improve(self.handle, n, nnz, col_ptr.data_ptr(), row_idx.data_ptr(),
                                        w.data_ptr(), mate_in.data_ptr(), perm_out.data_ptr(),
                                        ws.data_ptr(), ws.numel(), opt)
        if st != HWPM_OK:
            raise HwpmError(st, "hwpm_improve")
        return ImproveResult(perm_out, total, stats.as_dict())
