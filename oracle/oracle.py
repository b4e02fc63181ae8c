"""ctypes wrapper over the C oracle (test infrastructure only).

The C source (hwpm_oracle.c) holds the arithmetic; this module only builds
it with gcc and marshals numpy arrays.  See hwpm_oracle.c for the paper
passages each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hwpm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_ROUND_STATS = 256


class _Stats(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int32),
        ("hit_round_cap", ctypes.c_int32),
        ("cycles_applied", ctypes.c_int64),
        ("init_weight", ctypes.c_double),
        ("final_weight", ctypes.c_double),
        ("round_candidates", ctypes.c_int32 * MAX_ROUND_STATS),
        ("round_applied", ctypes.c_int32 * MAX_ROUND_STATS),
        ("greedy_rounds", ctypes.c_int32),
        ("greedy_cardinality", ctypes.c_int32),
        ("mcm_phases", ctypes.c_int32),
        ("mcm_levels", ctypes.c_int32),
    ]


def build_oracle(force: bool = True) -> str:
    """Compile hwpm_oracle.c into liboracle.so (plain binary64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        lib.oracle_tree_sum.restype = ctypes.c_double
        lib.oracle_tree_sum.argtypes = [p, ctypes.c_int64]
        lib.oracle_improve.restype = ctypes.c_int
        lib.oracle_improve.argtypes = [ctypes.c_int32, p, p, p, p, ctypes.c_int32, p, p,
                                       ctypes.POINTER(_Stats)]
        lib.oracle_greedy.restype = ctypes.c_int32
        lib.oracle_greedy.argtypes = [ctypes.c_int32, p, p, p, ctypes.c_int32, p, p, p]
        lib.oracle_mcm.restype = ctypes.c_int32
        lib.oracle_mcm.argtypes = [ctypes.c_int32, p, p, p, ctypes.c_int32, p, p, p, p]
        lib.oracle_match.restype = ctypes.c_int
        lib.oracle_match.argtypes = [ctypes.c_int32, p, p, p, ctypes.c_int32, ctypes.c_int32,
                                     p, p, ctypes.POINTER(_Stats), p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csc(col_ptr, row_idx, w):
    col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int64)
    row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    return col_ptr, row_idx, w


@dataclass
class OracleResult:
    status: int
    perm: np.ndarray
    total: float
    rounds: int = 0
    hit_round_cap: bool = False
    cycles_applied: int = 0
    init_weight: float = 0.0
    final_weight: float = 0.0
    round_candidates: list = field(default_factory=list)
    round_applied: list = field(default_factory=list)
    mcm_cardinality: int = -1
    greedy_rounds: int = 0
    greedy_cardinality: int = 0
    mcm_phases: int = 0
    mcm_levels: int = 0


def _result(status, perm, total, st: _Stats, card=-1) -> OracleResult:
    nr = min(st.rounds, MAX_ROUND_STATS)
    return OracleResult(
        status=status, perm=perm, total=total, rounds=st.rounds,
        hit_round_cap=bool(st.hit_round_cap), cycles_applied=st.cycles_applied,
        init_weight=st.init_weight, final_weight=st.final_weight,
        round_candidates=list(st.round_candidates[:nr]),
        round_applied=list(st.round_applied[:nr]), mcm_cardinality=card,
        greedy_rounds=st.greedy_rounds, greedy_cardinality=st.greedy_cardinality,
        mcm_phases=st.mcm_phases, mcm_levels=st.mcm_levels)


def oracle_tree_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return _load().oracle_tree_sum(_ptr(x), x.size)


def oracle_improve(n, col_ptr, row_idx, w, mate_in, max_rounds: int = 0) -> OracleResult:
    col_ptr, row_idx, w = _csc(col_ptr, row_idx, w)
    mate_in = np.ascontiguousarray(mate_in, dtype=np.int32)
    perm = np.full(max(n, 0), -1, dtype=np.int32)
    total = ctypes.c_double(0.0)
    st = _Stats()
    rc = _load().oracle_improve(n, _ptr(col_ptr), _ptr(row_idx), _ptr(w), _ptr(mate_in),
                                max_rounds, _ptr(perm), ctypes.cast(ctypes.pointer(total), ctypes.c_void_p),
                                ctypes.byref(st))
    return _result(rc, perm, total.value, st)


def _i32_out():
    v = ctypes.c_int32(0)
    return v, ctypes.cast(ctypes.pointer(v), ctypes.c_void_p)


def oracle_greedy(n, col_ptr, row_idx, w, heavy: bool = True, counts: bool = False):
    """(cardinality, mc, mr); with counts=True also the number of proposal rounds."""
    col_ptr, row_idx, w = _csc(col_ptr, row_idx, w)
    mc = np.empty(max(n, 0), dtype=np.int32)
    mr = np.empty(max(n, 0), dtype=np.int32)
    rounds, rp = _i32_out()
    card = _load().oracle_greedy(n, _ptr(col_ptr), _ptr(row_idx), _ptr(w), int(heavy), _ptr(mc), _ptr(mr), rp)
    return (card, mc, mr, rounds.value) if counts else (card, mc, mr)


def oracle_mcm(n, col_ptr, row_idx, w, mc, mr, heavy: bool = True, counts: bool = False):
    """(cardinality, mc, mr) from the matching (mc, mr); with counts=True also
    the number of BFS phases and of levels."""
    col_ptr, row_idx, w = _csc(col_ptr, row_idx, w)
    mc = np.array(mc, dtype=np.int32, copy=True)
    mr = np.array(mr, dtype=np.int32, copy=True)
    phases, pp = _i32_out()
    levels, lp = _i32_out()
    card = _load().oracle_mcm(n, _ptr(col_ptr), _ptr(row_idx), _ptr(w), int(heavy), _ptr(mc), _ptr(mr), pp, lp)
    return (card, mc, mr, phases.value, levels.value) if counts else (card, mc, mr)


def oracle_match(n, col_ptr, row_idx, w, heavy: bool = True, max_rounds: int = 0) -> OracleResult:
    col_ptr, row_idx, w = _csc(col_ptr, row_idx, w)
    perm = np.full(max(n, 0), -1, dtype=np.int32)
    total = ctypes.c_double(0.0)
    st = _Stats()
    card = ctypes.c_int32(-1)
    rc = _load().oracle_match(n, _ptr(col_ptr), _ptr(row_idx), _ptr(w), int(heavy), max_rounds,
                              _ptr(perm), ctypes.cast(ctypes.pointer(total), ctypes.c_void_p),
                              ctypes.byref(st), ctypes.cast(ctypes.pointer(card), ctypes.c_void_p))
    return _result(rc, perm, total.value, st, card.value)
