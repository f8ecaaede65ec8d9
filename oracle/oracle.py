"""ctypes front end of the C oracle (``oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg use it.
It compiles ``oracle.c`` with gcc when the shared object is missing or older
than the source, then exposes :func:`normalize` (one ground term) and
:func:`normalize_many` (a batch, term by term).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ORC_OK, ORC_E_ARG, ORC_E_RULE, ORC_E_TERM, ORC_E_STEPS, ORC_E_MEM = 0, -1, -3, -4, -6, -9


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L",
                               "-Wall", "-Wextra", "-shared", "-fPIC", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        i32p, i64p = P(ctypes.c_int32), P(ctypes.c_int64)
        lib.orc_new.restype = ctypes.c_void_p
        lib.orc_new.argtypes = [ctypes.c_int32, i32p, ctypes.c_int32, i32p, i32p, i32p]
        lib.orc_free.argtypes = [ctypes.c_void_p]
        lib.orc_run.restype = ctypes.c_int32
        lib.orc_run.argtypes = [ctypes.c_void_p, i32p, ctypes.c_int64, ctypes.c_int64]
        lib.orc_result_len.restype = ctypes.c_int64
        lib.orc_result_len.argtypes = [ctypes.c_void_p]
        lib.orc_result_copy.argtypes = [ctypes.c_void_p, i32p]
        lib.orc_result_fnv.restype = ctypes.c_uint64
        lib.orc_result_fnv.argtypes = [ctypes.c_void_p]
        lib.orc_counts.argtypes = [ctypes.c_void_p, i64p]
        lib.orc_steps.restype = ctypes.c_int64
        lib.orc_steps.argtypes = [ctypes.c_void_p]
        lib.orc_seconds.restype = ctypes.c_double
        lib.orc_seconds.argtypes = [ctypes.c_void_p]
        lib.orc_peak_live.restype = ctypes.c_int64
        lib.orc_peak_live.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OracleError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"oracle status {code} {msg}")
        self.code = code


@dataclass
class Result:
    nf: np.ndarray          # canonical serialisation (prefix symbol ids)
    fnv: int                # FNV-1a 64 of its little-endian bytes
    counts: np.ndarray      # rule applications per rule
    seconds: float          # normalisation time (excludes parsing/serialising)
    peak_live: int

    @property
    def steps(self) -> int:
        return int(self.counts.sum())


class Oracle:
    def __init__(self, arity, rule_off, rule_code):
        lib = _load()
        self._lib = lib
        self.arity = np.ascontiguousarray(arity, dtype=np.int32)
        self.rule_off = np.ascontiguousarray(rule_off, dtype=np.int32)
        self.rule_code = np.ascontiguousarray(rule_code, dtype=np.int32)
        self.n_rules = len(self.rule_off) - 1
        st = ctypes.c_int32(0)
        self._h = lib.orc_new(len(self.arity), _ptr(self.arity, ctypes.c_int32), self.n_rules,
                              _ptr(self.rule_off, ctypes.c_int32),
                              _ptr(self.rule_code, ctypes.c_int32), ctypes.byref(st))
        if not self._h:
            raise OracleError(st.value, "rule load")

    @classmethod
    def from_trs(cls, trs):
        return cls(*trs.encode_rules())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def run(self, term, max_steps: int = 1 << 62, with_nf: bool = True) -> Result:
        t = np.ascontiguousarray(term, dtype=np.int32)
        st = self._lib.orc_run(self._h, _ptr(t, ctypes.c_int32), len(t), int(max_steps))
        if st != ORC_OK:
            raise OracleError(st)
        n = self._lib.orc_result_len(self._h)
        out = np.empty(n if with_nf else 0, dtype=np.int32)
        if with_nf:
            self._lib.orc_result_copy(self._h, _ptr(out, ctypes.c_int32))
        cnt = np.zeros(max(self.n_rules, 1), dtype=np.int64)
        self._lib.orc_counts(self._h, _ptr(cnt, ctypes.c_int64))
        return Result(out, int(self._lib.orc_result_fnv(self._h)), cnt[:self.n_rules],
                      float(self._lib.orc_seconds(self._h)),
                      int(self._lib.orc_peak_live(self._h)))


def normalize(trs, term, max_steps: int = 1 << 62) -> Result:
    o = Oracle.from_trs(trs)
    try:
        return o.run(term, max_steps)
    finally:
        o.close()


def normalize_many(trs, terms, max_steps: int = 1 << 62, with_nf: bool = True):
    o = Oracle.from_trs(trs)
    try:
        return [o.run(t, max_steps, with_nf) for t in terms]
    finally:
        o.close()


def fnv1a64(codes) -> int:
    """FNV-1a 64 over the little-endian int32 bytes (same definition as the C
    side; used to compare serialisations compactly)."""
    b = np.ascontiguousarray(codes, dtype="<i4").tobytes()
    x = 1469598103934665603
    for byte in b:
        x ^= byte
        x = (x * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return x
