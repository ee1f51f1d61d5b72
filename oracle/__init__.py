"""Plain CPU oracle for exact simulation (ES) of AIG miters.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are its only users; the GPU path never calls it.

It reads ASCII AIGER with its own reader and simulates one pattern at a time
(paper, Section 2.1 miter definition; Section 2.2 exact simulation: enumerate
every primary-input assignment and check the miter output).  Pattern p sets
input i to bit i of p.  ``lowest_failure`` returns the lowest p whose miter
output (OR of all outputs) is 1, or None when the circuit is equivalent.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build as _build  # noqa: F401

NONE = (1 << 64) - 1


def load_library(path: str = LIB):
    """Load an oracle shared library (the default one is built on first use)."""
    if path == LIB and not os.path.exists(LIB):
        _build()
    lib = ctypes.CDLL(path)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_parse_aag.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p),
                                     ctypes.c_char_p, ctypes.c_size_t]
    lib.oracle_parse_aag.restype = ctypes.c_int
    lib.oracle_free.argtypes = [ctypes.c_void_p]
    for f in ("oracle_num_inputs", "oracle_num_outputs", "oracle_num_ands"):
        getattr(lib, f).argtypes = [ctypes.c_void_p]
        getattr(lib, f).restype = ctypes.c_uint32
    lib.oracle_eval_outputs.argtypes = [ctypes.c_void_p, u64p, ctypes.c_size_t, u64p]
    lib.oracle_eval_miter.argtypes = [ctypes.c_void_p, u64p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint8)]
    lib.oracle_lowest_failure.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, u64p]
    lib.oracle_lowest_failure.restype = ctypes.c_uint64
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


class OracleError(Exception):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Circuit:
    """An AIG parsed by the oracle's own ASCII AIGER reader."""

    def __init__(self, aag: bytes, library=None):
        L = library if library is not None else lib()
        self._lib = L
        h = ctypes.c_void_p()
        err = ctypes.create_string_buffer(256)
        rc = L.oracle_parse_aag(aag, len(aag), ctypes.byref(h), err, 256)
        if rc != 0:
            raise OracleError(rc, err.value.decode())
        self._h = h
        self.num_inputs = L.oracle_num_inputs(h)
        self.num_outputs = L.oracle_num_outputs(h)
        self.num_ands = L.oracle_num_ands(h)

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.oracle_free(self._h)
            self._h = None

    def outputs(self, patterns) -> np.ndarray:
        """uint64 array: bit j of entry t is output j at pattern patterns[t]."""
        ps = np.ascontiguousarray(np.asarray(patterns, dtype=np.uint64))
        out = np.zeros(ps.shape, dtype=np.uint64)
        rc = self._lib.oracle_eval_outputs(self._h, ps.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ps.size,
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        if rc != 0:
            raise OracleError(rc, "more than 64 outputs")
        return out

    def miter(self, patterns) -> np.ndarray:
        """uint8 array: OR of all outputs at each pattern."""
        ps = np.ascontiguousarray(np.asarray(patterns, dtype=np.uint64))
        out = np.zeros(ps.shape, dtype=np.uint8)
        self._lib.oracle_eval_miter(self._h, ps.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ps.size,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return out

    def lowest_failure(self, lo: int = 0, hi=None, threads: int = 1):
        """(lowest failing p in [lo, hi) or None, patterns simulated).  hi defaults to 2^n."""
        if hi is None:
            hi = 1 << self.num_inputs
            if hi > NONE:
                raise ValueError("2^64 patterns: give hi explicitly")
        ev = ctypes.c_uint64(0)
        p = self._lib.oracle_lowest_failure(self._h, lo, hi, threads, ctypes.byref(ev))
        return (None if p == NONE else int(p)), int(ev.value)


def check(aag: bytes, threads: int = 1, library=None):
    """Exhaustive check: None if the miter is 0 on all 2^n patterns, else the lowest failing p."""
    return Circuit(aag, library).lowest_failure(threads=threads)[0]
