"""Python side of the C++ oracle (oracle/cpp/oracle.cpp) -- test
infrastructure only, like the rest of oracle/.

The C++ oracle evaluates the same plain set semantics as oracle/dl.py with one
byte per membership and OpenMP over hypotheses; it is the timed CPU baseline.
This module builds it (g++ -fopenmp), turns nested-tuple hypotheses into its
prefix token streams and calls it through ctypes.  It shares no code with the
library's binding or encoder.

Parity status: pinned bit for bit to oracle/dl.py (the pinned Python oracle)
on the whole c1 workload and on random tiny knowledge bases
(tests/test_oracle_cpp.py).
"""
from __future__ import annotations

import ctypes
import os
import struct
import subprocess
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpp", "oracle.cpp")
LIB = os.path.join(HERE, "cpp", "liboracle_cpp.so")

_CODES = {"top": 0, "bot": 1, "atom": 2, "not": 3, "and": 4, "or": 5, "exists": 6, "forall": 7,
          "atleast": 8, "atmost": 9, "exactly": 10, "dge": 11, "dle": 12, "deq": 13}
_lib = None


def build() -> str:
    """Compile the C++ oracle (every call compiles)."""
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed on {SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.ocpp_create.argtypes = [I64, I32, I64, P, I32, P, P, I32, P, P, P]
        L.ocpp_create.restype = P
        L.ocpp_destroy.argtypes = [P]
        L.ocpp_destroy.restype = None
        L.ocpp_ext.argtypes = [P, P, I64, P]
        L.ocpp_ext.restype = ctypes.c_int
        L.ocpp_coverage.argtypes = [P, P, P, I64, I32, P]
        L.ocpp_coverage.restype = I64
        L.ocpp_threads.argtypes = []
        L.ocpp_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _f32_bits(t: float) -> int:
    return struct.unpack("<I", struct.pack("<f", float(t)))[0]


def tokens(h, out: list) -> None:
    """Append the prefix token stream of nested-tuple hypothesis h to out."""
    op = h[0]
    out.append(_CODES[op])
    if op in ("top", "bot"):
        return
    if op == "atom":
        out.append(int(h[1]))
    elif op == "not":
        tokens(h[1], out)
    elif op in ("and", "or"):
        out.append(len(h) - 1)
        for c in h[1:]:
            tokens(c, out)
    elif op in ("exists", "forall"):
        out += [int(h[1]), int(h[2])]
        tokens(h[3], out)
    elif op in ("atleast", "atmost", "exactly"):
        out += [int(h[1]), int(h[2]), int(h[3])]
        tokens(h[4], out)
    else:                                   # dge / dle / deq
        out += [int(h[1]), _f32_bits(h[2])]


def batch_tokens(hyps: Sequence):
    toks, offs = [], [0]
    for h in hyps:
        tokens(h, toks)
        offs.append(len(toks))
    return np.asarray(toks, dtype=np.int64), np.asarray(offs, dtype=np.int64)


class CppOracle:
    """The C++ oracle over one knowledge base (the synth KB container:
    n, concept_bits, role_offsets, role_targets, data, pos_bits, neg_bits)."""

    def __init__(self, kb):
        L = lib()
        self.n = int(kb.n)
        w = (self.n + 63) // 64
        self._c = np.ascontiguousarray(np.asarray(kb.concept_bits, dtype=np.uint64).reshape(-1, w))
        self._off = np.ascontiguousarray(kb.role_offsets, dtype=np.int64)
        self._tg = np.ascontiguousarray(kb.role_targets, dtype=np.int32)
        self._d = np.ascontiguousarray(kb.data, dtype=np.float32)
        self._p = np.ascontiguousarray(kb.pos_bits, dtype=np.uint64)
        self._q = np.ascontiguousarray(kb.neg_bits, dtype=np.uint64)
        n_roles = self._off.shape[0] if self._off.ndim == 2 else 0
        n_data = self._d.shape[0] if self._d.ndim == 2 else 0
        ptr = lambda a: a.ctypes.data if a.size else None   # noqa: E731
        self._h = L.ocpp_create(self.n, self._c.shape[0], w, ptr(self._c), n_roles, ptr(self._off),
                                ptr(self._tg), n_data, ptr(self._d), ptr(self._p), ptr(self._q))
        if not self._h:
            raise ValueError("ocpp_create rejected the knowledge base")

    def close(self):
        if getattr(self, "_h", None):
            lib().ocpp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ext(self, h) -> np.ndarray:
        t = []
        tokens(h, t)
        t = np.asarray(t, dtype=np.int64)
        out = np.empty(max(self.n, 1), dtype=np.uint8)
        if lib().ocpp_ext(self._h, t.ctypes.data, t.size, out.ctypes.data) != 0:
            raise ValueError(f"malformed hypothesis {h!r}")
        return out[: self.n].astype(bool)

    def coverages_tokens(self, toks: np.ndarray, offs: np.ndarray, threads: int = 0) -> np.ndarray:
        H = offs.size - 1
        out = np.zeros((max(H, 1), 2), dtype=np.uint32)
        if H:
            r = lib().ocpp_coverage(self._h, toks.ctypes.data, offs.ctypes.data, H, threads, out.ctypes.data)
            if r != 0:
                raise ValueError(f"malformed hypothesis {-1 - r}")
        return out[:H]

    def coverages(self, hyps: Sequence, threads: int = 0) -> np.ndarray:
        """uint32 [H][2] (covered positives, covered negatives) per hypothesis."""
        toks, offs = batch_tokens(hyps)
        return self.coverages_tokens(toks, offs, threads)


def max_threads() -> int:
    return int(lib().ocpp_threads())
