"""Oracle search space: enumeration, validity and repair -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg import
this package.  The GPU library never does, and nothing here imports it.

The heavy loops live in ct_oracle.c (plain scalar C, OpenMP across
independent items); this module holds the search-space object and the
plain definitions that sit on top (rank of a configuration in the valid
list, per-parameter presence used by the "adjacent" neighbour rule).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import List, Optional, Sequence

import numpy as np

from . import expr as _expr

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ct_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lock = threading.Lock()
_lib = None

HAMMING, INDEX_L1, TIER_EUCLID, TIER_RANDOM, HAM1_RANDOM = 0, 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile the oracle's C core with gcc (plain -O2, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
                        "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Space(ctypes.Structure):
    _fields_ = [("n_params", ctypes.c_int32), ("radices", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("n_cons", ctypes.c_int32), ("expr", ctypes.c_void_p), ("expr_off", ctypes.c_void_p)]


class _Valid(ctypes.Structure):
    _fields_ = [("n_params", ctypes.c_int32), ("n_valid", ctypes.c_int64), ("vrows", ctypes.c_void_p),
                ("vlin", ctypes.c_void_p), ("present", ctypes.c_void_p)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = ctypes.CDLL(build())
            vp, i64, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32
            L.or_mask_words.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, vp]
            L.or_valid_rows.argtypes = [vp, vp, i64, vp]
            L.or_valid_lin.argtypes = [vp, vp, i64, vp]
            L.or_decode_many.argtypes = [vp, vp, i64, vp]
            L.or_encode_many.argtypes = [vp, vp, i64, vp]
            L.or_philox.argtypes = [u32, u32, vp, vp]
            L.or_philox_many.argtypes = [u32, u32, vp, i64, vp]
            L.or_argmin.argtypes = [vp, vp, ctypes.c_int, vp, u32, u32, u32, u32]
            L.or_argmin.restype = i64
            L.or_argmin_many.argtypes = [vp, vp, i64, ctypes.c_int, vp, u32, u32, vp, u32, vp]
            L.or_overflow_flag.restype = ctypes.c_int
            L.or_num_threads.restype = ctypes.c_int
            L.or_set_num_threads.argtypes = [ctypes.c_int]
            _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check_overflow():
    if lib().or_overflow_flag():
        lib().or_clear_overflow()
        raise OverflowError("constraint evaluation overflowed 64-bit integers; the oracle cannot decide it")


def philox(key: int, ctr: Sequence[int]) -> List[int]:
    """Philox4x32-10 of one 128-bit counter under a 64-bit key (key low word first)."""
    c = np.asarray(ctr, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox(key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF, _ptr(c), _ptr(o))
    return [int(x) for x in o]


def philox_many(key: int, ctrs: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(ctrs, dtype=np.uint32)
    o = np.zeros_like(c)
    lib().or_philox_many(key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF, _ptr(c), c.shape[0], _ptr(o))
    return o


class Space:
    """The CSP (X, D, C) of Section IV-A and, once enumerated, its solution list."""

    def __init__(self, names: Sequence[str], values: Sequence[Sequence[int]], constraints: Sequence[str]):
        self.names = list(names)
        self.values = [list(map(int, v)) for v in values]
        self.constraints = list(constraints)
        self.D = len(self.names)
        if not (1 <= self.D <= 64):
            raise ValueError("1..64 parameters supported")
        self.radices = np.array([len(v) for v in self.values], dtype=np.int32)
        if np.any(self.radices < 1) or np.any(self.radices > 255):
            raise ValueError("each parameter needs 1..255 values")
        self.n_cartesian = int(np.prod(self.radices.astype(object)))
        self._vals = np.array([x for v in self.values for x in v], dtype=np.int64)
        enc = [_expr.encode(c, self.names) for c in self.constraints]
        offs, flat = [], []
        for e in enc:
            offs.append(len(flat))
            flat += e
        self._expr = np.array(flat if flat else [0], dtype=np.int64)
        self._expr_off = np.array(offs if offs else [0], dtype=np.int64)
        self._s = _Space(self.D, _ptr(self.radices), _ptr(self._vals), len(enc),
                         _ptr(self._expr), _ptr(self._expr_off))
        self.words: Optional[np.ndarray] = None
        self.vlin: Optional[np.ndarray] = None
        self.vrows: Optional[np.ndarray] = None
        self.present: Optional[np.ndarray] = None
        self._V = None

    @classmethod
    def from_spec(cls, spec) -> "Space":
        return cls(spec.names, list(spec.params.values()), spec.constraints)

    # -- Section IV-A: validity of configurations -------------------------------------
    def valid_rows(self, rows: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1, self.D)
        out = np.zeros(r.shape[0], dtype=np.uint8)
        lib().or_valid_rows(ctypes.byref(self._s), _ptr(r), r.shape[0], _ptr(out))
        _check_overflow()
        return out.astype(bool)

    def valid_lin(self, lin: np.ndarray) -> np.ndarray:
        l = np.ascontiguousarray(lin, dtype=np.uint64)
        out = np.zeros(l.shape[0], dtype=np.uint8)
        lib().or_valid_lin(ctypes.byref(self._s), _ptr(l), l.shape[0], _ptr(out))
        _check_overflow()
        return out.astype(bool)

    def mask_words(self, w0: int, w1: int) -> np.ndarray:
        out = np.zeros(max(0, w1 - w0), dtype=np.uint64)
        if w1 > w0:
            lib().or_mask_words(ctypes.byref(self._s), self.n_cartesian, w0, w1, _ptr(out))
        _check_overflow()
        return out

    def decode(self, lin: np.ndarray) -> np.ndarray:
        l = np.ascontiguousarray(lin, dtype=np.uint64).ravel()
        out = np.zeros((l.shape[0], self.D), dtype=np.int32)
        lib().or_decode_many(ctypes.byref(self._s), _ptr(l), l.shape[0], _ptr(out))
        return out

    def encode(self, rows: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1, self.D)
        out = np.zeros(r.shape[0], dtype=np.uint64)
        lib().or_encode_many(ctypes.byref(self._s), _ptr(r), r.shape[0], _ptr(out))
        return out

    # -- Section IV-A: full enumeration before tuning ----------------------------------
    def enumerate(self, progress=None, chunk_words: int = 1 << 22) -> "Space":
        """Every configuration, in chunks of chunk_words bitmask words (progress(msg) after each)."""
        n_words = (self.n_cartesian + 63) // 64
        self.words = np.zeros(n_words, dtype=np.uint64)
        parts = []
        for w0 in range(0, n_words, chunk_words):
            w1 = min(n_words, w0 + chunk_words)
            self.words[w0:w1] = self.mask_words(w0, w1)
            parts.append(words_to_lin(self.words[w0:w1], w0))
            if progress:
                progress(f"oracle enumeration: words {w1}/{n_words}")
        self.vlin = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint64)
        self._finish_list()
        return self

    def set_valid_list(self, vlin: np.ndarray) -> "Space":
        """Adopt a valid list computed elsewhere by this oracle (e.g. a stored golden)."""
        self.vlin = np.ascontiguousarray(vlin, dtype=np.uint64)
        self._finish_list()
        return self

    def _finish_list(self):
        self.vrows = self.decode(self.vlin)
        self.present = np.zeros((self.D, 256), dtype=np.uint8)
        for j in range(self.D):
            self.present[j, np.unique(self.vrows[:, j])] = 1
        self._V = _Valid(self.D, len(self.vlin), _ptr(self.vrows), _ptr(self.vlin), _ptr(self.present))

    @property
    def n_valid(self) -> int:
        return int(len(self.vlin))

    def pos(self, lin) -> np.ndarray:
        """Position of valid linear indices in the ascending valid list (rank)."""
        l = np.asarray(lin, dtype=np.uint64)
        p = np.searchsorted(self.vlin, l)
        assert np.all(p < len(self.vlin)) and np.all(self.vlin[np.minimum(p, len(self.vlin) - 1)] == l), \
            "configuration is not in the valid list"
        return p.astype(np.int64)

    # -- repair / neighbour argmin (Section IV-A neighbour rules, Alg. 1-3) -------------
    def argmin(self, cands: np.ndarray, metric: int, who: Optional[np.ndarray] = None, key: int = 0,
               gen: int = 0, pos_q16: Optional[np.ndarray] = None) -> np.ndarray:
        c = np.ascontiguousarray(cands, dtype=np.int32).reshape(-1, self.D)
        n = c.shape[0]
        w = np.ascontiguousarray(np.arange(n) if who is None else who, dtype=np.uint32)
        out = np.zeros(n, dtype=np.int64)
        pq = None if pos_q16 is None else np.ascontiguousarray(pos_q16, dtype=np.int64).reshape(n, self.D)
        if n:
            lib().or_argmin_many(ctypes.byref(self._V), _ptr(c), n, metric,
                                 None if pq is None else _ptr(pq),
                                 key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF, _ptr(w), gen, _ptr(out))
        return out

    def repair(self, cands: np.ndarray, metric: int, who=None, key: int = 0, gen: int = 0,
               pos_q16=None) -> np.ndarray:
        """ct_repair by definition: valid rows unchanged, invalid rows -> argmin row.

        HAM1_RANDOM (GA mutation) applies to every row and leaves a row
        unchanged when it has no valid Hamming-1 neighbour.
        Returns the repaired rows (value indices).
        """
        c = np.ascontiguousarray(cands, dtype=np.int32).reshape(-1, self.D)
        out = c.copy()
        n = c.shape[0]
        w = np.arange(n, dtype=np.uint32) if who is None else np.asarray(who, dtype=np.uint32)
        if metric == HAM1_RANDOM:
            sel = np.arange(n)
        else:
            sel = np.flatnonzero(~self.valid_rows(c))
        if len(sel) == 0:
            return out
        pq = None if pos_q16 is None else np.asarray(pos_q16, dtype=np.int64).reshape(n, self.D)[sel]
        best = self.argmin(c[sel], metric, w[sel], key, gen, pq)
        for k, i in enumerate(sel):
            if best[k] >= 0:
                out[i] = self.vrows[best[k]]
        return out


def words_to_lin(words: np.ndarray, w0: int, chunk: int = 1 << 20) -> np.ndarray:
    """Ascending linear indices of the set bits of bitmask words starting at word w0."""
    parts = []
    for s in range(0, len(words), chunk):
        part = words[s:s + chunk]
        nz = np.flatnonzero(part)
        if len(nz) == 0:
            continue
        bits = np.unpackbits(part[nz].view(np.uint8).reshape(-1, 8), axis=1, bitorder="little")
        r, b = np.nonzero(bits)
        parts.append((np.uint64(w0 + s) + nz[r].astype(np.uint64)) * np.uint64(64) + b.astype(np.uint64))
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint64)


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the C core's parallel loops (timing the single-threaded oracle)."""
    lib().or_set_num_threads(int(n))
