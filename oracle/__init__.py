"""CPU oracle for seed-and-extend X-Drop (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It loads ``liboracle.so`` built from
``xdrop_oracle.c`` (plain C, int64, full matrix; see that file's header for the
definition and the paper passages it follows) and shares nothing with the HIP
library.

Sequences are handed over as one symbol code per byte; the oracle reverses the
left-extension prefixes itself, as the seed definition says (paper Sec. 4.1.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xdrop_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
E_RANGE = -2
E_SYMBOL = -6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over seeds)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
             "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Scoring(ctypes.Structure):
    _fields_ = [("alphabet_size", ctypes.c_int32),
                ("matrix", ctypes.POINTER(ctypes.c_int32)),
                ("gap", ctypes.c_int64),
                ("X", ctypes.c_int64)]


class _Ext(ctypes.Structure):
    _fields_ = [("best", ctypes.c_int64), ("x", ctypes.c_int64),
                ("y", ctypes.c_int64), ("cells", ctypes.c_int64)]


SEED_DTYPE = np.dtype([("q", "<i4"), ("t", "<i4"), ("q_pos", "<i4"),
                       ("t_pos", "<i4"), ("k", "<i4")])
RESULT_DTYPE = np.dtype([("score", "<i8"), ("left", "<i8"), ("right", "<i8"),
                         ("seed_score", "<i8"), ("q_begin", "<i8"),
                         ("q_end", "<i8"), ("t_begin", "<i8"),
                         ("t_end", "<i8"), ("cells", "<i8"),
                         ("status", "<i8")])

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.xo_extend_dense.argtypes = [u8p, ctypes.c_int64, u8p,
                                        ctypes.c_int64,
                                        ctypes.POINTER(_Scoring),
                                        ctypes.POINTER(_Ext), i64p, u8p]
        lib.xo_extend_span.argtypes = [u8p, ctypes.c_int64, u8p,
                                       ctypes.c_int64,
                                       ctypes.POINTER(_Scoring),
                                       ctypes.POINTER(_Ext),
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int64)]
        lib.xo_seed_extend.argtypes = [u8p, ctypes.c_int64, u8p,
                                       ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int64,
                                       ctypes.POINTER(_Scoring),
                                       ctypes.c_int64, ctypes.c_void_p]
        lib.xo_batch.argtypes = [u8p, i64p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.POINTER(_Scoring),
                                 ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_int32)]
        for f in (lib.xo_extend_dense, lib.xo_extend_span, lib.xo_seed_extend,
                  lib.xo_batch):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Scoring:
    """Substitution matrix (row = query code, column = target code), linear
    gap added per gap symbol, and X."""
    matrix: np.ndarray
    gap: int
    X: int

    @property
    def alphabet_size(self) -> int:
        return int(self.matrix.shape[0])

    def _c(self):
        m = np.ascontiguousarray(self.matrix, dtype=np.int32)
        sc = _Scoring(m.shape[0], m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      int(self.gap), int(self.X))
        return sc, m  # keep the array alive with the struct


def dna_scoring(match: int = 1, mismatch: int = -1, gap: int = -1,
                X: int = 15) -> Scoring:
    """Match / mismatch scoring over the 4 DNA codes."""
    m = np.full((4, 4), mismatch, dtype=np.int32)
    np.fill_diagonal(m, match)
    return Scoring(m, gap, X)


def _u8(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint8))
    if a.size == 0:
        a = np.zeros(1, dtype=np.uint8)[:0]
    return a


def _ptr(a: np.ndarray, t=ctypes.c_uint8):
    if a.size == 0:
        a = np.zeros(1, dtype=a.dtype)
    return a.ctypes.data_as(ctypes.POINTER(t)), a


def extend(a, b, scoring: Scoring, tier: str = "dense"):
    """One extension E(a, b).  Returns (best, x, y, cells)."""
    lib = _load()
    a = _u8(a)
    b = _u8(b)
    sc, keep = scoring._c()
    out = _Ext()
    pa, ka = _ptr(a)
    pb, kb = _ptr(b)
    if tier == "dense":
        rc = lib.xo_extend_dense(pa, a.size, pb, b.size, ctypes.byref(sc),
                                 ctypes.byref(out), None, None)
    elif tier == "span":
        rc = lib.xo_extend_span(pa, a.size, pb, b.size, ctypes.byref(sc),
                                ctypes.byref(out), None, None)
    else:
        raise ValueError(tier)
    if rc != OK:
        raise RuntimeError(f"oracle error {rc}")
    return int(out.best), int(out.x), int(out.y), int(out.cells)


def extend_matrix(a, b, scoring: Scoring):
    """Dense tier with the whole matrix returned: (result, S, finite)."""
    lib = _load()
    a = _u8(a)
    b = _u8(b)
    sc, keep = scoring._c()
    out = _Ext()
    S = np.zeros((a.size + 1, b.size + 1), dtype=np.int64)
    F = np.zeros((a.size + 1, b.size + 1), dtype=np.uint8)
    pa, ka = _ptr(a)
    pb, kb = _ptr(b)
    rc = lib.xo_extend_dense(pa, a.size, pb, b.size, ctypes.byref(sc),
                             ctypes.byref(out),
                             S.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             F.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != OK:
        raise RuntimeError(f"oracle error {rc}")
    return (int(out.best), int(out.x), int(out.y), int(out.cells)), S, F.astype(bool)


def band_widths(a, b, scoring: Scoring, finite: bool = False):
    """Working band hi_d - lo_d + 1 per antidiagonal (Sec. 6.1 study); with
    finite=True also the finite range (L_d, U_d; -1 when dead) per d."""
    lib = _load()
    a = _u8(a)
    b = _u8(b)
    sc, keep = scoring._c()
    out = _Ext()
    w = np.zeros(a.size + b.size + 1, dtype=np.int32)
    fr = np.zeros((a.size + b.size + 1, 2), dtype=np.int64)
    pa, ka = _ptr(a)
    pb, kb = _ptr(b)
    rc = lib.xo_extend_span(pa, a.size, pb, b.size, ctypes.byref(sc),
                            ctypes.byref(out),
                            w.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            fr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != OK:
        raise RuntimeError(f"oracle error {rc}")
    return (w, fr) if finite else w


def seed_extend(q, t, q_pos: int, t_pos: int, k: int, scoring: Scoring,
                dense_limit: int = 1 << 22) -> dict:
    """Left + seed + right for one seed; returns a dict of RESULT_DTYPE fields."""
    lib = _load()
    q = _u8(q)
    t = _u8(t)
    sc, keep = scoring._c()
    out = np.zeros(1, dtype=RESULT_DTYPE)
    pq, kq = _ptr(q)
    pt, kt = _ptr(t)
    rc = lib.xo_seed_extend(pq, q.size, pt, t.size, q_pos, t_pos, k,
                            ctypes.byref(sc), dense_limit,
                            out.ctypes.data_as(ctypes.c_void_p))
    if rc != OK:
        raise RuntimeError(f"oracle error {rc}")
    return {f: int(out[0][f]) for f in RESULT_DTYPE.names}


def batch(codes: np.ndarray, offsets: np.ndarray, seeds: np.ndarray,
          scoring: Scoring, threads: int = 0, dense_limit: int = 1 << 20):
    """All seeds of a batch (OpenMP dynamic over seeds).

    Returns (results as a RESULT_DTYPE array, threads used)."""
    lib = _load()
    codes = _u8(codes)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    sd = np.ascontiguousarray(seeds).astype(SEED_DTYPE, copy=False)
    out = np.zeros(len(sd), dtype=RESULT_DTYPE)
    sc, keep = scoring._c()
    used = ctypes.c_int32(0)
    pc, kc = _ptr(codes)
    rc = lib.xo_batch(pc, offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      len(offsets) - 1,
                      sd.ctypes.data_as(ctypes.c_void_p) if len(sd) else None,
                      len(sd), ctypes.byref(sc), dense_limit, int(threads),
                      out.ctypes.data_as(ctypes.c_void_p) if len(sd) else None,
                      ctypes.byref(used))
    if rc != OK:
        raise RuntimeError(f"oracle error {rc}")
    return out, int(used.value)


def traceback(S: np.ndarray, F: np.ndarray, a, b, scoring: Scoring, x: int,
              y: int):
    """Walk back from (x, y) to (0, 0) through finite predecessors whose value
    plus the step score equals the cell.  Returns the list of cells."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    M = scoring.matrix
    path = [(x, y)]
    while (x, y) != (0, 0):
        v = S[x, y]
        if x >= 1 and y >= 1 and F[x - 1, y - 1] and \
                S[x - 1, y - 1] + M[a[x - 1], b[y - 1]] == v:
            x, y = x - 1, y - 1
        elif x >= 1 and F[x - 1, y] and S[x - 1, y] + scoring.gap == v:
            x = x - 1
        elif y >= 1 and F[x, y - 1] and S[x, y - 1] + scoring.gap == v:
            y = y - 1
        else:
            raise AssertionError(f"no predecessor for cell {(x, y)}")
        path.append((x, y))
    return path[::-1]
