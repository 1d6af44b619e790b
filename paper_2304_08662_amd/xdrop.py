"""Python binding of the C ABI in include/xdrop.h (argument marshalling only).

Device buffers are PyTorch tensors on the GPU; their data pointers and the
current HIP stream are handed to the library.  Every step of the alignment
runs in the library's HIP kernels; there is no fallback: if ``libxdrop.so``
is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libxdrop.so")

OK = 0
E_INVALID = -1
E_RANGE = -2
E_NOMEM = -3
E_DEVICE = -4
E_BUDGET = -5
E_SYMBOL = -6
BAND_OVERFLOW = -7
E_SCRATCH = -8
NOALLOC_MAX_SEEDS = 65536
NOALLOC_MAX_SEQS = 1048576
PENDING = 1

DNA2 = 0
BYTE = 1

VARIANT_AUTO = 0
VARIANT_WAVE = 1
VARIANT_WORKGROUP = 2
VARIANT_PLAIN = 3
VARIANT_PAIR = 4
VARIANT_DUAL16 = 5
VARIANT_ROWS16 = 6

SEED_DTYPE = np.dtype([("q", "<i4"), ("t", "<i4"), ("q_pos", "<i4"),
                       ("t_pos", "<i4"), ("k", "<i4")])
RESULT_DTYPE = np.dtype([("score", "<i4"), ("left", "<i4"), ("right", "<i4"),
                         ("seed_score", "<i4"), ("q_begin", "<i4"),
                         ("q_end", "<i4"), ("t_begin", "<i4"),
                         ("t_end", "<i4"), ("cells", "<i8"),
                         ("status", "<i4"), ("reserved", "<i4")])
assert RESULT_DTYPE.itemsize == 48 and SEED_DTYPE.itemsize == 20


class XdropError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class Scoring(ctypes.Structure):
    _fields_ = [("alphabet", ctypes.c_int32),
                ("alphabet_size", ctypes.c_int32),
                ("match", ctypes.c_int32),
                ("mismatch", ctypes.c_int32),
                ("matrix", ctypes.POINTER(ctypes.c_int32)),
                ("gap", ctypes.c_int32),
                ("X", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32),
                ("tile", ctypes.c_int32),
                ("chunk", ctypes.c_int32),
                ("band_cap", ctypes.c_int32),
                ("order", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class CtxOpts(ctypes.Structure):
    _fields_ = [("device_tier_slots", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 7)]


class Request(ctypes.Structure):
    _fields_ = [("seqs", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p),
                ("n_seqs", ctypes.c_int32),
                ("seeds", ctypes.c_void_p),
                ("n_seeds", ctypes.c_int32),
                ("scoring", Scoring),
                ("seq_set", ctypes.c_uint64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32),
                ("streams", ctypes.c_int32),
                ("arena_mib", ctypes.c_int32),
                ("staging_mib", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "requests_submitted", "requests_done", "batches_launched",
        "batches_in_flight", "max_batches_in_flight", "admitted_while_busy",
        "h2d_bytes", "reused_bytes")] + [("reserved", ctypes.c_int64 * 8)]


EXPORTS = ["xdrop_ctx_create", "xdrop_ctx_destroy", "xdrop_extend_batch",
           "xdrop_extend_batch_noalloc",
           "xdrop_ctx_set_timing", "xdrop_last_timing",
           "xdrop_autotune", "xdrop_load_tuning", "xdrop_resolve_options",
           "xdrop_extend_batch_graph",
           "xdrop_last_stats", "xdrop_server_create", "xdrop_server_submit",
           "xdrop_server_poll", "xdrop_server_wait", "xdrop_server_destroy",
           "xdrop_server_put_sequences", "xdrop_server_release_sequences",
           "xdrop_server_stats",
           "xdrop_strerror"]

_lib = None


def bind(lib):
    """Declare the argument and result types of every entry point of a
    loaded copy of the library."""
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.xdrop_strerror.restype = ctypes.c_char_p
    lib.xdrop_strerror.argtypes = [ctypes.c_int]
    lib.xdrop_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(CtxOpts),
                                     ctypes.POINTER(vp)]
    lib.xdrop_ctx_destroy.argtypes = [vp]
    batch_args = [vp, vp, vp, i32, vp, i32, ctypes.POINTER(Scoring),
                  ctypes.POINTER(Options), vp, vp]
    lib.xdrop_extend_batch.argtypes = batch_args
    lib.xdrop_extend_batch_graph.argtypes = batch_args
    lib.xdrop_extend_batch_noalloc.argtypes = batch_args
    lib.xdrop_autotune.argtypes = [vp, vp, vp, i32, vp, i32,
                                   ctypes.POINTER(Scoring), vp, vp,
                                   ctypes.c_char_p, ctypes.POINTER(Options)]
    lib.xdrop_load_tuning.argtypes = [vp, ctypes.c_char_p]
    lib.xdrop_resolve_options.argtypes = [vp, ctypes.POINTER(Scoring), i32,
                                          ctypes.POINTER(Options),
                                          ctypes.POINTER(Options)]
    lib.xdrop_last_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), i32]
    lib.xdrop_ctx_set_timing.argtypes = [vp, i32]
    lib.xdrop_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32,
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.xdrop_server_create.argtypes = [ctypes.c_int, ctypes.c_size_t,
                                        ctypes.POINTER(ServerOpts),
                                        ctypes.POINTER(vp)]
    lib.xdrop_server_submit.argtypes = [vp, ctypes.POINTER(Request),
                                        ctypes.POINTER(ctypes.c_uint64)]
    lib.xdrop_server_poll.argtypes = [vp, ctypes.c_uint64, vp]
    lib.xdrop_server_wait.argtypes = [vp, ctypes.c_uint64, vp,
                                      ctypes.c_int64]
    lib.xdrop_server_destroy.argtypes = [vp]
    lib.xdrop_server_put_sequences.argtypes = [
        vp, vp, vp, i32, i32, ctypes.POINTER(ctypes.c_uint64)]
    lib.xdrop_server_release_sequences.argtypes = [vp, ctypes.c_uint64]
    lib.xdrop_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    for f in EXPORTS:
        if f != "xdrop_strerror":
            getattr(lib, f).restype = ctypes.c_int
    return lib


def load_library(path: str = LIB_PATH):
    """Load libxdrop.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing; build it with "
                           "paper_2304_08662_amd/build.py")
    _lib = bind(ctypes.CDLL(path))
    return _lib


def strerror(status: int) -> str:
    try:
        return load_library().xdrop_strerror(status).decode()
    except RuntimeError:
        return f"status {status}"


def _check(rc: int, what: str):
    if rc != OK:
        raise XdropError(rc, what)


@dataclass
class ScoringSpec:
    """Scoring scheme; matrix (alphabet_size^2, row = query code) or
    match / mismatch."""
    alphabet: int = DNA2
    alphabet_size: int = 4
    match: int = 1
    mismatch: int = -1
    gap: int = -1
    X: int = 15
    matrix: np.ndarray | None = None
    _keep: list = field(default_factory=list, repr=False)

    def c(self) -> Scoring:
        s = Scoring(self.alphabet, self.alphabet_size, self.match,
                    self.mismatch, None, self.gap, self.X)
        if self.matrix is not None:
            m = np.ascontiguousarray(self.matrix, dtype=np.int32)
            self._keep = [m]
            s.matrix = m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        return s


def options(variant=0, tile=0, chunk=0, band_cap=0, order=0,
            waves_per_cu=0) -> Options:
    return Options(variant, tile, chunk, band_cap, order, waves_per_cu)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context on one device (owns the device workspace)."""

    def __init__(self, device: int = 0, device_tier_slots: int = 0, lib=None):
        self.lib = lib if lib is not None else load_library()
        h = ctypes.c_void_p()
        o = CtxOpts(device_tier_slots)
        _check(self.lib.xdrop_ctx_create(device, ctypes.byref(o), ctypes.byref(h)),
               "xdrop_ctx_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            self.lib.xdrop_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def extend_batch(self, seqs, offsets, seeds, scoring: ScoringSpec,
                     results, opts: Options | None = None, stream=None,
                     graph: bool = False, noalloc: bool = False):
        """Enqueue the batch.  seqs: uint8 device tensor (packed stream),
        offsets: int64 (n_seqs+1), seeds: int32 (n, 5), results: any device
        tensor of n * 48 bytes.  graph: record / replay a HIP graph;
        noalloc: the allocation-free entry point.  Returns the status
        (raises on error)."""
        sc = scoring.c()
        n_seeds = int(seeds.shape[0]) if seeds.dim() > 1 else int(seeds.numel() // 5)
        f = (self.lib.xdrop_extend_batch_noalloc if noalloc else
             self.lib.xdrop_extend_batch_graph if graph else
             self.lib.xdrop_extend_batch)
        rc = f(self.handle, _ptr(seqs), _ptr(offsets), int(offsets.numel() - 1),
               _ptr(seeds), n_seeds, ctypes.byref(sc),
               ctypes.byref(opts) if opts is not None else None,
               _ptr(results), _stream_handle(stream))
        _check(rc, "xdrop_extend_batch")
        return rc

    def autotune(self, seqs, offsets, seeds, scoring: ScoringSpec, results,
                 cache_path: str | None = None, stream=None) -> Options:
        sc = scoring.c()
        best = Options()
        rc = self.lib.xdrop_autotune(
            self.handle, _ptr(seqs), _ptr(offsets), int(offsets.numel() - 1),
            _ptr(seeds), int(seeds.shape[0]), ctypes.byref(sc), _ptr(results),
            _stream_handle(stream),
            cache_path.encode() if cache_path else None, ctypes.byref(best))
        _check(rc, "xdrop_autotune")
        return best

    def load_tuning(self, cache_path: str):
        _check(self.lib.xdrop_load_tuning(self.handle, cache_path.encode()),
               "xdrop_load_tuning")

    def resolve_options(self, scoring: ScoringSpec, n_seeds: int,
                        opts: Options | None = None) -> Options:
        """The options a batch of n_seeds seeds would run with."""
        sc = scoring.c()
        out = Options()
        _check(self.lib.xdrop_resolve_options(
            self.handle, ctypes.byref(sc), n_seeds,
            ctypes.byref(opts) if opts is not None else None,
            ctypes.byref(out)), "xdrop_resolve_options")
        return out

    def set_timing(self, on: bool = True):
        _check(self.lib.xdrop_ctx_set_timing(self.handle, int(on)),
               "xdrop_ctx_set_timing")

    def last_timing(self):
        """Per-phase ms summed over the batches recorded since the last read
        (prep, wave kernel, unused, workgroup tier, combine) and their
        number."""
        arr = (ctypes.c_float * 5)()
        nb = ctypes.c_int32()
        _check(self.lib.xdrop_last_timing(self.handle, arr, 5,
                                          ctypes.byref(nb)),
               "xdrop_last_timing")
        return list(arr), int(nb.value)

    def last_stats(self) -> list:
        """Extensions finished per tier: 1, 2, 4, 8 cells per lane, pair
        kernel, block tier, device-memory tier, two-extension 16-bit
        kernel, four-row kernel."""
        arr = (ctypes.c_int64 * 9)()
        _check(self.lib.xdrop_last_stats(self.handle, arr, 9),
               "xdrop_last_stats")
        return list(arr)


class Server:
    """Continuous-batching server (host API of include/xdrop.h)."""

    def __init__(self, device: int = 0, budget_bytes: int = 64 << 30,
                 max_inflight: int = 0, streams: int = 0, arena_mib: int = 0,
                 staging_mib: int = 0, lib=None):
        self.lib = lib if lib is not None else load_library()
        h = ctypes.c_void_p()
        so = ServerOpts(max_inflight, streams, arena_mib, staging_mib)
        _check(self.lib.xdrop_server_create(device, budget_bytes,
                                            ctypes.byref(so), ctypes.byref(h)),
               "xdrop_server_create")
        self.handle = h

    def submit(self, packed: np.ndarray | None, offsets: np.ndarray | None,
               seeds: np.ndarray, scoring: ScoringSpec,
               seq_set: int = 0) -> int:
        """A request over its own sequences (packed, offsets), or over a
        resident set (seq_set from put_sequences; packed and offsets
        None)."""
        seeds = np.ascontiguousarray(seeds).astype(SEED_DTYPE, copy=False)
        if seq_set:
            req = Request(None, None, 0, seeds.ctypes.data, len(seeds),
                          scoring.c(), seq_set)
        else:
            packed = np.ascontiguousarray(packed, dtype=np.uint8)
            offsets = np.ascontiguousarray(offsets, dtype=np.int64)
            req = Request(packed.ctypes.data, offsets.ctypes.data,
                          len(offsets) - 1, seeds.ctypes.data, len(seeds),
                          scoring.c(), 0)
        t = ctypes.c_uint64()
        _check(self.lib.xdrop_server_submit(self.handle, ctypes.byref(req),
                                            ctypes.byref(t)),
               "xdrop_server_submit")
        return int(t.value)

    def put_sequences(self, packed: np.ndarray, offsets: np.ndarray,
                      alphabet: int) -> int:
        """Register sequences that requests seed against (copied once)."""
        packed = np.ascontiguousarray(packed, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        sid = ctypes.c_uint64()
        _check(self.lib.xdrop_server_put_sequences(
            self.handle, packed.ctypes.data, offsets.ctypes.data,
            len(offsets) - 1, alphabet, ctypes.byref(sid)),
            "xdrop_server_put_sequences")
        return int(sid.value)

    def release_sequences(self, set_id: int):
        _check(self.lib.xdrop_server_release_sequences(self.handle, set_id),
               "xdrop_server_release_sequences")

    def stats(self) -> dict:
        st = ServerStats()
        _check(self.lib.xdrop_server_stats(self.handle, ctypes.byref(st)),
               "xdrop_server_stats")
        return {n: int(getattr(st, n)) for n, _ in ServerStats._fields_[:-1]}

    def poll(self, ticket: int, n_seeds: int):
        out = np.zeros(n_seeds, dtype=RESULT_DTYPE)
        rc = self.lib.xdrop_server_poll(self.handle, ticket, out.ctypes.data)
        if rc == PENDING:
            return None
        _check(rc, "xdrop_server_poll")
        return out

    def wait(self, ticket: int, n_seeds: int, timeout_s: float = -1.0):
        out = np.zeros(n_seeds, dtype=RESULT_DTYPE)
        ns = -1 if timeout_s < 0 else int(timeout_s * 1e9)
        rc = self.lib.xdrop_server_wait(self.handle, ticket, out.ctypes.data,
                                        ns)
        if rc == PENDING:
            return None
        _check(rc, "xdrop_server_wait")
        return out

    def close(self):
        if self.handle:
            self.lib.xdrop_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- helpers
def to_device(batch_packed: np.ndarray, offsets: np.ndarray,
              seeds: np.ndarray, device="cuda"):
    """Copy a packed batch to the GPU as tensors (host -> device)."""
    import torch
    packed = np.ascontiguousarray(batch_packed, dtype=np.uint8)
    pad = (-len(packed)) % 16
    if pad:
        packed = np.concatenate([packed, np.zeros(pad, np.uint8)])
    s = np.ascontiguousarray(seeds).astype(SEED_DTYPE, copy=False)
    d_seqs = torch.from_numpy(packed).to(device)
    d_offs = torch.from_numpy(np.ascontiguousarray(offsets, np.int64)).to(device)
    d_seeds = torch.from_numpy(s.view(np.int32).reshape(-1, 5).copy()).to(device)
    return d_seqs, d_offs, d_seeds


def result_buffer(n_seeds: int, device="cuda"):
    import torch
    return torch.zeros((max(n_seeds, 1), 12), dtype=torch.int32, device=device)


def results_to_numpy(t, n_seeds: int) -> np.ndarray:
    a = t.cpu().numpy().reshape(-1)[: n_seeds * 12]
    return np.ascontiguousarray(a).view(RESULT_DTYPE)
