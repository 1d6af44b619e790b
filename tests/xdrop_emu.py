"""The library's C ABI on the CPU emulation (tests/emu): the kernel and host
sources of libxdrop.so built for the host, every GPU thread a fiber.  Test
infrastructure only; "device" buffers are host numpy arrays."""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))

from paper_2304_08662_amd import xdrop  # noqa: E402  (ctypes structs only)


def build(csrc=None, out=None, include=None):
    import build as emu_build  # tests/emu/build.py
    kw = {"include": include}
    if out:
        kw["out"] = out
    return emu_build.build(csrc, **kw)


class EmuLib:
    def __init__(self, path=None):
        if path is None:
            import build as emu_build
            path = emu_build.LIB
            if not os.path.exists(path):
                build()
        lib = xdrop.bind(ctypes.CDLL(path))
        self.lib = lib
        h = ctypes.c_void_p()
        rc = lib.xdrop_ctx_create(0, None, ctypes.byref(h))
        assert rc == 0, rc
        self.ctx = h

    def close(self):
        if self.ctx:
            self.lib.xdrop_ctx_destroy(self.ctx)
            self.ctx = None

    def run(self, batch, scoring: "xdrop.ScoringSpec", opts=None,
            noalloc=False):
        packed = batch.packed() if batch.alphabet == 4 and \
            scoring.alphabet == xdrop.DNA2 else \
            np.ascontiguousarray(batch.codes, dtype=np.uint8)
        pad = (-len(packed)) % 16 + 16
        packed = np.concatenate([packed, np.zeros(pad, np.uint8)])
        offs = np.ascontiguousarray(batch.offsets, dtype=np.int64)
        sd = np.ascontiguousarray(batch.seeds).astype(xdrop.SEED_DTYPE,
                                                      copy=False)
        n = len(sd)
        res = np.zeros(max(n, 1), dtype=xdrop.RESULT_DTYPE)
        res.view(np.int32)[:] = -12345
        sc = scoring.c()
        f = (self.lib.xdrop_extend_batch_noalloc if noalloc
             else self.lib.xdrop_extend_batch)
        rc = f(
            self.ctx, packed.ctypes.data, offs.ctypes.data, len(offs) - 1,
            sd.ctypes.data, n, ctypes.byref(sc),
            ctypes.byref(opts) if opts is not None else None,
            res.ctypes.data, None)
        if rc != 0:
            raise RuntimeError(f"xdrop_extend_batch (emu): status {rc}")
        return res[:n]

    def last_stats(self):
        arr = (ctypes.c_int64 * 9)()
        assert self.lib.xdrop_last_stats(self.ctx, arr, 9) == 0
        return list(arr)
