"""Autotuner: tuned launch options are keyed by (device architecture,
alphabet, X class, batch size class); a cache line is used only when it
holds every key, a later line of the same key replaces an earlier one, and
a tuned choice never changes a result.  The CPU part runs the host code of
the library in its CPU build (tests/emu); the GPU part tunes a real batch."""
import ctypes
import json
import os

import numpy as np
import pytest

from paper_2304_08662_amd import inputs, xdrop
from tests.xdrop_testutil import compare, make_batch, oracle_run, product_scoring


def _resolve(lib, ctx, sc, n_seeds, opts=None):
    out = xdrop.Options()
    c = sc.c()
    rc = lib.xdrop_resolve_options(ctx, ctypes.byref(c), n_seeds,
                                   ctypes.byref(opts) if opts else None,
                                   ctypes.byref(out))
    assert rc == 0, rc
    return (out.variant, out.tile, out.chunk)


@pytest.fixture(scope="module")
def emu():
    from tests.xdrop_emu import EmuLib, build
    build()
    e = EmuLib()
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    e.lib.xdrop_load_tuning.argtypes = [vp, ctypes.c_char_p]
    e.lib.xdrop_resolve_options.argtypes = [vp, ctypes.POINTER(xdrop.Scoring),
                                            i32, ctypes.POINTER(xdrop.Options),
                                            ctypes.POINTER(xdrop.Options)]
    yield e
    e.close()


def _line(**kw):
    base = {"arch": "gfx950-emu", "alphabet": 0, "x_class": 0,
            "size_class": 0, "variant": 1, "tile": 2, "chunk": 4,
            "waves_per_cu": 0}
    base.update(kw)
    return json.dumps({k: v for k, v in base.items() if v is not None})


def test_cache_keys_read_back(emu, tmp_path):
    dna15 = xdrop.ScoringSpec(xdrop.DNA2, 4, 1, -1, -1, 15)     # x class 0
    dna50 = xdrop.ScoringSpec(xdrop.DNA2, 4, 1, -1, -1, 50)     # x class 1
    prot = xdrop.ScoringSpec(xdrop.BYTE, 20, 0, 0, -2, 49,
                             matrix=inputs.stand_in_substitution_matrix())
    default = _resolve(emu.lib, emu.ctx, dna15, 1000)
    path = tmp_path / "tune.jsonl"
    path.write_text("\n".join([
        _line(variant=1, tile=2, chunk=4),                       # (0, 0, 0)
        _line(variant=1, tile=4, chunk=16),                      # replaces it
        _line(x_class=1, variant=3, tile=8, chunk=1),            # (0, 1, 0)
        _line(alphabet=1, x_class=1, size_class=2, variant=1, tile=1,
              chunk=8),                                          # (1, 1, 2)
        _line(arch="gfx942", x_class=2, variant=2),              # other arch
        _line(x_class=2, waves_per_cu=None, variant=2),          # key missing
        _line(x_class=2, variant=1, tile=3),                     # bad tile
    ]) + "\n")
    assert emu.lib.xdrop_load_tuning(emu.ctx, str(path).encode()) == 0
    assert _resolve(emu.lib, emu.ctx, dna15, 1000) == (1, 4, 16)
    assert _resolve(emu.lib, emu.ctx, dna50, 1000) == (3, 8, 1)
    assert _resolve(emu.lib, emu.ctx, prot, 100000) == (1, 1, 8)
    # other size class, or an X class with no usable line: the defaults
    assert _resolve(emu.lib, emu.ctx, dna15, 5000) == _resolve(
        emu.lib, emu.ctx, dna15, 5000, xdrop.options())
    big_x = xdrop.ScoringSpec(xdrop.DNA2, 4, 1, -1, -1, 400)
    assert _resolve(emu.lib, emu.ctx, big_x, 1000) == default
    # the caller's fields win over the tuned entry
    assert _resolve(emu.lib, emu.ctx, dna15, 1000,
                    xdrop.options(variant=3))[0] == 3
    # a file with no usable line is refused
    bad = tmp_path / "bad.jsonl"
    bad.write_text(_line(arch="gfx942") + "\n")
    assert emu.lib.xdrop_load_tuning(emu.ctx, str(bad).encode()) == xdrop.E_INVALID


def test_tuned_choice_keeps_results(emu, tmp_path):
    """A batch run under the tuned entry of its key equals the oracle."""
    from tests.test_gpu_parity import _fuzz_pairs
    rng = np.random.default_rng(70)
    batch = make_batch(_fuzz_pairs(rng, 30, 4, 500), 4)
    scheme = inputs.Scheme(4, 1, -1, -1, 15)
    ref = oracle_run(batch, scheme)
    for v, t, ch in ((4, 2, 4), (2, 1, 1), (1, 8, 2)):
        path = tmp_path / f"t{v}.jsonl"
        path.write_text(_line(variant=v, tile=t, chunk=ch) + "\n")
        assert emu.lib.xdrop_load_tuning(emu.ctx, str(path).encode()) == 0
        assert not compare(emu.run(batch, product_scoring(scheme)), ref), v


@pytest.mark.gpu
def test_autotune_then_batch_on_gpu(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests.test_gpu_parity import _fuzz_pairs
    from tests.xdrop_testutil import Runner
    r = Runner()
    try:
        rng = np.random.default_rng(71)
        batch = make_batch(_fuzz_pairs(rng, 400, 4, 800, related_p=0.7), 4)
        scheme = inputs.Scheme(4, 1, -1, -1, 20)
        sc = product_scoring(scheme)
        d = r.upload(batch)
        res = xdrop.result_buffer(len(batch.seeds))
        cache = str(tmp_path / "tune.jsonl")
        best = r.ctx.autotune(*d, sc, res, cache_path=cache, stream=r.stream)
        r.stream.synchronize()
        chosen = (best.variant, best.tile, best.chunk)
        assert best.variant in (1, 2, 3, 4), chosen
        got = r.ctx.resolve_options(sc, len(batch.seeds))
        assert got.variant == best.variant and got.tile == best.tile
        # the batch under the tuned choice (automatic options) is bit-exact
        ref = oracle_run(batch, scheme)
        assert not compare(r.run(batch, scheme, dev=d), ref)
        line = json.loads(open(cache).read().splitlines()[-1])
        assert line["arch"].startswith("gfx") and line["size_class"] == 0
        assert line["x_class"] == 0 and line["alphabet"] == 0
        assert line["plain_ms"] > 0 and line["ms"] <= line["plain_ms"]
        # a fresh context reads the entry back
        ctx2 = xdrop.Context(0)
        try:
            ctx2.load_tuning(cache)
            o2 = ctx2.resolve_options(sc, len(batch.seeds))
            assert (o2.variant, o2.tile, o2.chunk) == (
                got.variant, got.tile, got.chunk)
        finally:
            ctx2.close()
    finally:
        r.ctx.close()
