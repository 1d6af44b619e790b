"""The serving loop (its host code and the library's kernels) on the CPU
build of the library (tests/emu): continuous batching, resident sequence
sets shared by requests, memory backpressure; every result equals the
oracle's and the request served alone."""
import numpy as np
import pytest

from paper_2304_08662_amd import inputs, xdrop
from tests.xdrop_testutil import FIELDS, make_batch, oracle_run, product_scoring


@pytest.fixture(scope="module")
def lib():
    from tests.xdrop_emu import EmuLib, build
    build()
    e = EmuLib()
    yield e.lib
    e.close()


def _packed(b):
    return b.packed() if b.alphabet == 4 else b.codes


def _same(a, b):
    return all(np.array_equal(a[f].astype(np.int64), b[f].astype(np.int64))
               for f in FIELDS)


def test_mix_alone_oracle(lib):
    rng = inputs.rng_for(5, 1)
    reqs = [(b, s) for _, b, s in inputs.request_stream(rng, 10, 0.0,
                                                         max_pairs=24)]
    srv = xdrop.Server(0, budget_bytes=2 << 30, lib=lib)
    tickets = [srv.submit(_packed(b), b.offsets, b.seeds, product_scoring(s))
               for b, s in reqs]
    mixed = [srv.wait(t, len(b.seeds), 120) for t, (b, _) in zip(tickets, reqs)]
    for (b, s), m in zip(reqs, mixed):
        t = srv.submit(_packed(b), b.offsets, b.seeds, product_scoring(s))
        assert _same(m, srv.wait(t, len(b.seeds), 120))
        assert _same(m, oracle_run(b, s))
    st = srv.stats()
    assert st["requests_done"] == 2 * len(reqs) and st["batches_launched"] >= 2
    srv.close()


def test_resident_sets_and_release(lib):
    rng = np.random.default_rng(81)
    pool = make_batch([(rng.integers(0, 4, int(rng.integers(50, 400))).astype(np.uint8),
                        rng.integers(0, 4, int(rng.integers(50, 400))).astype(np.uint8),
                        0, 0, 0) for _ in range(16)], 4)
    scheme = inputs.Scheme(4, 1, -1, -1, 20)
    sc = product_scoring(scheme)
    srv = xdrop.Server(0, budget_bytes=2 << 30, lib=lib)
    sid = srv.put_sequences(pool.packed(), pool.offsets, xdrop.DNA2)
    L = np.diff(pool.offsets)
    reqs = []
    for _ in range(6):
        n = int(rng.integers(1, 12))
        q = rng.integers(0, pool.n_seqs, n)
        t = rng.integers(0, pool.n_seqs, n)
        k = np.minimum(np.minimum(L[q], L[t]), 8)
        sd = np.zeros(n, dtype=xdrop.SEED_DTYPE)
        sd["q"], sd["t"], sd["k"] = q, t, k
        sd["q_pos"] = (rng.random(n) * (L[q] - k + 1)).astype(np.int64)
        sd["t_pos"] = (rng.random(n) * (L[t] - k + 1)).astype(np.int64)
        reqs.append(sd)
    tickets = [srv.submit(None, None, sd, sc, seq_set=sid) for sd in reqs]
    # released while requests use it: they still finish, new ones are refused
    srv.release_sequences(sid)
    with pytest.raises(xdrop.XdropError):
        srv.submit(None, None, reqs[0], sc, seq_set=sid)
    for tk, sd in zip(tickets, reqs):
        g = srv.wait(tk, len(sd), 120)
        b = inputs.Batch(pool.codes, pool.offsets, sd, 4)
        assert _same(g, oracle_run(b, scheme))
    st = srv.stats()
    assert st["reused_bytes"] > 0 and st["h2d_bytes"] == len(pool.packed())
    srv.close()


def test_backpressure(lib):
    rng = inputs.rng_for(5, 2)
    reqs = [(b, s) for _, b, s in inputs.request_stream(rng, 8, 0.0,
                                                         max_pairs=64)]
    srv = xdrop.Server(0, budget_bytes=1 << 30, arena_mib=1, staging_mib=1,
                       lib=lib)
    tickets = [srv.submit(_packed(b), b.offsets, b.seeds, product_scoring(s))
               for b, s in reqs]
    for t, (b, s) in zip(tickets, reqs):
        assert _same(srv.wait(t, len(b.seeds), 120), oracle_run(b, s))
    srv.close()
