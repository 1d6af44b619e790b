"""Serving loop: continuous batching of requests of mixed size and alphabet;
every result must equal the oracle's and the request's result when served
alone (bit-exact)."""
import numpy as np
import pytest

from paper_2304_08662_amd import inputs
from tests.xdrop_testutil import FIELDS, oracle_run, product_scoring

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_08662_amd import xdrop
    return xdrop


def _packed(b):
    return b.packed() if b.alphabet == 4 else b.codes


def _same(a, b):
    return all(np.array_equal(a[f].astype(np.int64), b[f].astype(np.int64))
               for f in FIELDS)


def test_alone_equals_mix_equals_oracle(xd):
    rng = inputs.rng_for(5, 1)
    reqs = [(b, s) for _, b, s in inputs.request_stream(rng, 24, 0.0,
                                                         max_pairs=64)]
    srv = xd.Server(0, budget_bytes=2 << 30)
    # mixed: everything submitted at once, served in overlapping micro-batches
    tickets = [srv.submit(_packed(b), b.offsets, b.seeds, product_scoring(s))
               for b, s in reqs]
    mixed = [srv.wait(t, len(b.seeds), 120) for t, (b, _) in zip(tickets, reqs)]
    # alone: one request in flight at a time
    for (b, s), m in zip(reqs, mixed):
        t = srv.submit(_packed(b), b.offsets, b.seeds, product_scoring(s))
        alone = srv.wait(t, len(b.seeds), 120)
        assert m is not None and alone is not None
        assert _same(m, alone)
        assert _same(m, oracle_run(b, s))
    srv.close()


def test_budget_backpressure_and_rejection(xd):
    rng = inputs.rng_for(5, 2)
    reqs = [(b, s) for _, b, s in inputs.request_stream(rng, 12, 0.0,
                                                         max_pairs=128)]
    # a 1 MiB sequence arena holds only a few requests at once: the rest
    # waits for space and is still served correctly
    srv = xd.Server(0, budget_bytes=1 << 30, arena_mib=1)
    tickets = [srv.submit(_packed(b), b.offsets, b.seeds, product_scoring(s))
               for b, s in reqs]
    for t, (b, s) in zip(tickets, reqs):
        g = srv.wait(t, len(b.seeds), 120)
        assert _same(g, oracle_run(b, s))
    # a request larger than the whole arena can never be admitted
    big = np.zeros(16, dtype=np.uint8)  # never read: sized from offsets
    offs = np.array([0, 4 << 30], dtype=np.int64)
    seeds = np.zeros(1, dtype=xd.SEED_DTYPE)
    with pytest.raises(xd.XdropError) as e:
        srv.submit(big, offs, seeds, product_scoring(inputs.Scheme(4)))
    assert e.value.status == xd.E_BUDGET
    srv.close()
