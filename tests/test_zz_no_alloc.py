"""The allocation-free entry point (xdrop_extend_batch_noalloc) against
xdrop_extend_batch through the C ABI: identical results, bit for bit, on two
calls in a row (the second batch smaller, so the fixed scratch holds the
first call's leftovers), and against the oracle; batches past the scratch
limits are refused before anything runs."""
import numpy as np
import pytest

from paper_2304_08662_amd import inputs
from tests.xdrop_testutil import FIELDS, Runner, compare, make_batch, oracle_run

pytestmark = pytest.mark.gpu


def _pairs(rng, n, alphabet, lmax):
    from tests.test_gpu_parity import _fuzz_pairs
    return _fuzz_pairs(rng, n, alphabet, lmax, related_p=0.5)


def _same(a, b):
    return [(i, f) for i in range(len(a)) for f in FIELDS
            if int(a[i][f]) != int(b[i][f])]


def test_noalloc_equals_extend_batch_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = Runner()
    try:
        rng = np.random.default_rng(60)
        # first call: 400 DNA seeds, X = 50, plus two unrelated pairs whose
        # bands pass 2,048 cells (device-memory tier rings in the scratch)
        pairs = _pairs(rng, 400, 4, 900)
        for L in (2300, 2500):
            pairs.append((rng.integers(0, 4, L).astype(np.uint8),
                          rng.integers(0, 4, L).astype(np.uint8), 0, 0, 0))
        big = make_batch(pairs, 4)
        s_big = inputs.Scheme(4, 1, -1, -1, 50)
        # second call: fewer seeds, byte codes (symbol-state region used)
        small = make_batch(_pairs(rng, 60, 20, 500), 20)
        s_small = inputs.Scheme(20, gap=-2, X=49,
                                matrix=inputs.stand_in_substitution_matrix())
        wide = make_batch(pairs[-2:], 4)
        s_wide = inputs.Scheme(4, 1, -1, -1, 2**31 - 1)
        for batch, scheme in ((big, s_big), (wide, s_wide), (small, s_small)):
            ref = r.run(batch, scheme)
            got = r.run(batch, scheme, noalloc=True)
            assert not _same(got, ref), _same(got, ref)[:5]
            assert not compare(got, oracle_run(batch, scheme))
        assert r.ctx.last_stats()[6] == 0  # (the small batch ran last)
    finally:
        r.ctx.close()


def test_noalloc_limits():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_08662_amd import xdrop
    r = Runner()
    try:
        q = np.zeros(8, np.uint8)
        batch = make_batch([(q, q, 0, 0, 1)] * (xdrop.NOALLOC_MAX_SEEDS + 1), 4)
        with pytest.raises(xdrop.XdropError) as ei:
            r.run(batch, inputs.Scheme(4, 1, -1, -1, 5), noalloc=True)
        assert ei.value.status == xdrop.E_SCRATCH
    finally:
        r.ctx.close()
