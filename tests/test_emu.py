"""The library's kernels and host code built for the CPU (tests/emu: every GPU
thread a fiber, the lanes of a wave meeting at every cross-lane operation)
against the oracle, bit-exact.  These run the exact sources of libxdrop.so
without a GPU: long extensions whose sequences wrap the LDS rings, the
register tiers up to 512 cells, the workgroup tier, every launch form, and
samples of the dna-100k workload.  A lane that diverges at a cross-lane
operation, or a wave that stops making progress, aborts the run."""
import os

import numpy as np
import pytest

from paper_2304_08662_amd import inputs, xdrop
from tests.xdrop_testutil import compare, make_batch, oracle_run, product_scoring

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DNA = {c: i for i, c in enumerate("ACGT")}


@pytest.fixture(scope="module")
def emu():
    from tests.xdrop_emu import EmuLib, build
    build()
    e = EmuLib()
    yield e
    e.close()


def test_host_translation_leaves_no_device_instruction():
    """The CPU build's source translation maps every instruction the kernel
    source writes as an asm statement (the bit scans) to a host function;
    only the empty register barriers stay asm, with the host's register
    class.  A new device instruction without a mapping fails here, not in
    the host assembler."""
    import re
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "emu"))
    import build as emu_build
    src = os.path.join(emu_build.CSRC, "xdrop_kernels.hip")
    with open(src, encoding="utf-8") as f:
        text = f.read()
    assert re.search(r'asm\("v_ffb', text)  # the scans are written out
    host = emu_build.host_source(text)
    code = "\n".join(ln.split("//")[0] for ln in host.splitlines())
    for m in re.finditer(r'\basm\s*(?:volatile\s*)?\(\s*"([^"]*)"', code):
        assert m.group(1) == "", m.group(0)
    assert "emu_ffbl_32(" in host and "emu_ffbh_32(" in host


def _enc(s):
    return np.array([DNA[c] for c in s], dtype=np.uint8)


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_golden(emu):
    for name, a, b, X, best, x, y, W in _rows("extensions.txt"):
        batch = make_batch([(_enc(a), _enc(b), 0, 0, 0)], 4)
        g = emu.run(batch, product_scoring(inputs.Scheme(4, 1, -1, -1, int(X))))[0]
        assert (g["score"], g["q_end"], g["t_end"]) == (int(best), int(x), int(y)), name
        if W != "-":
            assert g["cells"] == 1 + int(W), name
    for row in _rows("seeds.txt"):
        name, q, t, qp, tp, k, X = row[:7]
        batch = make_batch([(_enc(q), _enc(t), int(qp), int(tp), int(k))], 4)
        g = emu.run(batch, product_scoring(inputs.Scheme(4, 1, -1, -1, int(X))))[0]
        got = [int(g[f]) for f in ("score", "left", "seed_score", "right",
                                   "q_begin", "q_end", "t_begin", "t_end")]
        assert got == list(map(int, row[7:])), name


def _fuzz(rng, n, alphabet, lmax, related_p=0.6):
    from tests.test_gpu_parity import _fuzz_pairs
    return _fuzz_pairs(rng, n, alphabet, lmax, related_p)


@pytest.mark.parametrize("X", [0, 3, 50, 2**31 - 1])
def test_fuzz_dna(emu, X):
    rng = np.random.default_rng([40, X % 1000])
    batch = make_batch(_fuzz(rng, 60, 4, 300 if X > 1000 else 600), 4)
    scheme = inputs.Scheme(4, 2, -3, -2, X)
    assert not compare(emu.run(batch, product_scoring(scheme)),
                       oracle_run(batch, scheme))


@pytest.mark.parametrize("X", [0, 49, 2**31 - 1])
def test_fuzz_protein(emu, X):
    rng = np.random.default_rng([41, X % 1000])
    batch = make_batch(_fuzz(rng, 60, 20, 250 if X > 1000 else 500), 20)
    scheme = inputs.Scheme(20, gap=-2, X=X,
                           matrix=inputs.stand_in_substitution_matrix())
    assert not compare(emu.run(batch, product_scoring(scheme)),
                       oracle_run(batch, scheme))


def test_long_byte_codes_wrap_rings(emu):
    """Byte-coded pairs of 3,000-10,000 codes: every extension passes the
    2,048-code LDS ring several times (the mirror words and the ring margin
    of the 4- and 8-cell tiers included); related and unrelated pairs, left
    and right extensions, seeds near both ends, and an X large enough that
    windows widen to 8 cells per lane and beyond."""
    rng = np.random.default_rng(42)
    M = inputs.stand_in_substitution_matrix()
    pairs = []
    for i in range(8):
        L = int(rng.integers(3000, 10001))
        q = rng.integers(0, 20, L).astype(np.uint8)
        if i % 2 == 0:
            t, _ = inputs.mutate(rng, q, 0.2, 0.03, 0.03, 20)
        else:
            t = rng.integers(0, 20, int(rng.integers(3000, 10001))).astype(np.uint8)
        k = 6
        where = [0.02, 0.5, 0.98][i % 3]
        qp = int(where * (len(q) - k))
        tp = min(int(where * (len(t) - k)), len(t) - k)
        t = t.copy()
        t[tp:tp + k] = q[qp:qp + k]
        pairs.append((q, t, qp, tp, k))
    batch = make_batch(pairs, 20)
    for X in (49, 400):
        scheme = inputs.Scheme(20, gap=-2, X=X, matrix=M)
        g = emu.run(batch, product_scoring(scheme))
        assert not compare(g, oracle_run(batch, scheme)), X
    stats = emu.last_stats()
    assert stats[2] + stats[3] + stats[5] > 0, stats  # wide tiers reached


def test_wide_bands_all_tiers(emu):
    rng = np.random.default_rng(43)
    pairs = []
    for L in (40, 300, 600, 1100):
        q = rng.integers(0, 4, L).astype(np.uint8)
        t = rng.integers(0, 4, L + int(rng.integers(-20, 20))).astype(np.uint8)
        pairs.append((q, t, 0, 0, 0))
    batch = make_batch(pairs, 4)
    scheme = inputs.Scheme(4, 1, -1, -1, 2**31 - 1)
    assert not compare(emu.run(batch, product_scoring(scheme)),
                       oracle_run(batch, scheme))
    stats = emu.last_stats()
    assert stats[3] >= 1 and stats[5] >= 1, stats


def test_launch_forms(emu):
    rng = np.random.default_rng(44)
    batch = make_batch(_fuzz(rng, 40, 4, 900, related_p=0.4), 4)
    scheme = inputs.Scheme(4, 1, -1, -1, 40)
    ref = oracle_run(batch, scheme)
    for v, tile, chunk, order in [(1, 1, 1, 0), (1, 4, 8, 1), (3, 2, 1, 0),
                                  (2, 1, 1, 0), (4, 1, 1, 0), (4, 2, 4, 1)]:
        g = emu.run(batch, product_scoring(scheme),
                    xdrop.options(v, tile, chunk, 0, order))
        assert not compare(g, ref), (v, tile, chunk, order)


def test_dna_100k_sample(emu):
    """Seeds of the dna-100k workload (X = 50): the widest bands of its
    0.4% sample (up to ~700 cells, past the 512-cell register window) and
    ordinary related and unrelated pairs of 1-30 kb."""
    batch, scheme = inputs.workload("dna-100k", 0.004)
    idx = [166, 76, 107, 330, 0, 1, 2, 3, 4, 5]
    b = batch.subset(idx)
    g = emu.run(b, product_scoring(scheme))
    assert not compare(g, oracle_run(b, scheme))
    assert emu.last_stats()[5] >= 2  # bands past 512 cells


@pytest.mark.parametrize("alphabet", [4, 20])
def test_block_tier_bands_512_to_2048_and_beyond(emu, alphabet):
    """X -> infinity on unrelated pairs: bands grow to min(m, n) + 1 cells.
    Lengths 520..2000 end on the block tier (four waves, 1,024 then 2,048
    cells), one pair of 2,300 goes on to the device-memory tier; left and
    right extensions, seeds inside the pairs."""
    rng = np.random.default_rng([45, alphabet])
    pairs = []
    for L in (520, 700, 1000, 1500, 2000, 2300):
        q = rng.integers(0, alphabet, L).astype(np.uint8)
        t = rng.integers(0, alphabet, L + int(rng.integers(-30, 30))).astype(np.uint8)
        pairs.append((q, t, 0, 0, 0))
    for L in (1400, 2600):  # a seed in the middle: both sides wide
        q = rng.integers(0, alphabet, L).astype(np.uint8)
        t = rng.integers(0, alphabet, L).astype(np.uint8)
        t[L // 2:L // 2 + 6] = q[L // 2:L // 2 + 6]
        pairs.append((q, t, L // 2, L // 2, 6))
    batch = make_batch(pairs, alphabet)
    if alphabet == 4:
        scheme = inputs.Scheme(4, 1, -1, -1, 2**31 - 1)
    else:
        scheme = inputs.Scheme(20, gap=-2, X=2**31 - 1,
                               matrix=inputs.stand_in_substitution_matrix())
    assert not compare(emu.run(batch, product_scoring(scheme)),
                       oracle_run(batch, scheme))
    stats = emu.last_stats()
    assert stats[5] >= 5 and stats[6] >= 1, stats


def test_noalloc_equals_extend_batch_twice(emu):
    """The allocation-free entry point on the CPU build: identical to
    xdrop_extend_batch on two calls in a row, the second smaller."""
    rng = np.random.default_rng(60)
    pairs = _fuzz(rng, 80, 4, 900, related_p=0.5)
    for L in (2300,):
        pairs.append((rng.integers(0, 4, L).astype(np.uint8),
                      rng.integers(0, 4, L).astype(np.uint8), 0, 0, 0))
    big = make_batch(pairs, 4)
    small = make_batch(_fuzz(rng, 20, 20, 400), 20)
    for batch, scheme in (
            (big, inputs.Scheme(4, 1, -1, -1, 2**31 - 1)),
            (small, inputs.Scheme(20, gap=-2, X=49,
                                  matrix=inputs.stand_in_substitution_matrix()))):
        sc = product_scoring(scheme)
        ref = emu.run(batch, sc)
        got = emu.run(batch, sc, noalloc=True)
        assert not compare(got, ref)
        assert not compare(got, oracle_run(batch, scheme))


def test_seeds_share_sequences(emu):
    from tests.xdrop_testutil import shared_sequence_batches
    rng = np.random.default_rng([82, 4])
    shared, unique = shared_sequence_batches(rng, n_seeds=60)
    scheme = inputs.Scheme(4, 1, -1, -1, 20)
    sc = product_scoring(scheme)
    g = emu.run(shared, sc)
    assert not compare(g, emu.run(unique, sc))
    assert not compare(g, oracle_run(shared, scheme))


@pytest.mark.parametrize("alphabet,X", [(20, 49), (4, 15), (4, 0)])
def test_dual16_kernel(emu, alphabet, X):
    """The two-extension 16-bit kernel on the CPU build: fuzz batches, a
    long-extension sample (ring wrap), hand-on of wide bands."""
    rng = np.random.default_rng([93, alphabet, X])
    b = make_batch(_fuzz(rng, 60, alphabet, 700), alphabet)
    s = (inputs.Scheme(4, 2, -3, -2, X) if alphabet == 4 else
         inputs.Scheme(20, gap=-2, X=X,
                       matrix=inputs.stand_in_substitution_matrix()))
    g = emu.run(b, product_scoring(s), xdrop.options(variant=5))
    assert not compare(g, oracle_run(b, s))
    assert emu.last_stats()[7] > 0


def test_dual16_long_extensions(emu):
    b, s = inputs.workload("dna-tail", 1.0)
    n = len(b.seeds)
    b = b.subset([n - 1, n - 2, 0, 1])
    g = emu.run(b, product_scoring(s), xdrop.options(variant=5))
    assert not compare(g, oracle_run(b, s))
    assert emu.last_stats()[7] == 8


@pytest.mark.parametrize("variant,tier", [(4, 4), (6, 8)])
@pytest.mark.parametrize("alphabet,X", [(20, 49), (4, 15), (4, 0), (4, 200)])
def test_row_kernels(emu, alphabet, X, variant, tier):
    """The row kernels on the CPU build (two rows of 32 lanes, four rows of
    16 lanes per wave): fuzz batches of related and unrelated pairs; rows
    refilled from the queue as their extensions end, bands that fill a row
    handed on to the wave kernel (X = 200 makes most of them do so)."""
    rng = np.random.default_rng([95, alphabet, X])
    b = make_batch(_fuzz(rng, 60, alphabet, 700), alphabet)
    s = (inputs.Scheme(4, 2, -3, -2, X) if alphabet == 4 else
         inputs.Scheme(20, gap=-2, X=X,
                       matrix=inputs.stand_in_substitution_matrix()))
    for chunk in (1, 4):
        g = emu.run(b, product_scoring(s), xdrop.options(variant=variant,
                                                         chunk=chunk))
        assert not compare(g, oracle_run(b, s)), chunk
        st = emu.last_stats()
        assert sum(st) == 2 * len(b.seeds), st
    assert st[tier] > 0, st


@pytest.mark.parametrize("variant,tier,X", [(4, 4, 15), (6, 8, 6)])
def test_row_kernels_long_extensions(emu, variant, tier, X):
    """Extensions of 50-100 kb on the row kernels: ring wrap and many window
    slides, beside short ones that end early and free their row (X = 6 keeps
    the bands of the long extensions within 16-lane rows)."""
    b, s = inputs.workload("dna-tail", 1.0)
    s = inputs.Scheme(4, s.match, s.mismatch, s.gap, X)
    n = len(b.seeds)
    b = b.subset([n - 1, n - 2, 0, 1, 2, 3])
    g = emu.run(b, product_scoring(s), xdrop.options(variant=variant))
    assert not compare(g, oracle_run(b, s))
    assert emu.last_stats()[tier] == 12


@pytest.mark.parametrize("asize", [20, 32])
def test_symbol_check(emu, asize):
    """The symbol check on the CPU build: out-of-alphabet codes (just above
    the alphabet, up to 127, and 128..255) in the first, last or any byte of
    sequences of 1..130 bytes that share words and 16-byte pieces with their
    neighbours; a bad code in a neighbour never marks a sequence.  Statuses
    and results equal the oracle's seed by seed."""
    rng = np.random.default_rng([41, asize])
    pairs, n_bad = [], 0
    for i in range(300):
        lq = int(rng.integers(1, 131))
        q = rng.integers(0, asize, lq).astype(np.uint8)
        t = q.copy()
        kind = i % 6
        if kind == 1:
            q[0] = asize + int(rng.integers(0, 128 - asize))
        elif kind == 2:
            t[-1] = asize + int(rng.integers(0, 128 - asize))
        elif kind == 3:
            q[int(rng.integers(0, lq))] = int(rng.integers(128, 256))
        elif kind == 4:
            t[int(rng.integers(0, lq))] = 255
        n_bad += kind in (1, 2, 3, 4)
        k = int(rng.integers(0, min(lq, 6) + 1))
        pos = int(rng.integers(0, lq - k + 1))
        pairs.append((q, t, pos, pos, k))
    b = make_batch(pairs, asize)
    m = rng.integers(-4, 9, (asize, asize)).astype(np.int32)
    m = np.minimum(m, m.T)
    np.fill_diagonal(m, 5)
    s = inputs.Scheme(asize, gap=-2, X=10, matrix=m)
    g = emu.run(b, product_scoring(s))
    assert not compare(g, oracle_run(b, s))
    assert (g["status"] == xdrop.E_SYMBOL).sum() == n_bad
