"""Pins for the CPU oracle: it is checked here against things other than
itself -- hand-worked tables, the unpruned limit X -> infinity (a row-major
textbook DP and brute-force path enumeration, both written independently
below), closed forms and invariants.  CPU only."""
import itertools
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DNA = {c: i for i, c in enumerate("ACGT")}
BIG_X = 1 << 40


def enc(s):
    return np.array([DNA[c] for c in s], dtype=np.uint8)


def read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- references
def textbook_prefix_best(a, b, M, gap):
    """Unpruned semi-global DP filled row by row (NW with free end):
    best over all cells of the prefix-alignment score, first reached in
    antidiagonal order, lowest x on ties."""
    m, n = len(a), len(b)
    S = np.zeros((m + 1, n + 1), dtype=np.int64)
    for x in range(m + 1):
        for y in range(n + 1):
            if x == 0 and y == 0:
                continue
            c = []
            if x and y:
                c.append(S[x - 1, y - 1] + M[a[x - 1], b[y - 1]])
            if x:
                c.append(S[x - 1, y] + gap)
            if y:
                c.append(S[x, y - 1] + gap)
            S[x, y] = max(c)
    best = None
    for d in range(m + n + 1):
        for x in range(max(0, d - n), min(m, d) + 1):
            v = S[x, d - x]
            if best is None or v > best[0]:
                best = (int(v), x, d - x)
    return best, S


def brute_force_paths(a, b, M, gap):
    """Best score over every monotone alignment path from (0,0), by explicit
    enumeration; returns {cell: best path score}."""
    m, n = len(a), len(b)
    best = {}

    def walk(x, y, s):
        if best.get((x, y), None) is None or s > best[(x, y)]:
            best[(x, y)] = s
        if x < m and y < n:
            walk(x + 1, y + 1, s + int(M[a[x], b[y]]))
        if x < m:
            walk(x + 1, y, s + gap)
        if y < n:
            walk(x, y + 1, s + gap)

    walk(0, 0, 0)
    return best


# ---------------------------------------------------------------- golden
@pytest.mark.parametrize("row", read_rows("extensions.txt"), ids=lambda r: r[0])
@pytest.mark.parametrize("tier", ["dense", "span"])
def test_golden_extensions(row, tier):
    name, a, b, X, best, x, y, W = row
    sc = oracle.dna_scoring(1, -1, -1, int(X))
    got = oracle.extend(enc(a), enc(b), sc, tier=tier)
    assert got[:3] == (int(best), int(x), int(y)), name
    if W != "-":
        assert got[3] == int(W), name


def test_golden_t2_matrix():
    rows = read_rows("t2_matrix.txt")
    (best, x, y, W), S, F = oracle.extend_matrix(enc("ACGTT"), enc("AGGT"),
                                                 oracle.dna_scoring(X=1))
    for i, r in enumerate(rows):
        for j, v in enumerate(r):
            if v == ".":
                assert not F[i, j], (i, j)
            else:
                assert F[i, j] and S[i, j] == int(v), (i, j)


@pytest.mark.parametrize("row", read_rows("seeds.txt"), ids=lambda r: r[0])
def test_golden_seeds(row):
    name, q, t, qp, tp, k, X = row[:7]
    exp = list(map(int, row[7:]))
    sc = oracle.dna_scoring(1, -1, -1, int(X))
    r = oracle.seed_extend(enc(q), enc(t), int(qp), int(tp), int(k), sc)
    got = [r[f] for f in ("score", "left", "seed_score", "right", "q_begin",
                          "q_end", "t_begin", "t_end")]
    assert got == exp, name
    assert r["status"] == 0


def test_seed_s2_unchanged_at_infinite_x():
    sc = oracle.dna_scoring(X=BIG_X)
    r = oracle.seed_extend(enc("CATTAGACCA"), enc("CTTAGACGCA"), 3, 2, 4, sc)
    assert (r["score"], r["q_begin"], r["t_begin"]) == (7, 2, 1)


# ---------------------------------------------------------------- X -> inf
def _rand_matrix(rng, A):
    M = rng.integers(-4, 6, size=(A, A)).astype(np.int32)
    return M


@pytest.mark.parametrize("seed", range(40))
def test_infinite_x_equals_brute_force(seed):
    rng = np.random.default_rng([1, seed])
    A = 4 if seed % 2 == 0 else 3
    m, n = rng.integers(0, 6, size=2)
    a = rng.integers(0, A, size=m).astype(np.uint8)
    b = rng.integers(0, A, size=n).astype(np.uint8)
    M = _rand_matrix(rng, A)
    gap = int(rng.integers(-3, 0))
    paths = brute_force_paths(a, b, M, gap)
    exp = None
    for d in range(m + n + 1):
        for x in range(max(0, d - n), min(m, d) + 1):
            v = paths[(x, d - x)]
            if exp is None or v > exp[0]:
                exp = (v, x, d - x)
    sc = oracle.Scoring(M, gap, BIG_X)
    (best, x, y, W), S, F = oracle.extend_matrix(a, b, sc)
    assert (best, x, y) == exp
    assert F.all()
    for (i, j), v in paths.items():
        assert S[i, j] == v
    assert W == (m + 1) * (n + 1)


@pytest.mark.parametrize("seed", range(20))
def test_infinite_x_equals_textbook_dp(seed):
    rng = np.random.default_rng([2, seed])
    m, n = rng.integers(0, 40, size=2)
    A = int(rng.choice([4, 20]))
    a = rng.integers(0, A, size=m).astype(np.uint8)
    b = rng.integers(0, A, size=n).astype(np.uint8)
    M = rng.integers(-4, 8, size=(A, A)).astype(np.int32)
    gap = int(rng.integers(-4, 0))
    exp, S_ref = textbook_prefix_best(a, b, M, gap)
    sc = oracle.Scoring(M, gap, BIG_X)
    for tier in ("dense", "span"):
        assert oracle.extend(a, b, sc, tier=tier)[:3] == exp
    _, S, F = oracle.extend_matrix(a, b, sc)
    assert F.all() and (S == S_ref).all()


def test_infinite_x_is_reached_by_a_finite_x():
    # X larger than any possible drop behaves as X = infinity
    rng = np.random.default_rng(3)
    a = rng.integers(0, 4, 30).astype(np.uint8)
    b = rng.integers(0, 4, 25).astype(np.uint8)
    big = oracle.extend(a, b, oracle.dna_scoring(X=BIG_X))
    x_enough = (30 + 25) * 1 + 1
    assert oracle.extend(a, b, oracle.dna_scoring(X=x_enough)) == big


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("X", [0, 1, 3, 15, 50, BIG_X])
@pytest.mark.parametrize("L", [0, 1, 2, 17, 100])
def test_identical_dna_closed_form(X, L):
    rng = np.random.default_rng(L)
    s = rng.integers(0, 4, L).astype(np.uint8)
    for match in (1, 2, 5):
        sc = oracle.dna_scoring(match, -1, -1, X)
        for tier in ("dense", "span"):
            best, x, y, _ = oracle.extend(s, s, sc, tier=tier)
            assert (best, x, y) == (L * match, L, L)


def test_identical_protein_matches_unpruned():
    # identity score sum M[c, c] is the answer only if the unpruned DP agrees;
    # check against the textbook DP rather than assuming it
    rng = np.random.default_rng(5)
    M = rng.integers(-4, 3, size=(20, 20)).astype(np.int32)
    M = np.triu(M) + np.triu(M, 1).T
    np.fill_diagonal(M, rng.integers(4, 12, 20))
    s = rng.integers(0, 20, 30).astype(np.uint8)
    exp, _ = textbook_prefix_best(s, s, M, -2)
    assert oracle.extend(s, s, oracle.Scoring(M, -2, BIG_X))[:3] == exp


def test_empty_extensions():
    sc = oracle.dna_scoring(X=5)
    assert oracle.extend(enc(""), enc(""), sc) == (0, 0, 0, 1)
    assert oracle.extend(enc("ACGT"), enc(""), sc)[:3] == (0, 0, 0)
    assert oracle.extend(enc(""), enc("ACGT"), sc)[:3] == (0, 0, 0)
    # seed at both sequence ends: both extensions empty
    r = oracle.seed_extend(enc("ACG"), enc("ACG"), 0, 0, 3, sc)
    assert (r["score"], r["left"], r["right"], r["q_begin"], r["q_end"]) == \
        (3, 0, 0, 0, 3)


# ---------------------------------------------------------------- invariants
def _random_pair(rng, related=True, A=4, L=(0, 120)):
    m = int(rng.integers(*L))
    a = rng.integers(0, A, m).astype(np.uint8)
    if related:
        b = a.copy()
        mut = rng.random(m) < 0.2
        b[mut] = rng.integers(0, A, mut.sum())
        if m > 4:
            cut = int(rng.integers(0, m))
            b = np.concatenate([b[:cut], b[cut + 1:]])
    else:
        b = rng.integers(0, A, int(rng.integers(*L))).astype(np.uint8)
    return a, b


@pytest.mark.parametrize("seed", range(30))
def test_tiers_agree_and_invariants(seed):
    rng = np.random.default_rng([7, seed])
    a, b = _random_pair(rng, related=seed % 3 != 0)
    X = int(rng.choice([0, 1, 2, 5, 10, 30]))
    sc = oracle.dna_scoring(1, -1, -1, X)
    d = oracle.extend(a, b, sc, "dense")
    s = oracle.extend(a, b, sc, "span")
    assert d == s
    assert d[0] >= 0
    inf = oracle.extend(a, b, oracle.dna_scoring(X=BIG_X))
    assert d[0] <= inf[0]
    # pointwise: a pruned DP never exceeds the unpruned one
    _, S, F = oracle.extend_matrix(a, b, sc)
    _, Si, Fi = oracle.extend_matrix(a, b, oracle.dna_scoring(X=BIG_X))
    assert (S[F] <= Si[F]).all()
    # swapping query and target (transposed matrix) keeps the score
    sw = oracle.extend(b, a, sc)
    assert sw[0] == d[0]
    assert sw[3] == d[3]


@pytest.mark.parametrize("seed", range(20))
def test_traceback_rescoring(seed):
    rng = np.random.default_rng([8, seed])
    a, b = _random_pair(rng, related=True, L=(1, 60))
    sc = oracle.dna_scoring(2, -3, -2, int(rng.integers(0, 20)))
    (best, x, y, _), S, F = oracle.extend_matrix(a, b, sc)
    path = oracle.traceback(S, F, a, b, sc, x, y)
    assert path[0] == (0, 0) and path[-1] == (x, y)
    score = 0
    for (x0, y0), (x1, y1) in zip(path, path[1:]):
        assert F[x1, y1]
        if x1 == x0 + 1 and y1 == y0 + 1:
            score += int(sc.matrix[a[x0], b[y0]])
        else:
            score += sc.gap
    assert score == best


@pytest.mark.parametrize("seed", range(15))
def test_left_is_right_of_reversed(seed):
    rng = np.random.default_rng([9, seed])
    q, t = _random_pair(rng, related=True, L=(20, 80))
    k = 5
    qp = int(rng.integers(0, len(q) - k + 1))
    tp = min(qp, len(t) - k)
    sc = oracle.dna_scoring(X=int(rng.integers(1, 12)))
    r = oracle.seed_extend(q, t, qp, tp, k, sc)
    # the left extension equals a right extension (seed of length 0 at 0)
    # over the reversed prefixes
    rl = oracle.seed_extend(q[:qp][::-1], t[:tp][::-1], 0, 0, 0, sc)
    assert r["left"] == rl["right"]
    assert qp - r["q_begin"] == rl["q_end"]
    assert tp - r["t_begin"] == rl["t_end"]
    assert r["score"] == r["left"] + r["seed_score"] + r["right"]
    assert r["score"] >= r["seed_score"]


@pytest.mark.parametrize("seed", range(10))
def test_appending_after_termination_changes_nothing(seed):
    rng = np.random.default_rng([10, seed])
    a = rng.integers(0, 4, 200).astype(np.uint8)
    b = rng.integers(0, 4, 200).astype(np.uint8)   # unrelated: stops early
    sc = oracle.dna_scoring(1, -3, -3, 3)
    w = oracle.band_widths(a, b, sc)
    dead = np.nonzero(w == 0)[0]
    assert len(dead), "expected an early stop"
    stop = int(dead[0])
    # cut both sequences right after the last antidiagonal reached, then
    # append other symbols: the result must not change
    base = oracle.extend(a, b, sc)
    a2 = np.concatenate([a[:stop], rng.integers(0, 4, 50).astype(np.uint8)])
    b2 = np.concatenate([b[:stop], rng.integers(0, 4, 50).astype(np.uint8)])
    assert oracle.extend(a2, b2, sc) == base


def test_band_grows_with_x():
    # Sec. 6.1: a larger X keeps a wider working band
    rng = np.random.default_rng(11)
    a = rng.integers(0, 4, 600).astype(np.uint8)
    b = a.copy()
    mut = rng.random(600) < 0.15
    b[mut] = (b[mut] + rng.integers(1, 4, mut.sum())) % 4
    ws = [int(oracle.band_widths(a, b, oracle.dna_scoring(X=X)).max())
          for X in (5, 15, 50)]
    assert ws[0] <= ws[1] <= ws[2]


def test_seed_errors():
    sc = oracle.dna_scoring()
    r = oracle.seed_extend(enc("ACGT"), enc("ACGT"), 2, 0, 3, sc)
    assert r["status"] == oracle.E_RANGE
    bad = np.array([0, 1, 7], dtype=np.uint8)
    r = oracle.seed_extend(bad, enc("ACG"), 0, 0, 1, sc)
    assert r["status"] == oracle.E_SYMBOL


def test_batch_matches_single_calls():
    rng = np.random.default_rng(12)
    seqs, offs = [], [0]
    for _ in range(12):
        s = rng.integers(0, 4, int(rng.integers(10, 80))).astype(np.uint8)
        seqs.append(s)
        offs.append(offs[-1] + len(s))
    codes = np.concatenate(seqs)
    seeds = np.zeros(6, dtype=oracle.SEED_DTYPE)
    for i in range(6):
        q, t = 2 * i, 2 * i + 1
        k = 4
        seeds[i] = (q, t, int(rng.integers(0, len(seqs[q]) - k)),
                    int(rng.integers(0, len(seqs[t]) - k)), k)
    sc = oracle.dna_scoring(X=7)
    out, used = oracle.batch(codes, np.array(offs), seeds, sc, threads=2)
    assert used >= 1
    for i, s in enumerate(seeds):
        r = oracle.seed_extend(seqs[s["q"]], seqs[s["t"]], int(s["q_pos"]),
                               int(s["t_pos"]), int(s["k"]), sc)
        for f in oracle.RESULT_DTYPE.names:
            assert out[i][f] == r[f]
