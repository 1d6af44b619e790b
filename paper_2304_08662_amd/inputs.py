"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws sequences and seeds and packs them; it holds none of
the alignment arithmetic.  It feeds both the CPU oracle (one code per byte)
and the GPU library (2-bit packed DNA or one byte per protein residue).

Workloads (sizes and mixes follow the paper's Sec. 5.3 and Table 2: long reads
of 1-30 kb, 15% error synthetic reads with the seed window kept free of
edits, 17-mer seeds for DNA and 6-mers for protein, X in {15, 49, 50}):

* ``dna_pairs``      query uniform ACGT, target = query with edits (sub / ins /
                     del with equal odds, a substitution picks another symbol,
                     an insertion puts a random symbol before the position),
                     or an unrelated target with the seed k-mer copied in.
* ``protein_pairs``  20 codes, uniform background, 30% substitution and 5%
                     indel for related pairs, 50% unrelated.
* ``workload(name)`` the named configurations (see ``WORKLOADS``).

RNG: ``numpy.random.Generator(PCG64(SeedSequence([0, config_id])))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_DTYPE = np.dtype([("q", "<i4"), ("t", "<i4"), ("q_pos", "<i4"),
                       ("t_pos", "<i4"), ("k", "<i4")])

DNA_CODES = "ACGT"


def rng_for(config_id: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([0, config_id, sub] if sub else [0, config_id])))


@dataclass
class Batch:
    """Sequences (codes, one per byte, concatenated), offsets (n_seqs+1) and
    seed records.  ``alphabet`` is 4 (DNA) or 20 (protein)."""
    codes: np.ndarray
    offsets: np.ndarray
    seeds: np.ndarray
    alphabet: int
    meta: dict = field(default_factory=dict)

    @property
    def n_seqs(self) -> int:
        return len(self.offsets) - 1

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def gcups_cells(self) -> int:
        """Paper's GCUPS numerator: sum over seeds of |q| * |t| (Sec. 5.1)."""
        L = self.lengths()
        return int(np.sum(L[self.seeds["q"]].astype(np.int64) *
                          L[self.seeds["t"]].astype(np.int64)))

    def packed(self) -> np.ndarray:
        """Sequence bytes as handed to the GPU library: 2-bit DNA (16 codes per
        32-bit word, code i at bits 2*(i%16)) or one byte per code."""
        if self.alphabet == 4:
            return pack_dna2(self.codes)
        return np.ascontiguousarray(self.codes, dtype=np.uint8)

    def subset(self, idx) -> "Batch":
        """Seeds idx with only the sequences they reference."""
        sd = self.seeds[np.asarray(idx)]
        used = np.unique(np.concatenate([sd["q"], sd["t"]]))
        remap = np.full(self.n_seqs, -1, dtype=np.int64)
        remap[used] = np.arange(len(used))
        L = self.lengths()[used]
        offs = np.zeros(len(used) + 1, dtype=np.int64)
        np.cumsum(L, out=offs[1:])
        parts = [self.codes[self.offsets[s]:self.offsets[s + 1]] for s in used]
        codes = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        nsd = sd.copy()
        nsd["q"] = remap[sd["q"]]
        nsd["t"] = remap[sd["t"]]
        return Batch(codes, offs, nsd, self.alphabet, dict(self.meta))


def pack_dna2(codes: np.ndarray) -> np.ndarray:
    """Pack DNA codes 0..3 into 2 bits each, little-endian within 32-bit words;
    returned as bytes (length a multiple of 4)."""
    c = np.asarray(codes, dtype=np.uint8)
    n = len(c)
    nw = (n + 15) // 16
    pad = np.zeros(nw * 16, dtype=np.uint32)
    pad[:n] = c & 3
    pad = pad.reshape(nw, 16)
    shifts = (2 * np.arange(16, dtype=np.uint32))[None, :]
    words = np.bitwise_or.reduce(pad << shifts, axis=1).astype(np.uint32)
    if nw == 0:
        words = np.zeros(1, dtype=np.uint32)
    return words.view(np.uint8)


def mutate(rng, q: np.ndarray, rate_sub: float, rate_ins: float,
           rate_del: float, alphabet: int, protect=(0, 0)):
    """Apply per-position edits outside the protected window [p0, p1).
    Returns (t, image) where image[i] is the index in t of q[i] (for the
    seed's position in the target)."""
    L = len(q)
    u = rng.random(L)
    kind = np.zeros(L, dtype=np.int8)          # 0 keep, 1 sub, 2 ins, 3 del
    kind[u < rate_sub] = 1
    kind[(u >= rate_sub) & (u < rate_sub + rate_ins)] = 2
    kind[(u >= rate_sub + rate_ins) & (u < rate_sub + rate_ins + rate_del)] = 3
    kind[protect[0]:protect[1]] = 0
    out_sym = q.copy()
    subs = kind == 1
    out_sym[subs] = (q[subs] + rng.integers(1, alphabet, subs.sum())) % alphabet
    # each position emits: ins -> [random, q], del -> [], else [sym]
    emit = np.where(kind == 3, 0, np.where(kind == 2, 2, 1))
    start = np.zeros(L + 1, dtype=np.int64)
    np.cumsum(emit, out=start[1:])
    t = np.empty(start[-1], dtype=np.uint8)
    ins = kind == 2
    single = emit == 1
    t[start[:-1][single]] = out_sym[single]
    t[start[:-1][ins]] = rng.integers(0, alphabet, ins.sum())
    t[start[:-1][ins] + 1] = q[ins]
    image = start[:-1] + (emit == 2)          # q[i] lands after the insert
    return t, image


def _assemble(pairs, alphabet, meta):
    seqs, seeds = [], []
    for i, (q, t, qp, tp, k) in enumerate(pairs):
        seqs.append(q)
        seqs.append(t)
        seeds.append((2 * i, 2 * i + 1, qp, tp, k))
    L = np.array([len(s) for s in seqs], dtype=np.int64)
    offs = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(L, out=offs[1:])
    codes = np.concatenate(seqs) if seqs else np.zeros(0, np.uint8)
    sd = np.array(seeds, dtype=SEED_DTYPE) if seeds else np.zeros(0, SEED_DTYPE)
    return Batch(codes.astype(np.uint8), offs, sd, alphabet, meta)


def related_pair(rng, q, k, edit, alphabet, seed_pos=None, sub=None,
                 indel=None):
    """Target = edited query with the k-mer at seed_pos protected."""
    L = len(q)
    qp = int(rng.integers(0, L - k + 1)) if seed_pos is None else int(seed_pos)
    if sub is None:
        rs = ri = rd = edit / 3.0
    else:
        rs, ri, rd = sub, indel / 2.0, indel / 2.0
    t, image = mutate(rng, q, rs, ri, rd, alphabet, protect=(qp, qp + k))
    return t, qp, int(image[qp])


def unrelated_pair(rng, q, t, k):
    """Independent target with the query's k-mer copied over a random spot."""
    qp = int(rng.integers(0, len(q) - k + 1))
    tp = int(rng.integers(0, len(t) - k + 1))
    t = t.copy()
    t[tp:tp + k] = q[qp:qp + k]
    return t, qp, tp


def dna_pairs(rng, n, lengths, edit=0.15, k=17, related_frac=1.0,
              seed_at_mid=False):
    pairs = []
    rel = rng.random(n) < related_frac
    for i in range(n):
        L = int(lengths[i])
        q = rng.integers(0, 4, L).astype(np.uint8)
        if rel[i]:
            mid = L // 2 - k // 2 if seed_at_mid else None
            t, qp, tp = related_pair(rng, q, k, edit, 4, seed_pos=mid)
        else:
            Lt = int(lengths[(i + 1) % n]) if n > 1 else L
            t0 = rng.integers(0, 4, max(Lt, k)).astype(np.uint8)
            t, qp, tp = unrelated_pair(rng, q, t0, k)
        pairs.append((q, t, qp, tp, k))
    return pairs


def protein_pairs(rng, n, lengths, k=6, related_frac=0.5):
    pairs = []
    rel = rng.random(n) < related_frac
    for i in range(n):
        L = int(lengths[i])
        q = rng.integers(0, 20, L).astype(np.uint8)
        if rel[i]:
            t, qp, tp = related_pair(rng, q, k, 0.0, 20, sub=0.30, indel=0.05)
        else:
            Lt = int(rng.integers(50, 1001))
            t0 = rng.integers(0, 20, max(Lt, k)).astype(np.uint8)
            t, qp, tp = unrelated_pair(rng, q, t0, k)
        pairs.append((q, t, qp, tp, k))
    return pairs


def stand_in_substitution_matrix() -> np.ndarray:
    """A fixed, symmetric 20 x 20 integer matrix in the range of published
    protein substitution tables (diagonal 4..11, off-diagonal -4..3, mostly
    negative).  Stand-in for BLOSUM62, which is not available here; drawn from
    a fixed seed so it is reproducible.  The GPU path takes any matrix."""
    rng = rng_for(62)
    M = rng.choice(np.arange(-4, 4), size=(20, 20),
                   p=[0.06, 0.18, 0.26, 0.22, 0.14, 0.08, 0.04, 0.02])
    M = np.triu(M, 1)
    M = M + M.T
    np.fill_diagonal(M, rng.integers(4, 12, 20))
    return M.astype(np.int32)


# ------------------------------------------------------------------ workloads
@dataclass
class Scheme:
    """Scoring parameters of a workload (plain numbers, no arithmetic)."""
    alphabet: int
    match: int = 1
    mismatch: int = -1
    gap: int = -1
    X: int = 15
    matrix: np.ndarray | None = None

    def full_matrix(self) -> np.ndarray:
        if self.matrix is not None:
            return np.asarray(self.matrix, dtype=np.int32)
        M = np.full((self.alphabet, self.alphabet), self.mismatch, np.int32)
        np.fill_diagonal(M, self.match)
        return M


def workload_dna_1k(scale: float = 1.0, config_id: int = 1) -> tuple:
    """1,000 DNA pairs, |q| ~ U{1000..2000}, 15% edits, 17-mer seed at the
    query midpoint, +1/-1/-1, X = 15."""
    rng = rng_for(config_id)
    n = max(1, int(round(1000 * scale)))
    L = rng.integers(1000, 2001, n)
    b = _assemble(dna_pairs(rng, n, L, 0.15, 17, 1.0, seed_at_mid=True), 4,
                  {"workload": "dna-1k"})
    return b, Scheme(4, 1, -1, -1, 15)


def workload_dna_100k(scale: float = 1.0, config_id: int = 2) -> tuple:
    """100,000 DNA pairs, lengths lognormal (median 8 kb, sigma 0.5, clipped to
    1-30 kb), 70% related at 15% edits with a 17-mer seed at a random shared
    position, 30% unrelated with a forced 17-mer seed; +1/-1/-1, X = 50."""
    rng = rng_for(config_id)
    n = max(1, int(round(100000 * scale)))
    L = np.clip(np.round(np.exp(rng.normal(np.log(8000), 0.5, n))), 1000,
                30000).astype(np.int64)
    b = _assemble(dna_pairs(rng, n, L, 0.15, 17, 0.7), 4,
                  {"workload": "dna-100k"})
    return b, Scheme(4, 1, -1, -1, 50)


def workload_dna_tail(scale: float = 1.0, config_id: int = 3) -> tuple:
    """The 1k workload plus 100 pairs of 50-100 kb (10% long tail), X = 15."""
    base, _ = workload_dna_1k(scale, 1)
    rng = rng_for(config_id)
    n = max(1, int(round(100 * scale)))
    L = rng.integers(50000, 100001, n)
    tail = _assemble(dna_pairs(rng, n, L, 0.15, 17, 1.0, seed_at_mid=True), 4,
                     {})
    return concat(base, tail, {"workload": "dna-tail"}), Scheme(4, 1, -1, -1, 15)


def workload_protein(scale: float = 1.0, config_id: int = 4) -> tuple:
    """500,000 protein pairs, 20 codes uniform, |q| ~ U{50..1000}, 50% related
    (30% substitution + 5% indel), 6-mer seed, stand-in matrix, gap -2, X = 49."""
    rng = rng_for(config_id)
    n = max(1, int(round(500000 * scale)))
    L = rng.integers(50, 1001, n)
    b = _assemble(protein_pairs(rng, n, L, 6, 0.5), 20,
                  {"workload": "protein-500k"})
    return b, Scheme(20, gap=-2, X=49, matrix=stand_in_substitution_matrix())


WORKLOADS = {
    "dna-1k": workload_dna_1k,
    "dna-100k": workload_dna_100k,
    "dna-tail": workload_dna_tail,
    "protein-500k": workload_protein,
}


def workload(name: str, scale: float = 1.0):
    return WORKLOADS[name](scale)


def concat(a: Batch, b: Batch, meta=None) -> Batch:
    offs = np.concatenate([a.offsets, a.offsets[-1] + b.offsets[1:]])
    sd = b.seeds.copy()
    sd["q"] += a.n_seqs
    sd["t"] += a.n_seqs
    return Batch(np.concatenate([a.codes, b.codes]), offs,
                 np.concatenate([a.seeds, sd]), a.alphabet,
                 meta if meta is not None else dict(a.meta))


def request_pools(rng, pool_pairs=8192):
    """The two pools the pooled request stream draws from: DNA pairs of the
    1k generator and protein pairs of the protein generator.  Returns
    [(pool Batch, Scheme), (pool Batch, Scheme)]."""
    dna_scheme = Scheme(4, 1, -1, -1, 15)
    prot_scheme = Scheme(20, gap=-2, X=49,
                         matrix=stand_in_substitution_matrix())
    L = rng.integers(1000, 2001, pool_pairs)
    dna_pool = _assemble(dna_pairs(rng, pool_pairs, L, 0.15, 17, 1.0, True),
                         4, {"pool": "dna"})
    L = rng.integers(50, 1001, pool_pairs)
    prot_pool = _assemble(protein_pairs(rng, pool_pairs, L, 6, 0.5), 20,
                          {"pool": "protein"})
    return [(dna_pool, dna_scheme), (prot_pool, prot_scheme)]


def request_refs(rng, n_requests: int, mean_gap_s: float, pool_pairs: int,
                 max_pairs=4096):
    """Arrival times and pair selections of the pooled request stream: each
    request takes a contiguous run of pairs (cyclic) at a random start in
    pool 0 (DNA) or 1 (protein) with probability 1/2; sizes follow the
    request-size law.  Yields (arrival_time_s, pool index, pair indices)."""
    t = 0.0
    for _ in range(n_requests):
        t += float(rng.exponential(mean_gap_s))
        size = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(max_pairs + 1)))),
                           1, max_pairs))
        which = 0 if rng.random() < 0.5 else 1
        start = int(rng.integers(0, pool_pairs))
        yield t, which, (start + np.arange(size)) % pool_pairs


def request_stream_pooled(rng, n_requests: int, mean_gap_s: float,
                          max_pairs=4096, pool_pairs=8192):
    """As request_stream, but each request takes a contiguous run of pairs
    (cyclic) at a random start from one of two pools generated once
    (request_pools).  Request sizes, arrivals and the DNA/protein mix follow
    the same laws; the pools make long streams cheap to generate (pairs
    repeat across requests).  Yields (arrival_time_s, Batch, Scheme), the
    Batch holding its own copy of the pairs' sequences."""
    pools = request_pools(rng, pool_pairs)
    for r, (t, which, idx) in enumerate(
            request_refs(rng, n_requests, mean_gap_s, pool_pairs, max_pairs)):
        pool, scheme = pools[which]
        b = pool.subset(idx)
        b.meta = {"request": r}
        yield t, b, scheme


def request_stream(rng, n_requests: int, mean_gap_s: float, max_pairs=4096):
    """Serving workload: Poisson arrivals; each request holds
    floor(exp(U(ln 1, ln 4097))) pairs (clipped to [1, 4096]), DNA (1k
    generator) or protein (protein generator) with probability 1/2.
    Yields (arrival_time_s, Batch, Scheme)."""
    t = 0.0
    dna_scheme = Scheme(4, 1, -1, -1, 15)
    prot_scheme = Scheme(20, gap=-2, X=49,
                         matrix=stand_in_substitution_matrix())
    for r in range(n_requests):
        t += float(rng.exponential(mean_gap_s))
        size = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(max_pairs + 1)))),
                           1, max_pairs))
        if rng.random() < 0.5:
            L = rng.integers(1000, 2001, size)
            b = _assemble(dna_pairs(rng, size, L, 0.15, 17, 1.0, True), 4,
                          {"request": r})
            yield t, b, dna_scheme
        else:
            L = rng.integers(50, 1001, size)
            b = _assemble(protein_pairs(rng, size, L, 6, 0.5), 20,
                          {"request": r})
            yield t, b, prot_scheme
