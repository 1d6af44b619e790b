"""Shared helpers of the GPU tests: run a batch through the C ABI and through
the oracle and compare.  (Test code: the only place that touches both.)"""
import numpy as np

import oracle
from paper_2304_08662_amd import inputs

FIELDS = ("score", "left", "right", "seed_score", "q_begin", "q_end",
          "t_begin", "t_end", "cells", "status")


def product_scoring(scheme):
    from paper_2304_08662_amd import xdrop
    if scheme.alphabet == 4 and scheme.matrix is None:
        return xdrop.ScoringSpec(xdrop.DNA2, 4, scheme.match, scheme.mismatch,
                                 scheme.gap, int(min(scheme.X, 2**31 - 1)))
    return xdrop.ScoringSpec(xdrop.BYTE, scheme.alphabet, 0, 0, scheme.gap,
                             int(min(scheme.X, 2**31 - 1)),
                             matrix=scheme.full_matrix())


def oracle_scoring(scheme):
    return oracle.Scoring(scheme.full_matrix(), scheme.gap, scheme.X)


class Runner:
    """Keeps one library context and one stream for a test session."""

    def __init__(self):
        import torch
        from paper_2304_08662_amd import xdrop
        self.torch = torch
        self.xdrop = xdrop
        self.ctx = xdrop.Context(0)
        self.stream = torch.cuda.Stream()

    def upload(self, batch):
        packed = batch.packed() if batch.alphabet == 4 else \
            np.ascontiguousarray(batch.codes, dtype=np.uint8)
        return self.xdrop.to_device(packed, batch.offsets, batch.seeds)

    def run(self, batch, scheme, opts=None, graph=False, dev=None,
            alphabet=None, noalloc=False):
        torch, xdrop = self.torch, self.xdrop
        sc = product_scoring(scheme)
        if alphabet is not None:
            sc.alphabet = alphabet
        d_seqs, d_offs, d_seeds = dev if dev is not None else self.upload(batch)
        n = len(batch.seeds)
        res = xdrop.result_buffer(n)
        res.fill_(-12345)
        # the library runs on self.stream: order it after the uploads and the
        # fill made on the current stream
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            self.ctx.extend_batch(d_seqs, d_offs, d_seeds, sc, res, opts,
                                  stream=self.stream, graph=graph,
                                  noalloc=noalloc)
        self.stream.synchronize()
        return xdrop.results_to_numpy(res, n)


def oracle_run(batch, scheme, threads=0):
    out, _ = oracle.batch(batch.codes, batch.offsets, batch.seeds,
                          oracle_scoring(scheme), threads=threads)
    return out


def compare(gpu, ref, idx=None):
    """Element-by-element equality of every result field; returns a list of
    mismatch descriptions (empty when bit-exact)."""
    bad = []
    rows = range(len(ref)) if idx is None else idx
    for k, i in enumerate(rows):
        g = gpu[k] if idx is not None else gpu[i]
        r = ref[k] if idx is not None else ref[i]
        for f in FIELDS:
            if int(g[f]) != int(r[f]):
                bad.append((i, f, int(g[f]), int(r[f])))
    return bad


def make_batch(pairs, alphabet, meta=None):
    return inputs._assemble(pairs, alphabet, meta or {})


def shared_sequence_batches(rng, n_seqs=24, n_seeds=160, alphabet=4):
    """Seeds that share sequences: n_seqs sequences (half of them edited
    copies of the other half), n_seeds seeds drawn over them, several seeds
    on one pair at different positions and one sequence against several
    others.  Returns (shared batch, unique-copy batch with one fresh copy of
    both sequences per seed)."""
    from paper_2304_08662_amd import inputs
    half = n_seqs // 2
    seqs = [rng.integers(0, alphabet, int(rng.integers(150, 1200))).astype(np.uint8)
            for _ in range(half)]
    seqs += [inputs.mutate(rng, s, 0.05, 0.03, 0.03, alphabet)[0] for s in seqs]
    L = np.array([len(s) for s in seqs])
    offs = np.zeros(n_seqs + 1, dtype=np.int64)
    np.cumsum(L, out=offs[1:])
    codes = np.concatenate(seqs).astype(np.uint8)
    sd = np.zeros(n_seeds, dtype=inputs.SEED_DTYPE)
    q = rng.integers(0, n_seqs, n_seeds)
    t = np.where(rng.random(n_seeds) < 0.6, (q + half) % n_seqs,
                 rng.integers(0, n_seqs, n_seeds))
    k = np.minimum(np.minimum(L[q], L[t]), rng.integers(0, 18, n_seeds))
    sd["q"], sd["t"], sd["k"] = q, t, k
    sd["q_pos"] = (rng.random(n_seeds) * (L[q] - k + 1)).astype(np.int64)
    sd["t_pos"] = (rng.random(n_seeds) * (L[t] - k + 1)).astype(np.int64)
    shared = inputs.Batch(codes, offs, sd, alphabet)
    unique = make_batch([(seqs[a], seqs[b], int(x), int(y), int(z))
                         for a, b, x, y, z in zip(q, t, sd["q_pos"],
                                                  sd["t_pos"], k)], alphabet)
    return shared, unique
