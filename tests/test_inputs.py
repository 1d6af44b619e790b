"""CPU checks of the seeded input generators (shapes and laws of the
synthetic workloads; no alignment arithmetic lives in the generator)."""
import numpy as np

from paper_2304_08662_amd import inputs


def test_dna_1k_shape():
    b, s = inputs.workload("dna-1k", 0.05)
    L = b.lengths()
    assert len(b.seeds) == 50 and s.X == 15
    q = L[b.seeds["q"]]
    assert q.min() >= 1000 and q.max() <= 2000
    # the 17-mer seed sits at the query midpoint and matches exactly
    for sd in b.seeds:
        qa = b.codes[b.offsets[sd["q"]]:b.offsets[sd["q"] + 1]]
        ta = b.codes[b.offsets[sd["t"]]:b.offsets[sd["t"] + 1]]
        assert sd["k"] == 17 and sd["q_pos"] == len(qa) // 2 - 8
        assert np.array_equal(qa[sd["q_pos"]:sd["q_pos"] + 17],
                              ta[sd["t_pos"]:sd["t_pos"] + 17])


def test_generators_are_seeded():
    a, _ = inputs.workload("protein-500k", 0.0005)
    b, _ = inputs.workload("protein-500k", 0.0005)
    assert np.array_equal(a.codes, b.codes)
    assert np.array_equal(a.seeds, b.seeds)


def test_pooled_request_stream_laws():
    rng = inputs.rng_for(5)
    reqs = list(inputs.request_stream_pooled(rng, 300, 0.001, pool_pairs=512))
    sizes = np.array([len(b.seeds) for _, b, _ in reqs])
    assert sizes.min() >= 1 and sizes.max() <= 4096
    # log-uniform sizes: median near sqrt(4097) ~ 64
    assert 20 < np.median(sizes) < 200
    kinds = np.array([b.alphabet for _, b, _ in reqs])
    assert 0.35 < np.mean(kinds == 4) < 0.65
    times = np.array([t for t, _, _ in reqs])
    assert np.all(np.diff(times) >= 0)
    for _, b, s in reqs[:20]:
        # every seed references sequences of its own request
        assert b.seeds["q"].max() < b.n_seqs and b.seeds["t"].max() < b.n_seqs
        assert (s.alphabet == 4) == (b.alphabet == 4)
