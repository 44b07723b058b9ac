"""The batched workload's inputs: trivalency thresholds and the per-query recipe (CPU only)."""
from fractions import Fraction

import numpy as np

import synth


def test_trivalency_thresholds_are_the_floor_of_p_times_2_32_minus_1():
    # t = floor(p * 2^32) - 1, so an edge is live for exactly t + 1 of the 2^32 coin words:
    # (t + 1) / 2^32 <= p < (t + 2) / 2^32 for the binary value of p
    got = [synth.threshold_of(p) for p in synth.TRIVALENCY_P]
    assert got == [429_496_728, 42_949_671, 4_294_966]
    for p, t in zip(synth.TRIVALENCY_P, got):
        assert Fraction(t + 1, 2**32) <= Fraction(p) < Fraction(t + 2, 2**32)
    assert synth.threshold_of(1.0) == 0xFFFFFFFF
    assert synth.threshold_of(0.5) == 0x7FFFFFFF


def test_batch_queries_follow_the_recipe():
    qs = synth.batch_queries(64)
    assert qs == synth.batch_queries(64)  # seeded
    assert len(qs) == 64
    for j, q in enumerate(qs):
        assert 10_000 <= q["n"] <= 2_000_000
        assert 4 * q["n"] - 1 <= q["m"] <= 40 * q["n"] + 1
        assert 1 <= q["k"] <= 50 and q["eps"] in (0.1, 0.2, 0.5) and q["ell"] == 1.0
        assert q["model"] == j % 2 and q["seed"] == q["graph_seed"] == 1000 + j
        assert (q["thr_seed"] is None) == (q["model"] == 1)
    assert sum(q["model"] == 0 for q in qs) == 32
    # the draws spread over their ranges
    ns = np.array([q["n"] for q in qs], dtype=float)
    assert ns.min() < 30_000 and ns.max() > 1_000_000
    assert len({q["eps"] for q in qs}) == 3


def test_batch_graph_thresholds_and_csr():
    qs = synth.batch_queries(4, base_seed=77, n_range=(1_000, 3_000))
    for q in qs:
        g, thr = synth.batch_graph(q)
        g2, thr2 = synth.batch_graph(q)
        assert np.array_equal(g.off, g2.off) and np.array_equal(g.src, g2.src)
        assert g.n == q["n"] and g.m == q["m"] and g.off[0] == 0 and g.off[-1] == g.m
        dst = np.repeat(np.arange(g.n), np.diff(g.off))
        assert not np.any(g.src == dst)
        if q["model"] == 0:
            assert thr.dtype == np.uint32 and len(thr) == g.m and np.array_equal(thr, thr2)
            assert set(np.unique(thr).tolist()) == {429_496_728, 42_949_671, 4_294_966}
        else:
            assert thr is None


def test_serve_queries_follow_the_recipe():
    qs = synth.serve_queries(2000, 50.0, 7)
    assert qs == synth.serve_queries(2000, 50.0, 7)
    t = np.array([q["arrival"] for q in qs])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 50.0) < 0.003  # Poisson arrivals at 50 per second
    assert {q["graph"] for q in qs} == {0, 1, 2, 3} and {q["model"] for q in qs} == {0, 1}
    assert min(q["k"] for q in qs) >= 1 and max(q["k"] for q in qs) <= 100
    assert {q["eps"] for q in qs} == {0.1, 0.2, 0.3}
    assert len({q["seed"] for q in qs}) == len(qs)


def test_serve_graph_sizes():
    gs = synth.serve_graphs(scale=0.01)
    assert [g.n for g in gs] == [1000, 10000, 40000, 100000]
    assert all(g.m == 16 * g.n for g in gs)
