"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here runs on the GPU.  Each test checks the oracle against something
other than itself: published known-answer vectors, closed forms, exhaustive
enumeration of live-edge worlds (brute.c), textbook graph algorithms written
here in numpy, or the worked example printed in the paper.
"""
import math
import os
from fractions import Fraction
from itertools import combinations, product

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
IC, LT, TRIG = oracle.IC, oracle.LT, oracle.TRIGGER


def _read_kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


# ---------------------------------------------------------------- Philox --
def test_philox_known_answers():
    rows = _read_kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(oracle.philox(ctr, key)) == out


def test_philox_bits_balanced():
    # Each of the 128 output bits is set about half the time over 4096 counters.
    words = np.array([oracle.draw(12345, 64, 1, i, 7) for i in range(4096)], dtype=np.uint64)
    bits = np.stack([(words >> np.uint64(b)) & np.uint64(1) for b in range(32)], axis=-1).reshape(4096, 128)
    frac = bits.mean(axis=0)
    sigma = 0.5 / math.sqrt(4096)
    assert np.all(np.abs(frac - 0.5) < 5 * sigma)


def test_stream_layout_separates_phases_kinds_sets():
    a = oracle.draw(1, 5, 1, 10, 3)
    assert a != oracle.draw(1, 6, 1, 10, 3)
    assert a != oracle.draw(1, 5, 2, 10, 3)
    assert a != oracle.draw(1, 5, 1, 11, 3)
    assert a != oracle.draw(1, 5, 1, 10, 4)
    assert a != oracle.draw(2, 5, 1, 10, 3)
    # the documented counter layout: (idx lo, phase<<24|kind<<16|idx hi, set lo, set hi)
    idx, setid, seed = (0x1234 << 32) | 0x89ABCDEF, (7 << 32) | 9, (3 << 32) | 11
    ctr = [0x89ABCDEF, (5 << 24) | (1 << 16) | 0x1234, 9, 7]
    assert oracle.draw(seed, 5, 1, idx, setid) == oracle.philox(ctr, [11, 3])


# ------------------------------------------------------------ thresholds --
@pytest.mark.parametrize("d", [1, 2, 3, 5, 7, 10, 1000, 65537, 160819, 2**31 - 1])
def test_wc_threshold_counts_exactly_floor_p_2_32(d):
    t = oracle.wc_threshold(d)
    # words x in [0, 2^32) with x <= t: exactly t + 1 of them, which must be floor(2^32 / d)
    assert t + 1 == (2**32) // d
    assert (t + 1) * d <= 2**32 < (t + 2) * d


def test_wc_threshold_special_values():
    assert oracle.wc_threshold(1) == 0xFFFFFFFF  # p = 1 is representable
    assert oracle.wc_threshold(2) == 2147483647


# ------------------------------------------------------------------ root --
def test_root_uniform():
    n, N = 7, 70000
    counts = np.bincount([oracle.root(99, 64, s, n) for s in range(N)], minlength=n)
    chi2 = ((counts - N / n) ** 2 / (N / n)).sum()
    assert chi2 < 30.0  # 6 degrees of freedom; p ~ 4e-5
    big = 2**31 - 1
    assert all(0 <= oracle.root(5, 1, s, big) < big for s in range(1000))


def test_lt_pick_uniform():
    d, N = 5, 50000
    counts = np.bincount([oracle.lt_pick(3, 64, s, 17, d) for s in range(N)], minlength=d)
    chi2 = ((counts - N / d) ** 2 / (N / d)).sum()
    assert chi2 < 25.0


def _cumulative(weights):
    """uint32 cumulative thresholds t_j = floor(C_j * 2^32) - 1 of exact rational weights."""
    c, out = Fraction(0), []
    for w in weights:
        c += Fraction(w)
        out.append(int(c * 2**32) - 1)
    return np.array(out, dtype=np.uint32)


def test_lt_pick_cumulative_follows_the_weights():
    # weights 1/10, 1/5, 3/10, 1/5: the walk stops at v with probability 1/5
    w = [Fraction(1, 10), Fraction(1, 5), Fraction(3, 10), Fraction(1, 5)]
    t = _cumulative(w)
    N = 60000
    picks = np.array([oracle.lt_pick_cumulative(9, 64, s, 33, t) for s in range(N)])
    counts = np.array([(picks == j).sum() for j in range(4)] + [(picks == -1).sum()])
    p = np.array([float(x) for x in w] + [0.2])
    chi2 = ((counts - N * p) ** 2 / (N * p)).sum()
    assert chi2 < 30.0  # 4 degrees of freedom


def test_lt_pick_cumulative_boundaries():
    # the pick compares word 0 of the node's pick draw with each threshold, inclusively
    for s in range(20):
        x = oracle.draw(4, 64, 2, 12, s)[0]
        if 2 <= x <= 0xFFFFFFFD:
            assert oracle.lt_pick_cumulative(4, 64, s, 12, [x - 1, x, 0xFFFFFFFF]) == 1
            assert oracle.lt_pick_cumulative(4, 64, s, 12, [x, x, x]) == 0
            assert oracle.lt_pick_cumulative(4, 64, s, 12, [x - 2, x - 1]) == -1
        assert oracle.lt_pick_cumulative(4, 64, s, 12, [0xFFFFFFFF]) == 0


def test_lt_first_in_edge_when_it_holds_all_the_weight():
    # thresholds all 2^32 - 1: every node takes its first in-edge, so the set is the chain of first in-edges
    g = synth.chung_lu(300, 1500, 2.1, 5)
    t = np.full(g.m, 0xFFFFFFFF, dtype=np.uint32)
    for s in range(200):
        root = oracle.root(6, 64, s, g.n)
        chain, v = [root], root
        while g.off[v + 1] > g.off[v] and int(g.src[g.off[v]]) not in chain:
            v = int(g.src[g.off[v]])
            chain.append(v)
        nodes, w = oracle.rr_set(g, LT, 6, 64, s, thr=t)
        assert list(nodes) == sorted(chain)
        assert w == sum(int(g.off[u + 1] - g.off[u]) for u in chain)


def test_lt_sets_are_single_roots_when_weights_vanish():
    # cumulative thresholds 0: an in-edge is taken with probability 2^-32, so the walk stops at the root
    g = synth.chung_lu(300, 1500, 2.1, 5)
    t = np.zeros(g.m, dtype=np.uint32)
    so, nodes, widths = oracle.sample_sets(g, LT, 6, 64, 0, 2000, thr=t)
    assert np.all(np.diff(so) == 1)
    assert np.array_equal(widths, np.diff(g.off)[nodes].astype(np.uint64))


# ---------------------------------------------------- RR set = ancestors --
def _ancestors(n, live_edges, root):
    """Nodes that reach `root` along live edges: fixed-point iteration."""
    inr = np.zeros(n, dtype=bool)
    inr[root] = True
    changed = True
    while changed:
        changed = False
        for u, v in live_edges:
            if inr[v] and not inr[u]:
                inr[u] = True
                changed = True
    return np.flatnonzero(inr)


def _live_world(g, model, seed, phase, s, thr):
    el = synth.edge_list(g)
    live = []
    if model == IC:
        indeg = g.indeg()
        for e, (u, v) in enumerate(el):
            t = thr[e] if thr is not None else (2**32 // indeg[v]) - 1
            if oracle.coin_word(seed, phase, s, e) <= t:
                live.append((u, v))
    elif model == TRIG:
        for v in range(g.n):
            j = oracle.trig_pick(seed, phase, s, v, thr)
            if j >= 0:
                for i in range(int(thr.tset[j]), int(thr.tset[j + 1])):
                    live.append((int(g.src[g.off[v] + int(thr.tmem[i])]), v))
    else:
        for v in range(g.n):
            d = g.off[v + 1] - g.off[v]
            if d:
                if thr is None:
                    j = oracle.lt_pick(seed, phase, s, v, d)
                else:
                    j = oracle.lt_pick_cumulative(seed, phase, s, v, thr[g.off[v]:g.off[v + 1]])
                if j >= 0:
                    live.append((int(g.src[g.off[v] + j]), v))
    return live


@pytest.mark.parametrize("model", [IC, LT, "LT-weighted", TRIG])
@pytest.mark.parametrize("gseed", [1, 2, 3])
def test_rr_set_is_reverse_reachable_set(model, gseed):
    g = synth.random_small_graph(9, 24, gseed)
    thr = synth.random_thresholds(g.m, gseed, choices=[0x3FFFFFFF, 0x7FFFFFFF, 0xBFFFFFFF]) if model == IC else None
    if model == "LT-weighted":
        model, thr = LT, synth.random_lt_thresholds(g, gseed, total=0.8)
    if model == TRIG:
        thr = synth.random_triggering(g, gseed)
    indeg = g.indeg()
    for s in range(60):
        nodes, w = oracle.rr_set(g, model, 77, 64, s, thr=thr)
        root = oracle.root(77, 64, s, g.n)
        want = _ancestors(g.n, _live_world(g, model, 77, 64, s, thr), root)
        assert list(nodes) == list(want)
        assert w == int(indeg[want].sum())


def test_rr_set_weighted_cascade_matches_ancestors():
    g = synth.chung_lu(300, 1500, 2.1, 11)
    indeg = g.indeg()
    for s in range(40):
        nodes, w = oracle.rr_set(g, IC, 5, 3, s)
        root = oracle.root(5, 3, s, g.n)
        want = _ancestors(g.n, _live_world(g, IC, 5, 3, s, None), root)
        assert list(nodes) == list(want)
        assert w == int(indeg[want].sum())


def test_p_one_gives_ancestors_in_g():
    g = synth.random_small_graph(12, 30, 4)
    thr = np.full(g.m, 0xFFFFFFFF, dtype=np.uint32)
    # textbook transitive closure (Warshall) of the adjacency matrix
    reach = np.eye(g.n, dtype=bool)
    for u, v in synth.edge_list(g):
        reach[u, v] = True
    for k in range(g.n):
        reach |= reach[:, k:k + 1] & reach[k:k + 1, :]
    for s in range(50):
        root = oracle.root(1, 2, s, g.n)
        nodes, w = oracle.rr_set(g, IC, 1, 2, s, thr=thr)
        assert list(nodes) == list(np.flatnonzero(reach[:, root]))


def _trigger_of(g, outcomes):
    """A triggering distribution from, per node, a list of (probability numerator over 2^32, local indices)."""
    toff, tthr, tset, tmem = [0], [], [0], []
    for v in range(g.n):
        acc = 0
        for num, members in outcomes(v, int(g.off[v + 1] - g.off[v])):
            acc += num
            tthr.append(acc - 1)
            tmem.extend(members)
            tset.append(len(tmem))
        toff.append(len(tthr))
    return synth.Triggering(np.array(toff, dtype=np.int64), np.array(tthr, dtype=np.uint32),
                            np.array(tset, dtype=np.int64), np.array(tmem, dtype=np.uint32))


def test_trigger_pick_follows_the_distribution():
    # three outcomes of probability 1/8, 3/8, 1/4 and the empty set with the remaining 1/4
    g = synth.from_edges(4, [(1, 0), (2, 0), (3, 0)])
    tr = _trigger_of(g, lambda v, d: [(2**29, [0]), (3 * 2**29, [1, 2]), (2**30, [0, 2])] if v == 0 else [])
    N = 40000
    picks = np.array([oracle.trig_pick(9, 64, s, 0, tr) for s in range(N)])
    counts = np.array([(picks == j).sum() for j in range(3)] + [(picks == -1).sum()])
    p = np.array([1 / 8, 3 / 8, 1 / 4, 1 / 4])
    chi2 = ((counts - N * p) ** 2 / (N * p)).sum()
    assert chi2 < 25.0  # 3 degrees of freedom
    # the pick compares word 0 of the kind-3 draw with each threshold, inclusively
    for s in range(30):
        x = oracle.draw(9, 64, 3, 0, s)[0]
        if 1 <= x <= 0xFFFFFFFE:
            t = _trigger_of(g, lambda v, d: [(x, [0]), (1, [1]), (0xFFFFFFFF - x, [2])] if v == 0 else [])
            assert oracle.trig_pick(9, 64, s, 0, t) == 1  # x <= t_1 = x, x > t_0 = x - 1


def test_trigger_with_every_in_edge_certain_gives_ancestors_in_g():
    # one outcome holding all in-edges with probability 1: the RR set is the set of ancestors in G
    g = synth.random_small_graph(12, 30, 6)
    tr = _trigger_of(g, lambda v, d: [(2**32, list(range(d)))] if d else [])
    reach = np.eye(g.n, dtype=bool)
    for u, v in synth.edge_list(g):
        reach[u, v] = True
    for k in range(g.n):
        reach |= reach[:, k:k + 1] & reach[k:k + 1, :]
    indeg = g.indeg()
    for s in range(40):
        root = oracle.root(3, 5, s, g.n)
        nodes, w = oracle.rr_set(g, TRIG, 3, 5, s, thr=tr)
        want = np.flatnonzero(reach[:, root])
        assert list(nodes) == list(want) and w == int(indeg[want].sum())


def test_trigger_with_single_certain_members_is_a_chain():
    # every node's triggering set is always its first in-edge: the RR set is the chain of first in-edges
    g = synth.chung_lu(300, 1500, 2.1, 5)
    tr = _trigger_of(g, lambda v, d: [(2**32, [0])] if d else [])
    for s in range(100):
        root = oracle.root(6, 64, s, g.n)
        chain, v = [root], root
        while g.off[v + 1] > g.off[v] and int(g.src[g.off[v]]) not in chain:
            v = int(g.src[g.off[v]])
            chain.append(v)
        nodes, w = oracle.rr_set(g, TRIG, 6, 64, s, thr=tr)
        assert list(nodes) == sorted(chain)


def test_lt_functional_graph_chain():
    # every node has exactly one in-neighbour: the walk is deterministic
    n = 10
    pred = [3, 0, 1, 2, 3, 4, 5, 9, 7, 8]  # 0<-3<-2<-1<-0 cycle; 4<-3, 5<-4, 6<-5; 7<-9<-8<-7 cycle
    g = synth.from_edges(n, [(pred[v], v) for v in range(n)])
    for s in range(40):
        root = oracle.root(8, 64, s, n)
        chain, v = [root], root
        while pred[v] not in chain:
            chain.append(pred[v])
            v = pred[v]
        nodes, w = oracle.rr_set(g, LT, 8, 64, s)
        assert list(nodes) == sorted(chain)
        assert w == len(chain)


def test_in_star_with_p_one():
    L = 20
    g = synth.from_edges(L + 1, [(i, 0) for i in range(1, L + 1)])
    thr = np.full(g.m, 0xFFFFFFFF, dtype=np.uint32)
    for s in range(60):
        root = oracle.root(4, 64, s, g.n)
        nodes, w = oracle.rr_set(g, IC, 4, 64, s, thr=thr)
        if root == 0:
            assert list(nodes) == list(range(L + 1)) and w == L
        else:
            assert list(nodes) == [root] and w == 0


# ------------------------------------------- exhaustive-world identities --
def _tiny_cases():
    out = []
    for gs in (21, 22):
        g = synth.random_small_graph(7, 14, gs)
        out.append((g, IC, synth.random_thresholds(g.m, gs, choices=[0x1FFFFFFF, 0x7FFFFFFF, 0xDFFFFFFF])))
        out.append((g, IC, None))
        out.append((g, LT, None))
        out.append((g, LT, synth.random_lt_thresholds(g, gs)))                # normalized in-weights
        out.append((g, LT, synth.random_lt_thresholds(g, gs + 1, total=0.7)))  # weights summing to 0.7
        out.append((g, TRIG, synth.random_triggering(g, gs)))                      # general triggering sets
        out.append((g, TRIG, synth.random_triggering(g, gs + 7, max_outcomes=3, p_full=1.0)))  # total mass 1
    return out


_NCASES = len(_tiny_cases())


def _mask(nodes):
    return sum(1 << int(u) for u in nodes)


@pytest.mark.parametrize("case", range(_NCASES))
def test_lemma2_and_corollary1_rr_frequency_matches_exact_spread(case):
    g, model, thr = _tiny_cases()[case]
    spreads = oracle.brute_all_spreads(g, model, thr=thr)
    st = oracle.brute_rr_stats(g, model, 1, thr=thr)
    # Lemma 2, exactly: Pr[u in R] * n = E[I({u})]
    for u in range(g.n):
        assert st["p_in"][u] * g.n == pytest.approx(spreads[1 << u], rel=1e-9, abs=1e-12)
    # the oracle's sampler: frequencies within 5 sigma of the exact values
    N = 60000
    so, nodes, _ = oracle.sample_sets(g, model, 1000 + case, 64, 0, N, thr=thr)
    member = np.zeros((N, g.n), dtype=bool)
    setid = np.repeat(np.arange(N), np.diff(so))
    member[setid, nodes] = True
    freq = member.mean(axis=0)
    p = st["p_in"]
    sig = np.sqrt(np.maximum(p * (1 - p), 1e-12) / N)
    assert np.all(np.abs(freq - p) <= 5 * sig + 1e-12)
    for S in [(0, 1), (2, 5), (1, 3, 6)]:
        hit = member[:, list(S)].any(axis=1).mean()
        q = spreads[_mask(S)] / g.n
        assert abs(hit - q) <= 5 * math.sqrt(q * (1 - q) / N) + 1e-12


@pytest.mark.parametrize("case", range(_NCASES))
def test_lemma4_ept_and_sampled_width(case):
    g, model, thr = _tiny_cases()[case]
    spreads = oracle.brute_all_spreads(g, model, thr=thr)
    st = oracle.brute_rr_stats(g, model, 1, thr=thr)
    indeg = g.indeg()
    # Lemma 4: (n/m) EPT = E[I({v*})], v* drawn with probability indeg(v)/m
    lhs = g.n / g.m * st["ept"]
    rhs = sum(indeg[v] / g.m * spreads[1 << v] for v in range(g.n))
    assert lhs == pytest.approx(rhs, rel=1e-9)
    N = 40000
    _, _, widths = oracle.sample_sets(g, model, 2000 + case, 64, 0, N, thr=thr)
    wv = widths.astype(np.float64)
    assert abs(wv.mean() - st["ept"]) <= 5 * wv.std() / math.sqrt(N) + 1e-9


@pytest.mark.parametrize("case", range(_NCASES))
@pytest.mark.parametrize("k", [1, 2, 3])
def test_lemma5_kpt_equals_n_expected_kappa(case, k):
    g, model, thr = _tiny_cases()[case]
    spreads = oracle.brute_all_spreads(g, model, thr=thr)
    st = oracle.brute_rr_stats(g, model, k, thr=thr)
    indeg = g.indeg()
    nodes = [v for v in range(g.n) if indeg[v] > 0]
    # KPT: mean spread of k in-degree-weighted samples (duplicates collapse)
    kpt = 0.0
    for tup in product(nodes, repeat=k):
        pr = np.prod([indeg[v] / g.m for v in tup])
        kpt += pr * spreads[_mask(set(tup))]
    assert g.n * st["ekappa"] == pytest.approx(kpt, rel=1e-9)
    # the oracle's kappa over sampled widths estimates E[kappa]
    N = 30000
    _, _, widths = oracle.sample_sets(g, model, 3000 + case, 64, 0, N, thr=thr)
    kap = np.array([oracle.kappa(int(w), g.m, k) for w in widths])
    assert abs(kap.mean() - st["ekappa"]) <= 5 * kap.std() / math.sqrt(N) + 1e-12


# ----------------------------------------------------------------- kappa --
def test_kappa_within_rounding_bound_of_exact_value():
    rng = np.random.default_rng(5)
    u = 2.0 ** -53
    for _ in range(3000):
        m = int(rng.integers(1, 10**9))
        w = int(rng.integers(0, m + 1)) if rng.random() < 0.5 else int(rng.integers(0, min(m, 1000) + 1))
        k = int(rng.integers(1, 101))
        exact = 1 - (1 - Fraction(w, m)) ** k
        got = oracle.kappa(w, m, k)
        # q = fl(1 - fl(w/m)) has absolute error <= 2u; k-th power by squaring
        # multiplies it by <= k and adds <= 2*log2(k)+2 relative roundings.
        bound = (2 * k + 2 * math.log2(k) + 4) * u
        assert abs(Fraction(got) - exact) <= Fraction(bound)


def test_kappa_fixed_point_is_exact():
    rng = np.random.default_rng(6)
    for _ in range(2000):
        m = int(rng.integers(1, 10**8))
        w = int(rng.integers(0, m + 1))
        k = int(rng.integers(1, 101))
        K = oracle.kappa_fixed(w, m, k)
        assert Fraction(K, 2**53) == Fraction(oracle.kappa(w, m, k))


def test_kappa_special_values():
    assert oracle.kappa(0, 10, 5) == 0.0
    assert oracle.kappa(10, 10, 5) == 1.0
    assert oracle.kappa_fixed(10, 10, 1) == 2**53
    assert oracle.kappa(3, 12, 1) == 0.25  # k = 1: kappa = w/m


# ---------------------------------------------------------------- greedy --
def _read_example1():
    sets, expect, mode = [], None, None
    with open(os.path.join(GOLDEN, "example1_rr_sets.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line in ("sets", "expect"):
                mode = line
                continue
            vals = [int(x) for x in line.split()]
            if mode == "sets":
                sets.append(vals)
            else:
                expect = vals
    return sets, expect


def _csr(sets):
    off = np.zeros(len(sets) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(s) for s in sets])
    nodes = np.array([u for s in sets for u in s], dtype=np.int32)
    return off, nodes


def test_example1_greedy_picks_v4():
    sets, (k, seed, gain) = _read_example1()
    off, nodes = _csr(sets)
    seeds, gains = oracle.greedy(4, off, nodes, k)
    assert list(seeds) == [seed] and list(gains) == [gain]


def _greedy_reference_steps(n, sets, k):
    """Marginal gains recomputed from scratch at each step (ties: lowest id)."""
    covered = [False] * len(sets)
    chosen = []
    out = []
    for _ in range(k):
        gains = [sum(1 for i, s in enumerate(sets) if not covered[i] and u in s) if u not in chosen else -1
                 for u in range(n)]
        best = max(range(n), key=lambda u: (gains[u], -u))
        out.append((best, gains[best]))
        chosen.append(best)
        for i, s in enumerate(sets):
            if best in s:
                covered[i] = True
    return out


@pytest.mark.parametrize("trial", range(12))
def test_greedy_against_brute_force(trial):
    rng = np.random.default_rng(100 + trial)
    n = int(rng.integers(4, 11))
    nsets = int(rng.integers(0, 40))
    sets = [sorted(rng.choice(n, size=int(rng.integers(1, min(n, 4) + 1)), replace=False).tolist())
            for _ in range(nsets)]
    off, nodes = _csr(sets)
    for k in range(1, min(n, 4) + 1):
        seeds, gains = oracle.greedy(n, off, nodes, k)
        steps = _greedy_reference_steps(n, [set(s) for s in sets], k)
        assert [int(x) for x in seeds] == [u for u, _ in steps]
        assert [int(x) for x in gains] == [gval for _, gval in steps]
        opt, _ = oracle.brute_max_coverage(n, off, nodes, k)
        assert int(gains.sum()) >= (1 - 1 / math.e) * opt - 1e-9
        if k == 1:
            assert int(gains.sum()) == opt
        assert len(set(int(x) for x in seeds)) == k


def test_greedy_degenerate_cases():
    seeds, gains = oracle.greedy(6, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), 4)
    assert list(seeds) == [0, 1, 2, 3] and list(gains) == [0, 0, 0, 0]
    off, nodes = _csr([[2], [2], [2]])
    seeds, gains = oracle.greedy(5, off, nodes, 3)
    assert list(seeds) == [2, 0, 1] and list(gains) == [3, 0, 0]
    off, nodes = _csr([[0, 1, 2, 3]] * 5)
    seeds, gains = oracle.greedy(4, off, nodes, 4)
    assert list(seeds) == [0, 1, 2, 3] and list(gains) == [5, 0, 0, 0]


# -------------------------------------------------------------- scalars --
@pytest.mark.parametrize("n,k", [(10, 1), (10, 5), (10, 10), (15000, 50), (10**6, 50), (41_600_000, 50), (10**5, 100)])
def test_ln_binom_against_exact_binomial(n, k):
    exact = math.log(math.comb(n, k))  # exact integer binomial; math.log accepts big integers
    assert oracle.ln_binom(n, k) == pytest.approx(exact, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("n,k,eps,ell", [(15000, 50, 0.5, 1.0), (10**6, 1, 0.2, 1.0), (50, 3, 0.1, 2.0)])
def test_lambda_meets_lemma3_failure_bound(n, k, eps, ell):
    # Lemma 3's proof: with theta = lambda/OPT each set fails with probability
    # at most 2 exp(-eps^2 lambda / ((8+2eps) n)), which must equal n^-ell / C(n,k).
    lam = oracle.lam(n, k, eps, ell)
    lhs = math.log(2) - eps * eps * lam / ((8 + 2 * eps) * n)
    rhs = -ell * math.log(n) - math.log(math.comb(n, k))
    assert lhs == pytest.approx(rhs, rel=1e-10)


@pytest.mark.parametrize("n,want", [(2, 0), (3, 0), (4, 1), (7, 1), (8, 2), (15000, 12), (2**20 - 1, 18),
                                    (2**20, 19), (10**6, 18), (41_600_000, 24)])
def test_round_count_is_floor_log2_minus_one(n, want):
    assert oracle.i_max(n) == want
    assert want == max(0, n.bit_length() - 2)


def test_round_sizes_double():
    for n in (15000, 10**6):
        c = [oracle.c_i(n, 1.0, i) for i in range(1, 20)]
        for a, b in zip(c, c[1:]):
            assert 2 * a - 1 <= b <= 2 * a


@pytest.mark.parametrize("n,ell", [(15000, 1.0), (10**6, 1.0), (41_600_000, 1.0), (10**5, 1.0), (10**7, 1.0),
                                   (1000, 2.0), (4, 0.5)])
def test_round_sizes_meet_lemma6_failure_bound(n, ell):
    # Lemma 6's proof bounds an early stop in round i by exp(-c_i 2^(-i-1) / 3)
    # and needs it to be at most 1 / (n^ell log2 n): c_i is the least integer
    # with c_i 2^(-i-1) / 3 >= ell ln n + ln log2 n.
    target = ell * math.log(n) + math.log(math.log2(n))
    for i in range(1, max(2, oracle.i_max(n) + 1)):
        c = oracle.c_i(n, ell, i)
        assert c * 2.0 ** (-i - 1) / 3 >= target * (1 - 1e-14)
        assert (c - 1) * 2.0 ** (-i - 1) / 3 < target


@pytest.mark.parametrize("n,ell", [(15000, 1.0), (10**6, 1.0), (1000, 2.0)])
def test_round_sizes_meet_lemma7_bound(n, ell):
    # Lemma 7's proof: with mu >= 2^-j and i >= j+1 a late round misses its stop
    # with probability at most exp(-c_i mu / 8) < n^(-ell 2^(i-j-1)) / log2 n.
    for j in range(1, oracle.i_max(n)):
        mu = 2.0 ** -j
        for i in range(j + 1, oracle.i_max(n) + 1):
            c = oracle.c_i(n, ell, i)
            assert -c * mu / 8 < -ell * 2 ** (i - j - 1) * math.log(n) - math.log(math.log2(n))


def test_first_round_sizes_by_hand():
    # c_1 = ceil(2 (6 ell ln n + 6 ln log2 n)) at the benchmark sizes, worked by hand:
    # n = 15000: 2 (57.69 + 6 ln 13.87) = 146.9; n = 10^6: 2 (82.89 + 17.98) = 201.7;
    # n = 41.6M: 2 (105.2 + 19.45) = 249.3.
    assert oracle.c_i(15000, 1.0, 1) == 147
    assert oracle.c_i(10**6, 1.0, 1) == 202
    assert oracle.c_i(41_600_000, 1.0, 1) == 250


@pytest.mark.parametrize("n,k,eps,ell", [(15000, 50, 0.5, 1.0), (10**6, 1, 0.2, 1.0), (10**6, 10, 0.2, 1.0),
                                         (10**6, 50, 0.2, 1.0), (41_600_000, 50, 0.2, 1.0), (50, 3, 0.1, 2.0)])
def test_lambda_prime_meets_lemma8_failure_bound(n, k, eps, ell):
    # Lemma 8's proof: with theta' = lambda'/KPT* the event f n > (1+eps') OPT has
    # probability at most exp(-eps'^2 lambda' / ((2+eps') n)), which must be n^-ell.
    ep = oracle.eps_prime(k, eps, ell)
    lp = oracle.lambda_prime(n, ep, ell)
    assert -ep * ep * lp / ((2 + ep) * n) == pytest.approx(-ell * math.log(n), rel=1e-12)


def _eps_prime_hand_values():
    rows = []
    with open(os.path.join(GOLDEN, "eps_prime_hand_values.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, eps, ell, want = line.split()
                rows.append((int(k), float(eps), float(ell), want))
    return rows


@pytest.mark.parametrize("k,eps,ell,want", _eps_prime_hand_values())
def test_eps_prime_hand_values(k, eps, ell, want):
    got = oracle.eps_prime(k, eps, ell)
    assert f"{got:.4g}" == f"{float(want):.4g}"


def test_eps_prime_scales_as_a_cube_root():
    # The rule of Section 4.1 grows as eps^(2/3) and ell^(1/3) and falls as (k+ell)^(-1/3);
    # for every eps <= 1 it stays above eps / sqrt(k), where TIM+ keeps TIM's time bound.
    for k in (1, 3, 10, 50, 100):
        for eps in (0.05, 0.1, 0.2, 0.5, 1.0):
            a = oracle.eps_prime(k, eps, 1.0)
            assert oracle.eps_prime(k, eps / 8, 1.0) == pytest.approx(a / 4, rel=1e-14)
            assert oracle.eps_prime(8 * k + 7, eps, 1.0) == pytest.approx(a / 2, rel=1e-14)
            assert oracle.eps_prime(8 * k, eps, 8.0) == pytest.approx(a, rel=1e-14)
            assert a >= eps / math.sqrt(k)


# ------------------------------------------------ closed-form pipeline --
@pytest.mark.parametrize("n", [16, 50])
@pytest.mark.parametrize("model", [IC, LT])
def test_cycle_with_certain_edges_closed_form(n, model):
    # directed cycle, every node of in-degree 1: p = 1 under the weighted
    # cascade and under LT, so every RR set is the whole cycle.
    g = synth.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    k, eps, ell = 3, 0.5, 1.0
    r = oracle.tim_run(g, model, k, eps, ell, 42)
    c1 = oracle.c_i(n, ell, 1)
    assert r["i_last"] == 1 and r["c_last"] == c1
    assert r["round_sums"][1] == c1 * 2**53  # kappa = 1 for every set
    assert r["kpt_star"] == n / 2
    assert list(r["s_prime"]) == [0, 1, 2]
    assert r["covered_prime"] == r["theta_prime"]
    ep = r["eps_prime"]
    assert r["kpt_prime"] == pytest.approx(n / (1 + ep), rel=1e-15)
    assert r["kpt_plus"] == max(r["kpt_prime"], n / 2)
    assert r["theta"] == math.ceil(r["lambda"] / r["kpt_plus"])
    assert list(r["seeds"]) == [0, 1, 2]
    assert list(r["gains"]) == [r["theta"], 0, 0]
    assert r["ns_nodes"] == r["theta"] * n and r["ns_width"] == r["theta"] * n


def test_isolated_root_sets():
    # no edges into node 0 from anywhere reachable: R = {v} and w = indeg(v)
    g = synth.from_edges(5, [(1, 2), (2, 3), (3, 4)])
    thr = np.zeros(g.m, dtype=np.uint32)  # p = 2^-32: effectively never live
    thr[:] = 0
    hits = 0
    for s in range(200):
        nodes, w = oracle.rr_set(g, IC, 3, 64, s, thr=thr)
        root = oracle.root(3, 64, s, 5)
        if len(nodes) == 1:
            assert list(nodes) == [root] and w == int(g.indeg()[root])
            hits += 1
    assert hits >= 199


# ------------------------------------------------- statistical theorems --
def _tiny_model_cases():
    g1 = synth.random_small_graph(8, 16, 31)
    g2 = synth.random_small_graph(8, 18, 32)
    return [(g1, IC, synth.random_thresholds(g1.m, 31, choices=[0x3FFFFFFF, 0x9FFFFFFF])), (g2, LT, None)]


@pytest.mark.parametrize("case", [0, 1])
def test_theorem2_kpt_star_range_and_lemma8(case):
    g, model, thr = _tiny_model_cases()[case]
    k, eps, ell = 2, 0.5, 1.0
    spreads = oracle.brute_all_spreads(g, model, thr=thr)
    opt = max(spreads[_mask(S)] for S in combinations(range(g.n), k))
    indeg = g.indeg()
    nodes = [v for v in range(g.n) if indeg[v] > 0]
    kpt = sum(np.prod([indeg[v] / g.m for v in t]) * spreads[_mask(set(t))] for t in product(nodes, repeat=k))
    trials, ok_star, ok_plus = 150, 0, 0
    for s in range(trials):
        r = oracle.tim_run(g, model, k, eps, ell, 10_000 + s, thr=thr)
        ok_star += kpt / 4 <= r["kpt_star"] <= opt
        ok_plus += r["kpt_star"] <= r["kpt_plus"] <= opt
    # Theorem 2 / Lemma 8: each holds with probability >= 1 - n^-ell = 0.875
    assert ok_star / trials >= 0.875 - 3 * math.sqrt(0.875 * 0.125 / trials)
    assert ok_plus / trials >= 0.875 - 3 * math.sqrt(0.875 * 0.125 / trials)


@pytest.mark.parametrize("case", [0, 1])
def test_theorem1_and_3_approximation(case):
    g, model, thr = _tiny_model_cases()[case]
    k, eps, ell = 2, 0.3, 1.0
    spreads = oracle.brute_all_spreads(g, model, thr=thr)
    opt = max(spreads[_mask(S)] for S in combinations(range(g.n), k))
    trials, ok = 60, 0
    for s in range(trials):
        for flags in (0, oracle.FLAG_PLAIN):
            r = oracle.tim_run(g, model, k, eps, ell, 20_000 + s, flags=flags, thr=thr)
            ok += spreads[_mask(r["seeds"])] >= (1 - 1 / math.e - eps) * opt
    assert ok / (2 * trials) >= 1 - 3 / g.n  # TIM+: >= 1 - 3 n^-ell


# ------------------------------------------------- end-to-end invariants --
@pytest.mark.parametrize("model", [IC, LT])
def test_tim_plus_invariants_on_netHEPT_shaped_graph(model):
    g = synth.config_graph("cfg1")
    r = oracle.tim_run(g, model, 50, 0.5, 1.0, 1)
    seeds, gains = r["seeds"], r["gains"]
    assert len(set(seeds.tolist())) == 50
    assert np.all(np.diff(gains.astype(np.int64)) <= 0)  # coverage is submodular
    assert int(gains.sum()) == r["ns_covered"] <= r["theta"]
    assert r["kpt_plus"] >= r["kpt_star"] >= 1.0
    assert r["theta"] == math.ceil(r["lambda"] / r["kpt_plus"])
    i = r["i_last"]
    S = r["round_sums"][i]
    assert S * 2**i > r["round_c"][i] * 2**53
    for j in range(1, i):
        assert r["round_sums"][j] * 2**j <= r["round_c"][j] * 2**53


# ------------------------------------- random-number contract conformance --
# The stream layout is a convention shared by the oracle and the HIP path (the
# paper only asks for coins with probability p(e) and a uniform root); these
# tests pin the oracle to the documented formulas, using its Philox, which the
# known-answer vectors pin.
def test_contract_root_and_pick_formulas():
    rng = np.random.default_rng(9)
    for _ in range(300):
        seed = int(rng.integers(0, 2**63))
        s = int(rng.integers(0, 2**40))
        phase = int(rng.integers(1, 65))
        n = int(rng.integers(2, 2**31))
        x = oracle.draw(seed, phase, 0, 0, s)
        assert oracle.root(seed, phase, s, n) == (((x[1] << 32) | x[0]) * n) >> 64
        v = int(rng.integers(0, n))
        d = int(rng.integers(1, 2**20))
        y = oracle.draw(seed, phase, 2, v, s)
        assert oracle.lt_pick(seed, phase, s, v, d) == (((y[1] << 32) | y[0]) * d) >> 64


def test_contract_coin_word():
    rng = np.random.default_rng(10)
    for _ in range(300):
        seed, s, e = int(rng.integers(0, 2**63)), int(rng.integers(0, 2**40)), int(rng.integers(0, 2**40))
        assert oracle.coin_word(seed, 7, s, e) == oracle.draw(seed, 7, 1, e >> 2, s)[e & 3]


def test_threshold_boundary_is_inclusive():
    # one edge 0 -> 1; pick sets rooted at 1 and put the threshold exactly on
    # the set's coin word: live iff word <= t
    g = synth.from_edges(2, [(0, 1)])
    found = 0
    for s in range(200):
        if oracle.root(13, 64, s, 2) != 1:
            continue
        x = oracle.coin_word(13, 64, s, 0)
        if x == 0:
            continue
        at = oracle.rr_set(g, IC, 13, 64, s, thr=np.array([x], dtype=np.uint32))[0]
        below = oracle.rr_set(g, IC, 13, 64, s, thr=np.array([x - 1], dtype=np.uint32))[0]
        assert list(at) == [0, 1] and list(below) == [1]
        found += 1
    assert found > 50


@pytest.mark.parametrize("model", [IC, LT])
def test_stop_test_is_strict(model):
    # two disjoint certain cycles of 8 nodes: every RR set is one cycle, width
    # m/2, so with k = 1 every kappa is exactly 1/2.  Round 1 has mean exactly
    # 2^-1 (no stop: the test is strict); round 2 stops with KPT* = n/4.
    L = 8
    edges = [(i, (i + 1) % L) for i in range(L)] + [(L + i, L + (i + 1) % L) for i in range(L)]
    g = synth.from_edges(2 * L, edges)
    r = oracle.kpt_estimate(g, model, 3, 1, 1.0)
    assert r["round_sums"][1] == r["round_c"][1] * 2**52
    assert r["i_last"] == 2
    assert r["kpt_star"] == 2 * L / 4


@pytest.mark.parametrize("model", [IC, LT])
def test_round_sum_adds_kappa_of_the_sets(model):
    # one round's exact sum, width and size are those of its sets (Equation (8)),
    # split anywhere, and the rounds of KptEstimation are such sums
    g = synth.chung_lu(3000, 12000, 2.1, 5)
    k, seed = 7, 11
    so, nodes, w = oracle.sample_sets(g, model, seed, 2, 0, 500)
    want = sum(oracle.kappa_fixed(int(x), g.m, k) for x in w)
    r = oracle.round_sum(g, model, seed, 2, 0, 500, k)
    assert r["sum"] == want and r["width"] == int(np.sum(w)) and r["nodes"] == len(nodes)
    a = oracle.round_sum(g, model, seed, 2, 0, 123, k)
    b = oracle.round_sum(g, model, seed, 2, 123, 377, k)
    assert a["sum"] + b["sum"] == r["sum"] and a["width"] + b["width"] == r["width"]
    kp = oracle.kpt_estimate(g, model, seed, k, 1.0)
    for i, s in kp["round_sums"].items():
        assert oracle.round_sum(g, model, seed, i, 0, kp["round_c"][i], k)["sum"] == s


@pytest.mark.parametrize("model", [IC, LT])
def test_pipeline_is_composed_of_its_phases(model):
    # TIM+ = Algorithm 2, then Algorithm 3 on regenerated round-i_last sets and
    # fresh phase-63 sets, then Algorithm 1 on phase-64 sets.
    g = synth.chung_lu(2000, 9000, 2.1, 17)
    k, eps, ell, seed = 5, 0.5, 1.0, 23
    r = oracle.tim_run(g, model, k, eps, ell, seed)
    so, nodes, _ = oracle.sample_sets(g, model, seed, r["i_last"], 0, r["c_last"])
    sp, _ = oracle.greedy(g.n, so, nodes, k)
    assert list(sp) == list(r["s_prime"])
    so, nodes, _ = oracle.sample_sets(g, model, seed, oracle.PHASE_REFINE, 0, r["theta_prime"])
    hit = np.zeros(len(so) - 1, dtype=bool)
    setid = np.repeat(np.arange(len(so) - 1), np.diff(so))
    hit[setid[np.isin(nodes, sp)]] = True
    assert int(hit.sum()) == r["covered_prime"]
    so, nodes, widths = oracle.sample_sets(g, model, seed, oracle.PHASE_SELECT, 0, r["theta"])
    seeds, gains = oracle.greedy(g.n, so, nodes, k)
    assert list(seeds) == list(r["seeds"]) and list(gains) == list(r["gains"])
    assert int(widths.sum()) == r["ns_width"] and len(nodes) == r["ns_nodes"]


# ------------------------------------------------- forward spread (R10) --
def _descendants(n, live_edges, seeds):
    on = np.zeros(n, dtype=bool)
    on[list(seeds)] = True
    changed = True
    while changed:
        changed = False
        for u, v in live_edges:
            if on[u] and not on[v]:
                on[v] = True
                changed = True
    return int(on.sum())


@pytest.mark.parametrize("model", [IC, LT, "LT-weighted"])
def test_forward_spread_is_reach_in_the_runs_world(model):
    g = synth.random_small_graph(10, 30, 4)
    thr = synth.random_thresholds(g.m, 4, choices=[0x3FFFFFFF, 0x9FFFFFFF]) if model == IC else None
    if model == "LT-weighted":
        model, thr = LT, synth.random_lt_thresholds(g, 4, total=0.9)
    S = [1, 6]
    got = oracle.forward_spread(g, model, 31, 5, 80, S, thr=thr)
    for r in range(80):
        want = _descendants(g.n, _live_world(g, model, 31, oracle.PHASE_EVAL, 5 + r, thr), S)
        assert int(got[r]) == want, r


@pytest.mark.parametrize("case", range(_NCASES))
def test_forward_spread_mean_matches_exact_spread(case):
    g, model, thr = _tiny_cases()[case]
    spreads = oracle.brute_all_spreads(g, model, thr=thr)
    N = 40000
    for S in [(0,), (2, 5), (1, 3, 6)]:
        c = oracle.forward_spread(g, model, 500 + case, 0, N, list(S), thr=thr).astype(np.float64)
        assert abs(c.mean() - spreads[_mask(S)]) <= 5 * c.std() / math.sqrt(N) + 1e-9


def test_forward_spread_special_cases():
    g = synth.chung_lu(400, 2000, 2.1, 9)
    ones = np.full(g.m, 0xFFFFFFFF, dtype=np.uint32)  # p = 1: the spread is the set of descendants in G
    el = synth.edge_list(g)
    want = _descendants(g.n, [tuple(x) for x in el], [3, 77])
    c = oracle.forward_spread(g, IC, 2, 0, 20, [3, 77, 3], thr=ones)  # a repeated seed counts once
    assert np.all(c == want)
    assert np.all(oracle.forward_spread(g, IC, 2, 0, 5, list(range(g.n))) == g.n)
    assert np.all(oracle.forward_spread(g, LT, 2, 0, 5, []) == 0)
