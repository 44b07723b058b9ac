"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer results (every RR set as a node set, widths, sizes, exact kappa sums,
covered counts, rounds, theta values, seeds and gains) must be identical; the
binary64 scalars (KPT*, KPT', KPT+) are computed by both sides from identical
integers with the same operation order and must be bit-identical too.  The
order of nodes inside one RR set is not defined by the method, so sets are
compared sorted.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
IC, LT = 0, 1


@pytest.fixture(scope="module")
def eng():
    import paper_1404_0900_amd as tim
    e = tim.Engine(0)
    yield e
    e.close()


@pytest.fixture(scope="module")
def cfg1():
    return synth.config_graph("cfg1")


@pytest.fixture(scope="module")
def cfg2():
    return synth.config_graph("cfg2")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _sorted_sets(set_off, nodes):
    so = np.asarray(set_off, dtype=np.int64)
    nd = np.asarray(nodes, dtype=np.int32)
    sid = np.repeat(np.arange(len(so) - 1), np.diff(so))
    return so, nd[np.lexsort((nd, sid))]


def _gpu_sets(eng, dg, model, seed, phase, first, count):
    so, nodes, widths, st = eng.sample_rr(dg, model, seed, phase, first, count)
    so, nd = _sorted_sets(so.cpu().numpy(), nodes.cpu().numpy())
    return so, nd, widths.cpu().numpy().astype(np.uint64), st


def _check_sets(eng, g, model, seed, phase, first, count, thr=None, dg=None):
    dg = dg or eng.upload(g, thr=thr)
    _say(f"sets: {g.name} model={model} phase={phase} first={first} count={count}")
    so, nd, w, st = _gpu_sets(eng, dg, model, seed, phase, first, count)
    wso, wnd, ww = oracle.sample_sets(g, model, seed, phase, first, count, thr=thr)
    assert np.array_equal(so, wso)
    assert np.array_equal(nd, wnd)
    assert np.array_equal(w, ww)
    assert st.node_sum == len(wnd) and st.width_sum == int(ww.sum())
    return st


# ------------------------------------------------------------- RR sets --
@pytest.mark.parametrize("model", [IC, LT])
def test_rr_sets_cfg1_weighted_cascade(eng, cfg1, model):
    _check_sets(eng, cfg1, model, 1, 64, 0, 30000)


def test_rr_sets_cfg1_per_edge_thresholds(eng, cfg1):
    # p(e) in {0.1, 0.01, 0.001}: t = floor(p * 2^32) - 1
    thr = synth.random_thresholds(cfg1.m, 5, choices=[429496728, 42949671, 4294966])
    _check_sets(eng, cfg1, IC, 3, 64, 0, 20000, thr=thr)


def test_rr_sets_high_probability_thresholds(eng, cfg1):
    # supercritical: many sets outgrow LDS and finish in the large-set pass
    thr = synth.random_thresholds(cfg1.m, 6, choices=[0x7FFFFFFF, 0xBFFFFFFF, 0xFFFFFFFF])
    st = _check_sets(eng, cfg1, IC, 4, 64, 0, 3000, thr=thr)
    assert st.deferred > 0


@pytest.mark.parametrize("model", [IC, LT])
def test_rr_sets_ragged_ranges_and_large_ids(eng, cfg1, model):
    dg = eng.upload(cfg1)
    for first, count in [(0, 1), (7, 63), (2**40 + 5, 1000), (2**33 - 3, 4097)]:
        _check_sets(eng, cfg1, model, 11, 5, first, count, dg=dg)


@pytest.mark.parametrize("model", [IC, LT])
def test_rr_sets_certain_cycle_uses_large_set_pass(eng, model):
    # every set is the whole 2000-node cycle: longer than the LDS structures
    n = 2000
    g = synth.from_edges(n, [(i, (i + 1) % n) for i in range(n)], name="cycle2000")
    st = _check_sets(eng, g, model, 9, 64, 0, 300)
    assert st.deferred == 300


@pytest.mark.parametrize("model", [IC, LT])
def test_rr_sets_tiny_graphs(eng, model):
    for gs in range(4):
        g = synth.random_small_graph(9, 24, gs)
        thr = synth.random_thresholds(g.m, gs, choices=[0x3FFFFFFF, 0xBFFFFFFF]) if model == IC else None
        _check_sets(eng, g, model, 100 + gs, 64, 0, 2000, thr=thr)


@pytest.mark.parametrize("model", [IC, LT])
def test_rr_sets_cfg2_sampled(eng, cfg2, model):
    # full-size graph, a ragged slice of set ids well inside the NodeSelection range
    _check_sets(eng, cfg2, model, 2, 64, 123457, 20011)


def _functional_graph(n, seed, ends):
    """Each node has one in-edge from a random other node (a fraction `ends` has none): LT walks are
    deterministic rho shapes (a tail into a cycle, about sqrt(n) long) or paths to a node without in-edges."""
    rng = np.random.default_rng(seed)
    u = rng.integers(0, n - 1, size=n)
    v = np.arange(n)
    u = u + (u >= v)
    keep = rng.random(n) >= ends
    return synth.from_edges(n, np.stack([u[keep], v[keep]], axis=1).tolist(), name=f"functional_n{n}_s{seed}")


@pytest.mark.parametrize("which", ["functional", "dense"])
def test_lt_long_chains_all_modes(eng, which):
    """LT walks far longer than the first tier's 64-node chain (the long-chain tier finds where each walk
    repeats with Brent's cycle search): stored sets, widths with exact kappa sums, and coverage."""
    g = _functional_graph(300_000, 21, 0.0005) if which == "functional" else synth.chung_lu(300_000, 9_000_000, 2.1, 22)
    dg = eng.upload(g)
    count = 6000
    st = _check_sets(eng, g, LT, 31, 64, 5, count, dg=dg)
    so, nodes, ww = oracle.sample_sets(g, LT, 31, 64, 5, count)
    sizes = np.diff(so)
    _say(f"{which}: set sizes mean {sizes.mean():.1f} max {sizes.max()}, deferred {st.deferred}")
    assert sizes.max() > 100 and st.deferred > 0
    w, sz, wst = eng.sample_widths(dg, LT, 31, 64, 5, count, 9)
    assert np.array_equal(w.cpu().numpy().astype(np.uint64), ww)
    assert np.array_equal(sz.cpu().numpy(), sizes.astype(np.int32))
    assert wst.kappa_sum == sum(oracle.kappa_fixed(int(x), g.m, 9) for x in ww)
    seeds = np.unique(nodes[:: max(1, len(nodes) // 40)])[:30].astype(np.int32)
    cst = eng.sample_cover(dg, LT, 31, 64, 5, count, seeds)
    sid = np.repeat(np.arange(count), sizes)
    hit = np.zeros(count, dtype=bool)
    hit[sid[np.isin(nodes, seeds)]] = True
    assert cst.covered == int(hit.sum())
    eng.free(dg)


# ------------------------------------------------------ widths / kappa --
@pytest.mark.parametrize("model", [IC, LT])
@pytest.mark.parametrize("k", [1, 50])
def test_widths_sizes_and_exact_kappa_sum(eng, cfg1, model, k):
    dg = eng.upload(cfg1)
    count = 25000
    _say(f"widths: model={model} k={k}")
    w, sz, st = eng.sample_widths(dg, model, 1, 9, 0, count, k)
    so, nodes, ww = oracle.sample_sets(cfg1, model, 1, 9, 0, count)
    assert np.array_equal(w.cpu().numpy().astype(np.uint64), ww)
    assert np.array_equal(sz.cpu().numpy(), np.diff(so).astype(np.int32))
    want = sum(oracle.kappa_fixed(int(x), cfg1.m, k) for x in ww)
    assert st.kappa_sum == want
    assert st.width_sum == int(ww.sum()) and st.node_sum == int(so[-1])


def test_kappa_bit_identity_over_many_widths(eng):
    # a star-of-stars graph whose sets have widths spread over [0, m]
    g = synth.chung_lu(5000, 40000, 2.1, 3)
    thr = synth.random_thresholds(g.m, 8)
    dg = eng.upload(g, thr=thr)
    w, _, st = eng.sample_widths(dg, IC, 3, 2, 0, 20000, 7)
    ww = w.cpu().numpy()
    want = sum(oracle.kappa_fixed(int(x), g.m, 7) for x in ww)
    assert st.kappa_sum == want


# ------------------------------------------------------------ coverage --
@pytest.mark.parametrize("model", [IC, LT])
def test_cover_counts(eng, cfg1, model):
    dg = eng.upload(cfg1)
    seeds = np.array([1559, 11944, 8686, 2086, 7, 100, 14999], dtype=np.int32)
    st = eng.sample_cover(dg, model, 5, 63, 0, 30000, seeds)
    so, nodes, _ = oracle.sample_sets(cfg1, model, 5, 63, 0, 30000)
    sid = np.repeat(np.arange(30000), np.diff(so))
    hit = np.zeros(30000, dtype=bool)
    hit[sid[np.isin(nodes, seeds)]] = True
    assert st.covered == int(hit.sum())


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.asarray(a), dtype=dtype, device="cuda")


def test_max_coverage_example1(eng):
    import torch
    off = _dev([0, 2, 3, 4, 5], torch.int64)
    nodes = _dev([0, 3, 1, 2, 3], torch.int32)
    seeds, gains = eng.max_coverage(4, off, nodes, 1)
    assert list(seeds) == [3] and list(gains) == [2]


def test_max_coverage_random_collections(eng):
    import torch
    rng = np.random.default_rng(3)
    for trial in range(20):
        n = int(rng.integers(2, 400))
        nsets = int(rng.integers(0, 3000))
        sets = [rng.choice(n, size=int(rng.integers(1, min(n, 30) + 1)), replace=False) for _ in range(nsets)]
        off = np.zeros(nsets + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(s) for s in sets])
        nodes = np.concatenate(sets).astype(np.int32) if nsets else np.zeros(0, dtype=np.int32)
        k = int(rng.integers(1, min(n, 60) + 1))
        seeds, gains = eng.max_coverage(n, _dev(off, torch.int64), _dev(nodes, torch.int32), k)
        ws, wg = oracle.greedy(n, off, nodes, k)
        assert np.array_equal(seeds, ws) and np.array_equal(gains, wg), trial


@pytest.mark.parametrize("n", [20000, 5000])
def test_max_coverage_many_chunks_per_bucket(eng, n):
    # The counts and index are built by a counting sort over buckets of 8192 consecutive node ids, each
    # bucket counted in chunks of 65536 entries: sets drawn mostly from a few low ids put hundreds of
    # thousands of entries into the first bucket (many chunks, merged by device atomics) beside buckets of
    # one chunk (stored directly) and a last bucket shorter than 8192 ids.
    import torch
    rng = np.random.default_rng(11 + n)
    nsets = 60000
    sizes = rng.integers(1, 12, size=nsets)
    sets = []
    for sz in sizes:
        hot = rng.choice(64, size=min(int(sz), 64), replace=False)
        cold = rng.choice(n, size=int(sz), replace=False)
        sets.append(np.unique(np.where(rng.random(int(sz)) < 0.7, hot[: int(sz)], cold)))
    off = np.zeros(nsets + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(x) for x in sets])
    nodes = np.concatenate(sets).astype(np.int32)
    assert np.sum(nodes < 8192) > 4 * 65536
    for k in (1, 10):
        seeds, gains = eng.max_coverage(n, _dev(off, torch.int64), _dev(nodes, torch.int32), k)
        ws, wg = oracle.greedy(n, off, nodes, k)
        assert np.array_equal(seeds, ws) and np.array_equal(gains, wg), k


@pytest.mark.parametrize("k", [1, 2, 5])
def test_max_coverage_empty_collection(eng, k):
    # no sets: every gain is 0 and the tie rule takes the lowest unselected ids
    import torch
    off = _dev([0], torch.int64)
    nodes = _dev(np.zeros(0, dtype=np.int32), torch.int32)
    seeds, gains = eng.max_coverage(7, off, nodes, k)
    ws, wg = oracle.greedy(7, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), k)
    assert list(ws) == list(range(k))
    assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)


def test_max_coverage_rejects_bad_ids(eng):
    import torch

    import paper_1404_0900_amd as tim
    with pytest.raises(tim.TimError):
        eng.max_coverage(3, _dev([0, 2], torch.int64), _dev([0, 5], torch.int32), 1)


# -------------------------------------------------------------- phases --
def _kpt_equal(res, want):
    assert res.i_max == want["i_max"] and res.i_last == want["i_last"] and res.c_last == want["c_last"]
    assert res.kpt_star == want["kpt_star"]
    assert res.round_sums() == want["round_sums"]


@pytest.mark.parametrize("model", [IC, LT])
def test_kpt_estimate_cfg1(eng, cfg1, model):
    dg = eng.upload(cfg1)
    for k in (1, 5, 50):
        _say(f"kpt: model={model} k={k}")
        _kpt_equal(eng.kpt_estimate(dg, model, 1, k, 1.0), oracle.kpt_estimate(cfg1, model, 1, k, 1.0))


@pytest.mark.parametrize("model", [IC, LT])
def test_refine_and_node_select_cfg1(eng, cfg1, model):
    dg = eng.upload(cfg1)
    k, eps, ell = 50, 0.5, 1.0
    kp = oracle.kpt_estimate(cfg1, model, 1, k, ell)
    sp, rr = eng.refine_kpt(dg, model, 1, k, eps, ell, kp["kpt_star"], kp["i_last"], kp["c_last"])
    want = oracle.refine_kpt(cfg1, model, 1, k, eps, ell, kp["kpt_star"], kp["i_last"], kp["c_last"])
    assert np.array_equal(sp, want["s_prime"])
    assert rr.theta_prime == want["theta_prime"] and rr.covered_prime == want["covered_prime"]
    assert rr.kpt_prime == want["kpt_prime"] and rr.kpt_plus == want["kpt_plus"]
    seeds, gains, sel = eng.node_select(dg, model, 1, k, 40000)
    w = oracle.node_select(cfg1, model, 1, k, 40000)
    assert np.array_equal(seeds, w["seeds"]) and np.array_equal(gains, w["gains"])
    assert sel.nodes == w["ns_nodes"] and sel.width == w["ns_width"] and sel.covered == w["ns_covered"]


def _run_equal(eng, g, dg, model, k, eps, ell, seed, flags=0, thr=None):
    import paper_1404_0900_amd as tim
    _say(f"tim_run: {g.name} model={model} k={k} eps={eps} flags={flags}")
    seeds, gains, rep = eng.run(dg, model, k, eps, ell, seed, flags)
    r = tim.report_dict(rep, k)
    want = oracle.tim_run(g, model, k, eps, ell, seed, flags=flags, thr=thr)
    assert np.array_equal(seeds, want["seeds"])
    assert np.array_equal(gains, want["gains"])
    for key in ("ell_used", "lambda", "i_max", "i_last", "c_last", "kpt_star", "round_sums", "theta", "ns_nodes",
                "ns_width", "ns_covered"):
        assert r[key] == want[key], key
    if not flags & tim.FLAG_PLAIN:
        for key in ("eps_prime", "lambda_prime", "theta_prime", "covered_prime", "kpt_prime", "kpt_plus"):
            assert r[key] == want[key], key
        assert np.array_equal(r["s_prime"], want["s_prime"][:128])
    return r


@pytest.mark.parametrize("model", [IC, LT])
def test_tim_plus_cfg1(eng, cfg1, model):
    dg = eng.upload(cfg1)
    _run_equal(eng, cfg1, dg, model, 50, 0.5, 1.0, 1)


@pytest.mark.parametrize("flags", [1, 2, 3])
def test_tim_flags_cfg1(eng, cfg1, flags):
    dg = eng.upload(cfg1)
    _run_equal(eng, cfg1, dg, IC, 20, 0.5, 1.0, 2, flags=flags)


def test_tim_plus_per_edge_thresholds(eng, cfg1):
    thr = synth.random_thresholds(cfg1.m, 12, choices=[429496728, 42949671, 4294966])
    dg = eng.upload(cfg1, thr=thr)
    _run_equal(eng, cfg1, dg, IC, 10, 0.5, 1.0, 3, thr=thr)


@pytest.mark.parametrize("model", [IC, LT])
def test_tim_plus_degenerate_graphs(eng, model):
    # certain cycle (every set = V, closed form) and a tiny graph with k = n
    n = 700
    g = synth.from_edges(n, [(i, (i + 1) % n) for i in range(n)], name="cycle700")
    r = _run_equal(eng, g, eng.upload(g), model, 3, 0.5, 1.0, 4)
    assert r["kpt_star"] == n / 2
    g2 = synth.random_small_graph(6, 12, 2)
    _run_equal(eng, g2, eng.upload(g2), model, 6, 1.0, 1.0, 5)
    g3 = synth.from_edges(2, [(0, 1)])
    _run_equal(eng, g3, eng.upload(g3), model, 1, 0.5, 0.5, 6)


@pytest.mark.parametrize("model", [IC, LT])
def test_tim_plus_cfg2_k50(eng, cfg2, model):
    dg = eng.upload(cfg2)
    _run_equal(eng, cfg2, dg, model, 50, 0.2, 1.0, 2)


def _golden_timplus():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "timplus_chunglu_n1e6_m1e7_k1_k10.json")) as f:
        return json.load(f)


def _decode(v):
    if isinstance(v, str):
        return float.fromhex(v)
    if isinstance(v, dict):
        return {int(i): x for i, x in v.items()}
    return v


@pytest.mark.parametrize("model", [IC, LT])
@pytest.mark.parametrize("k", [1, 10])
def test_tim_plus_cfg2_k1_k10_against_stored_oracle(eng, cfg2, model, k):
    # The oracle needs minutes for these runs, so its results come from
    # tests/golden/make_timplus_golden.py (oracle only), stored with the graph's hash.
    import hashlib

    import paper_1404_0900_amd as tim
    doc = _golden_timplus()
    h = hashlib.sha256()
    h.update(cfg2.off.astype("<i8").tobytes())
    h.update(cfg2.src.astype("<i4").tobytes())
    assert doc["graph"]["sha256"] == h.hexdigest(), "stored oracle values belong to another graph"
    want = {key: _decode(v) for key, v in
            next(r["result"] for r in doc["runs"] if r["model"] == model and r["k"] == k).items()}
    dg = eng.upload(cfg2)
    _say(f"tim_run: cfg2 model={model} k={k} against the stored oracle run")
    seeds, gains, rep = eng.run(dg, model, k, doc["eps"], doc["ell"], doc["seed"])
    r = tim.report_dict(rep, k)
    assert list(seeds) == want["seeds"] and [int(x) for x in gains] == want["gains"]
    for key in ("ell_used", "lambda", "i_max", "i_last", "c_last", "kpt_star", "round_sums", "round_c",
                "round_width", "round_nodes", "eps_prime", "lambda_prime", "theta_prime", "covered_prime",
                "kpt_prime", "kpt_plus", "theta", "ns_nodes", "ns_width", "ns_covered"):
        assert r[key] == want[key], key
    assert [int(x) for x in r["s_prime"][:k]] == want["s_prime"][:128]


@pytest.mark.parametrize("k", [10, 50])
def test_grouped_rounds_count_once_and_keep_the_last_round(eng, cfg2, k):
    # The early KptEstimation rounds run together and the next ones in pairs.  Rounds computed past the
    # stopping one are dropped and not counted, and the last round, predicted here right after a group
    # (k = 50) or a pair (k = 10), is stored and reused as R' instead of being generated again: the sets
    # generated are exactly the rounds up to i_last, theta' and theta.
    import paper_1404_0900_amd as tim
    dg = eng.upload(cfg2)
    _, _, rep = eng.run(dg, IC, k, 0.2, 1.0, 2)
    r = tim.report_dict(rep, k)
    _say(f"grouped rounds: k={k} i_last={r['i_last']} sets_total={r['sets_total']}")
    assert r["i_last"] >= 12
    assert r["sets_total"] == sum(r["round_c"].values()) + r["theta_prime"] + r["theta"]


@pytest.mark.parametrize("model", [IC, LT])
def test_kpt_cfg2_k1_sampled(eng, cfg2, model):
    # k = 1 takes the oracle minutes end to end; check the GPU's rounds on
    # sampled sets of every round and by the exact stop rule.
    dg = eng.upload(cfg2)
    res = eng.kpt_estimate(dg, model, 2, 1, 1.0)
    rng = np.random.default_rng(model)
    for i in range(1, res.i_last + 1):
        ci = int(res.round_c[i])
        assert ci == oracle.c_i(cfg2.n, 1.0, i)
        stop = res.round_sums()[i] * 2**i > ci * 2**53
        assert stop == (i == res.i_last)
        ids = rng.choice(ci, size=min(ci, 200), replace=False)
        w, _, _ = eng.sample_widths(dg, model, 2, i, 0, ci, 1)
        w = w.cpu().numpy()
        for s in ids:
            _, ww = oracle.rr_set(cfg2, model, 2, i, int(s))
            assert int(w[s]) == ww
        assert sum(int(x) for x in w) == int(res.round_width[i])
    assert res.kpt_star == (res.round_sums()[res.i_last] / 2**53) * cfg2.n / (2 * int(res.round_c[res.i_last])) or \
        math.isclose(res.kpt_star, res.round_sums()[res.i_last] / 2**53 * cfg2.n / (2 * int(res.round_c[res.i_last])),
                     rel_tol=1e-15)


# -------------------------------------------------- determinism / errors --
def test_results_do_not_depend_on_context_or_repeat(eng, cfg1):
    import paper_1404_0900_amd as tim
    dg = eng.upload(cfg1)
    a = eng.run(dg, IC, 10, 0.5, 1.0, 77)
    b = eng.run(dg, IC, 10, 0.5, 1.0, 77)
    with tim.Engine(0) as e2:
        c = e2.run(e2.upload(cfg1), IC, 10, 0.5, 1.0, 77)
    for x in (b, c):
        assert np.array_equal(a[0], x[0]) and np.array_equal(a[1], x[1])
        assert a[2].select.width == x[2].select.width and a[2].kpt.kpt_star == x[2].kpt.kpt_star


def test_invalid_arguments_raise(eng, cfg1):
    import paper_1404_0900_amd as tim
    dg = eng.upload(cfg1)
    for args in [(IC, 0, 0.5, 1.0), (IC, cfg1.n + 1, 0.5, 1.0), (IC, 5, 0.0, 1.0), (IC, 5, 1.5, 1.0),
                 (IC, 5, 0.5, 0.4), (7, 5, 0.5, 1.0)]:
        with pytest.raises(tim.TimError) as ei:
            eng.run(dg, args[0], args[1], args[2], args[3], 1)
        assert ei.value.status == tim.EINVAL
    bad = synth.Graph(3, 2, np.array([0, 1, 2, 2]), np.array([0, 0], dtype=np.int32))  # self-loop 0->0
    with pytest.raises(tim.TimError):
        eng.upload(bad)


def test_budget_too_small_is_reported(cfg1):
    import paper_1404_0900_amd as tim
    with tim.Engine(0, budget_bytes=1 << 16) as e:
        dg = e.upload(cfg1)
        with pytest.raises(tim.TimError) as ei:
            e.run(dg, IC, 10, 0.5, 1.0, 1)
        assert ei.value.status == tim.EBUDGET


# ------------------------------------- NodeSelection under a memory budget --
def _select_equal(sel, seeds, gains, want):
    assert np.array_equal(seeds, want["seeds"]) and np.array_equal(gains, want["gains"])
    assert sel.nodes == want["ns_nodes"] and sel.width == want["ns_width"] and sel.covered == want["ns_covered"]


@pytest.mark.parametrize("model", [IC, LT])
def test_node_select_fully_regenerated(cfg1, model):
    # resident limit 0: every set is regenerated after every greedy step
    import paper_1404_0900_amd as tim
    k, theta = 20, 30000
    want = oracle.node_select(cfg1, model, 7, k, theta)
    with tim.Engine(0) as e:
        e.set_resident_limit(0)
        dg = e.upload(cfg1)
        _say(f"node_select regenerated: model={model} k={k} theta={theta}")
        seeds, gains, sel = e.node_select(dg, model, 7, k, theta)
    assert sel.resident_sets == 0 and sel.chunk_sets > 0
    assert sel.regenerated_sets == (k - 1) * theta
    _select_equal(sel, seeds, gains, want)


@pytest.mark.parametrize("model", [IC, LT])
def test_node_select_resident_prefix_and_chunks(cfg1, model):
    # a resident prefix with its index plus the rest in regenerated chunks
    import paper_1404_0900_amd as tim
    k, theta = 50, 100000
    want = oracle.node_select(cfg1, model, 8, k, theta)
    with tim.Engine(0) as e:
        e.set_resident_limit(theta // 3)
        dg = e.upload(cfg1)
        _say(f"node_select prefix: model={model} k={k} theta={theta}")
        seeds, gains, sel = e.node_select(dg, model, 8, k, theta)
        assert sel.resident_sets == theta // 3
        assert sel.regenerated_sets == (k - 1) * (theta - theta // 3)
        _select_equal(sel, seeds, gains, want)
        e.set_resident_limit(None)
        seeds2, gains2, sel2 = e.node_select(dg, model, 8, k, theta)
        assert sel2.resident_sets == theta and sel2.chunk_sets == 0 and sel2.regenerated_sets == 0
        _select_equal(sel2, seeds2, gains2, want)


@pytest.mark.parametrize("model", [IC, LT])
def test_node_select_under_budget_uses_many_chunks(cfg1, model):
    # a budget far below the collection: the plan keeps a prefix and streams
    # the rest in many chunks, under the budget throughout
    import paper_1404_0900_amd as tim
    k, theta, budget = 30, 400000, 12 << 20
    want = oracle.node_select(cfg1, model, 9, k, theta)
    with tim.Engine(0, budget_bytes=budget) as e:
        dg = e.upload(cfg1)
        _say(f"node_select budget: model={model} k={k} theta={theta} budget={budget}")
        seeds, gains, sel = e.node_select(dg, model, 9, k, theta)
        assert e.device_bytes() <= budget
    _say(f"  resident={sel.resident_sets} chunk={sel.chunk_sets} regenerated={sel.regenerated_sets}")
    assert 0 < sel.resident_sets < theta
    assert 0 < sel.chunk_sets and (theta - sel.resident_sets) // sel.chunk_sets >= 4
    _select_equal(sel, seeds, gains, want)


@pytest.mark.parametrize("limit", [None, 0])
def test_node_select_pool_regrowth(cfg1, limit):
    # supercritical probabilities: sets far larger than NodeSelection's size
    # estimate, so the node pool is regrown (resident and regenerated paths)
    import paper_1404_0900_amd as tim
    thr = np.full(cfg1.m, (1 << 31) - 1, dtype=np.uint32)  # p = 1/2
    k, theta = 10, 3000
    want = oracle.node_select(cfg1, IC, 21, k, theta, thr=thr)
    with tim.Engine(0) as e:
        e.set_resident_limit(limit)
        dg = e.upload(cfg1, thr=thr)
        _say(f"node_select regrowth: limit={limit}")
        seeds, gains, sel = e.node_select(dg, IC, 21, k, theta)
    assert sel.nodes > 16 * theta
    _select_equal(sel, seeds, gains, want)


def test_tim_plus_under_budget_cfg1(cfg1):
    # whole TIM+ (RefineKPT's greedy and NodeSelection) under a small budget
    import paper_1404_0900_amd as tim
    with tim.Engine(0, budget_bytes=6 << 20) as e:
        dg = e.upload(cfg1)
        r = _run_equal(e, cfg1, dg, IC, 50, 0.5, 1.0, 1)
        assert e.device_bytes() <= 6 << 20
    assert r["theta"] > 0


def test_max_coverage_large_tiles_overflow_lds_tables(eng):
    # tiles with more distinct nodes than the LDS aggregation tables hold, and
    # a few heavy nodes present in most sets (the hub pattern of RR sets)
    import torch
    rng = np.random.default_rng(11)
    n, nsets = 200_000, 3000
    hubs = np.arange(5)
    sets = []
    for _ in range(nsets):
        size = int(rng.integers(1, 400))
        body = rng.choice(n - 5, size=size, replace=False) + 5
        h = hubs[rng.random(5) < 0.6]
        sets.append(np.concatenate([h, body]))
    off = np.zeros(nsets + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(s) for s in sets])
    nodes = np.concatenate(sets).astype(np.int32)
    for k in (1, 7, 40):
        seeds, gains = eng.max_coverage(n, _dev(off, torch.int64), _dev(nodes, torch.int32), k)
        ws, wg = oracle.greedy(n, off, nodes, k)
        assert np.array_equal(seeds, ws) and np.array_equal(gains, wg), k


_LARGE = {}


@pytest.mark.parametrize("lanes", ["4", "8", "16", "32", "64"])
def test_large_launches_every_shape(cfg1, lanes, monkeypatch):
    # width, stored-set and coverage launches of 262144 sets or more run the context's first-tier shape
    # (smaller ones take the 64-lane shape): every shape's widths, sizes, exact kappa sum, stored sets and
    # coverage count
    import paper_1404_0900_amd as tim
    monkeypatch.setenv("TIM_IC_SEG_LANES", lanes)
    count, seed, phase, k = 300_000, 4, 11, 5
    seeds = np.array([1559, 11944, 8686, 2086], dtype=np.int32)
    if not _LARGE:
        so, nodes, ww = oracle.sample_sets(cfg1, IC, seed, phase, 0, count)
        sid = np.repeat(np.arange(count), np.diff(so))
        hit = np.zeros(count, dtype=bool)
        hit[sid[np.isin(nodes, seeds)]] = True
        _LARGE.update(so=so, nodes=nodes, ww=ww, covered=int(hit.sum()),
                      kappa=oracle.round_sum(cfg1, IC, seed, phase, 0, count, k)["sum"])
    want = _LARGE
    _say(f"large launches: {lanes} lanes per set")
    with tim.Engine(0) as e:
        dg = e.upload(cfg1)
        w, sz, st = e.sample_widths(dg, IC, seed, phase, 0, count, k)
        assert np.array_equal(w.cpu().numpy().astype(np.uint64), want["ww"])
        assert np.array_equal(sz.cpu().numpy(), np.diff(want["so"]).astype(np.int32))
        assert st.kappa_sum == want["kappa"]
        assert st.width_sum == int(want["ww"].sum()) and st.node_sum == int(want["so"][-1])
        cst = e.sample_cover(dg, IC, seed, phase, 0, count, seeds)
        assert cst.covered == want["covered"]
        so, nd, w2, st2 = _gpu_sets(e, dg, IC, seed, phase, 0, count)
        assert np.array_equal(so, want["so"]) and np.array_equal(nd, want["nodes"])
        assert np.array_equal(w2, want["ww"]) and st2.node_sum == int(want["so"][-1])


@pytest.mark.parametrize("lanes", ["4", "16", "32", "64"])
def test_segment_width_does_not_change_results(cfg1, cfg2, lanes, monkeypatch):
    # the IC tier-0 kernel's lanes per set is a launch-shape choice only
    import paper_1404_0900_amd as tim
    monkeypatch.setenv("TIM_IC_SEG_LANES", lanes)
    with tim.Engine(0) as e:
        _check_sets(e, cfg1, IC, 1, 64, 0, 20000)
        _check_sets(e, cfg2, IC, 2, 64, 5, 5000)
        _run_equal(e, cfg1, e.upload(cfg1), IC, 50, 0.5, 1.0, 1)
