"""TIM+ end to end against the oracle on seeded random small cases: graph size and density, the
model (IC with weighted cascade or per-edge trivalency probabilities, LT), k, eps and ell are drawn
per case, so that the runs stop in different KptEstimation rounds (from the first to the last),
keep or regenerate R', and take theta from KPT* or KPT'.  Seeds, gains and every scalar of
Algorithms 1-3 must match the oracle exactly."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KEYS = ("ell_used", "lambda", "i_max", "i_last", "c_last", "kpt_star", "round_sums", "theta", "ns_nodes", "ns_width",
        "ns_covered", "eps_prime", "lambda_prime", "theta_prime", "covered_prime", "kpt_prime", "kpt_plus")


def _case(cs):
    r = np.random.default_rng(1000 + cs)
    n = int(r.integers(30, 5000))
    m = int(min(n * (n - 1), n * r.uniform(1.5, 12.0)))
    model = int(r.integers(0, 2))
    k = int(r.integers(1, min(n, 40) + 1))
    eps = float(r.choice([0.4, 0.5, 0.7, 1.0]))
    ell = float(r.choice([0.5, 1.0, 2.0]))
    use_thr = model == 0 and bool(r.integers(0, 2))
    return n, m, model, k, eps, ell, use_thr


def _graph(n, m, seed):
    # m distinct random edges u -> v, u != v
    r = np.random.default_rng(seed)
    u = r.integers(0, n, size=3 * m + 16)
    v = r.integers(0, n, size=3 * m + 16)
    keep = u != v
    u, v = u[keep], v[keep]
    _, first = np.unique(u.astype(np.int64) * n + v, return_index=True)
    pick = np.sort(first)[:m]
    return synth.from_edges(n, [(int(a), int(b)) for a, b in zip(u[pick], v[pick])], name=f"rand_n{n}_s{seed}")


@pytest.fixture(scope="module")
def eng():
    import paper_1404_0900_amd as tim
    e = tim.Engine(0)
    yield e
    e.close()


@pytest.mark.parametrize("cs", range(24))
def test_tim_plus_random_case_equals_oracle(eng, cs):
    import paper_1404_0900_amd as tim
    n, m, model, k, eps, ell, use_thr = _case(cs)
    print(f"case {cs}: n={n} m={m} model={model} k={k} eps={eps} ell={ell} thresholds={use_thr}", file=sys.stderr,
          flush=True)
    g = _graph(n, m, cs)
    thr = synth.random_thresholds(g.m, cs, [synth.threshold_of(p) for p in synth.TRIVALENCY_P]) if use_thr else None
    seed = 77 + cs
    seeds, gains, rep = eng.run(eng.upload(g, thr=thr), model, k, eps, ell, seed)
    got = tim.report_dict(rep, k)
    want = oracle.tim_run(g, model, k, eps, ell, seed, thr=thr)
    assert np.array_equal(seeds, want["seeds"])
    assert np.array_equal(gains, want["gains"])
    for key in KEYS:
        assert got[key] == want[key], key
    assert np.array_equal(got["s_prime"], want["s_prime"][:128])


def _check_equal(seeds, gains, rep, k, want):
    import paper_1404_0900_amd as tim
    got = tim.report_dict(rep, k)
    assert np.array_equal(seeds, want["seeds"])
    assert np.array_equal(gains, want["gains"])
    for key in KEYS:
        assert got[key] == want[key], key


@pytest.mark.parametrize("concurrent", [5, 0])
def test_random_cases_as_one_batch_and_served(eng, concurrent):
    """The 24 cases as one batch (5 at a time, or all at once), then through a server with 6 slots:
    every query equals the oracle."""
    cases = [_case(cs) for cs in range(24)]
    graphs, thrs, wants, queries = [], [], [], []
    for cs, (n, m, model, k, eps, ell, use_thr) in enumerate(cases):
        g = _graph(n, m, cs)
        thr = synth.random_thresholds(g.m, cs, [synth.threshold_of(p) for p in synth.TRIVALENCY_P]) if use_thr else None
        wants.append(oracle.tim_run(g, model, k, eps, ell, 77 + cs, thr=thr))
        queries.append((eng.upload(g, thr=thr), model, k, eps, ell, 77 + cs))
    print(f"batch of 24 random cases, {concurrent} at a time", file=sys.stderr, flush=True)
    res, _ = eng.run_batch(queries, max_concurrent=concurrent)
    for (seeds, gains, rep), q, want in zip(res, queries, wants):
        _check_equal(seeds, gains, rep, q[2], want)
    print("server with 6 slots over the 24 random cases", file=sys.stderr, flush=True)
    with eng.serve(6) as srv:
        tickets = [srv.submit(*q) for q in queries]
        got = [srv.wait(t) for t in tickets]
    for (seeds, gains, rep, _lat), q, want in zip(got, queries, wants):
        _check_equal(seeds, gains, rep, q[2], want)


@pytest.mark.parametrize("cs", range(10))
def test_triggering_random_case_equals_oracle(eng, cs):
    """The general triggering model (Section 4.2) on seeded random graphs and random per-node
    distributions over in-edge subsets (synth.random_triggering), with random k, eps and ell."""
    import paper_1404_0900_amd as tim
    r = np.random.default_rng(2000 + cs)
    n = int(r.integers(30, 3000))
    m = int(min(n * (n - 1), n * r.uniform(1.5, 10.0)))
    k = int(r.integers(1, min(n, 30) + 1))
    eps = float(r.choice([0.5, 0.7, 1.0]))
    ell = float(r.choice([0.5, 1.0, 2.0]))
    outcomes, size = int(r.integers(1, 6)), int(r.integers(1, 5))
    p_full = float(r.choice([0.0, 0.25, 1.0]))
    print(f"triggering case {cs}: n={n} m={m} k={k} eps={eps} ell={ell} outcomes<={outcomes} size<={size} "
          f"p_full={p_full}", file=sys.stderr, flush=True)
    g = _graph(n, m, 500 + cs)
    trig = synth.random_triggering(g, 600 + cs, max_outcomes=outcomes, max_size=size, p_full=p_full)
    dg = eng.upload(g)
    eng.set_triggering(dg, g, trig)
    seed = 91 + cs
    seeds, gains, rep = eng.run(dg, tim.TRIGGER, k, eps, ell, seed)
    want = oracle.tim_run(g, tim.TRIGGER, k, eps, ell, seed, thr=trig)
    _check_equal(seeds, gains, rep, k, want)
    eng.free(dg)


@pytest.mark.parametrize("cs", range(8))
def test_lt_weights_random_case_equals_oracle(eng, cs):
    """LT with random in-weights (Section 7.1), normalized or summing to less than one, on seeded
    random graphs with random k, eps and ell."""
    import paper_1404_0900_amd as tim
    r = np.random.default_rng(3000 + cs)
    n = int(r.integers(30, 4000))
    m = int(min(n * (n - 1), n * r.uniform(1.5, 12.0)))
    k = int(r.integers(1, min(n, 40) + 1))
    eps = float(r.choice([0.4, 0.5, 0.7, 1.0]))
    ell = float(r.choice([0.5, 1.0, 2.0]))
    total = [None, 0.5, 0.9][int(r.integers(0, 3))]
    print(f"LT weights case {cs}: n={n} m={m} k={k} eps={eps} ell={ell} total={total}", file=sys.stderr, flush=True)
    g = _graph(n, m, 700 + cs)
    lthr = synth.random_lt_thresholds(g, 800 + cs, total=total)
    dg = eng.upload(g)
    eng.set_lt_weights(dg, g, lthr)
    seed = 31 + cs
    seeds, gains, rep = eng.run(dg, tim.LT, k, eps, ell, seed)
    want = oracle.tim_run(g, tim.LT, k, eps, ell, seed, thr=lthr)
    _check_equal(seeds, gains, rep, k, want)
    eng.free(dg)


@pytest.mark.parametrize("cs", range(10))
def test_spread_random_case_equals_oracle(eng, cs):
    """Forward Monte-Carlo spread (the live-edge view of Section 2.2) run by run on seeded random
    graphs: model (IC with weighted cascade or trivalency, LT with 1/indeg or random in-weights, the
    general triggering model), seed-set size, number of runs and first run id are drawn per case."""
    import paper_1404_0900_amd as tim
    r = np.random.default_rng(4000 + cs)
    n = int(r.integers(20, 3000))
    m = int(min(n * (n - 1), n * r.uniform(1.0, 10.0)))
    kind = ["ic-wc", "ic-trivalency", "lt", "lt-weighted", "trigger"][cs % 5]
    size = int(r.integers(0, min(n, 60) + 1))
    runs = int(r.integers(1, 2500))
    first = int(r.integers(0, 1 << 40))
    seed = int(r.integers(1, 1 << 62))
    print(f"spread case {cs}: {kind} n={n} m={m} |S|={size} runs={runs} first={first}", file=sys.stderr, flush=True)
    g = _graph(n, m, 900 + cs)
    S = r.choice(n, size=size, replace=False).astype(np.int32)
    thr, model = None, tim.IC
    if kind == "ic-trivalency":
        thr = synth.random_thresholds(g.m, cs, [synth.threshold_of(p) for p in synth.TRIVALENCY_P])
        dg = eng.upload(g, thr=thr)
    else:
        dg = eng.upload(g)
    if kind.startswith("lt"):
        model = tim.LT
        if kind == "lt-weighted":
            thr = synth.random_lt_thresholds(g, 950 + cs, total=0.8)
            eng.set_lt_weights(dg, g, thr)
    if kind == "trigger":
        model = tim.TRIGGER
        thr = synth.random_triggering(g, 960 + cs, max_outcomes=3, max_size=3)
        eng.set_triggering(dg, g, thr)
    mean, total, counts = eng.spread(dg, model, seed, S, runs, first=first, per_run=True)
    want = oracle.forward_spread(g, model, seed, first, runs, S, thr=thr)
    assert np.array_equal(counts.cpu().numpy().astype(np.uint64), want)
    assert total == int(want.sum())
    eng.free(dg)


def _sorted_sets(so, nodes):
    out = nodes.copy()
    for i in range(len(so) - 1):
        out[so[i]:so[i + 1]] = np.sort(nodes[so[i]:so[i + 1]])
    return so, out


@pytest.mark.parametrize("cs", range(10))
def test_rr_sets_random_case_equal_oracle(eng, cs):
    """Every RR set (sorted), its width and the launch totals on seeded random graphs: the model and
    its weights, the phase, the first set id (up to 2^45) and the count are drawn per case, so that
    launches take the 64-lane or the 8-lane first tier and sets of every size reach every tier."""
    import paper_1404_0900_amd as tim
    r = np.random.default_rng(5000 + cs)
    n = int(r.integers(10, 6000))
    m = int(min(n * (n - 1), n * r.uniform(1.0, 14.0)))
    kind = ["ic-wc", "ic-trivalency", "ic-high", "lt", "lt-weighted", "trigger"][cs % 6]
    phase = int(r.integers(1, 65))
    first = int(r.integers(0, 1 << 45))
    count = int(r.integers(1, 300_000))
    if kind in ("ic-high", "trigger"):
        count = count % 5000 + 1  # sets of thousands of nodes (a giant reverse-reachable component)
    seed = int(r.integers(1, 1 << 62))
    print(f"sets case {cs}: {kind} n={n} m={m} phase={phase} first={first} count={count}", file=sys.stderr,
          flush=True)
    g = _graph(n, m, 1100 + cs)
    thr, model = None, tim.IC
    if kind in ("ic-trivalency", "ic-high"):
        ps = synth.TRIVALENCY_P if kind == "ic-trivalency" else (0.5, 0.25, 0.1)
        thr = synth.random_thresholds(g.m, cs, [synth.threshold_of(p) for p in ps])
        dg = eng.upload(g, thr=thr)
    else:
        dg = eng.upload(g)
    if kind.startswith("lt"):
        model = tim.LT
        if kind == "lt-weighted":
            thr = synth.random_lt_thresholds(g, 1150 + cs)
            eng.set_lt_weights(dg, g, thr)
    if kind == "trigger":
        model = tim.TRIGGER
        thr = synth.random_triggering(g, 1160 + cs, max_outcomes=4, max_size=4)
        eng.set_triggering(dg, g, thr)
    so, nodes, widths, st = eng.sample_rr(dg, model, seed, phase, first, count)
    so, nd = _sorted_sets(so.cpu().numpy(), nodes.cpu().numpy())
    wso, wnd, ww = oracle.sample_sets(g, model, seed, phase, first, count, thr=thr)
    assert np.array_equal(so, wso)
    assert np.array_equal(nd, wnd)
    assert np.array_equal(widths.cpu().numpy().astype(np.uint64), ww)
    assert st.node_sum == len(wnd) and st.width_sum == int(ww.sum())
    eng.free(dg)


@pytest.mark.parametrize("kind", ["ic-high", "lt", "trigger"])
def test_rr_sets_few_sets_per_launch_equal_oracle(eng, kind):
    """Launches of 1 to 65 sets: fewer sets than work-cursor parts (eight per tier), ragged part
    sizes, and sets large enough to be deferred to the later tiers."""
    import paper_1404_0900_amd as tim
    g = _graph(1500, 12000, 77)
    thr, model = None, tim.IC
    if kind == "ic-high":
        thr = synth.random_thresholds(g.m, 78, [synth.threshold_of(p) for p in (0.5, 0.25, 0.1)])
        dg = eng.upload(g, thr=thr)
    else:
        dg = eng.upload(g)
    if kind == "lt":
        model = tim.LT
    if kind == "trigger":
        model = tim.TRIGGER
        thr = synth.random_triggering(g, 79, max_outcomes=4, max_size=4, p_full=1.0)
        eng.set_triggering(dg, g, thr)
    for count in (1, 2, 3, 7, 8, 9, 15, 16, 17, 63, 64, 65):
        print(f"few sets: {kind} count={count}", file=sys.stderr, flush=True)
        so, nodes, widths, st = eng.sample_rr(dg, model, 5, 9, 1000 + count, count)
        so, nd = _sorted_sets(so.cpu().numpy(), nodes.cpu().numpy())
        wso, wnd, ww = oracle.sample_sets(g, model, 5, 9, 1000 + count, count, thr=thr)
        assert np.array_equal(so, wso), count
        assert np.array_equal(nd, wnd), count
        assert np.array_equal(widths.cpu().numpy().astype(np.uint64), ww), count
    eng.free(dg)
