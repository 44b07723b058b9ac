"""Forward Monte-Carlo spread (tim_spread_mc) against the CPU oracle, run by run."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
IC, LT = 0, 1


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def eng():
    import paper_1404_0900_amd as tim
    e = tim.Engine(0)
    yield e
    e.close()


@pytest.fixture(scope="module")
def cfg1():
    return synth.config_graph("cfg1")


def _seeds(g, k, seed):
    return np.random.default_rng(seed).choice(g.n, size=k, replace=False).astype(np.int32)


@pytest.mark.parametrize("case", ["ic-wc", "ic-trivalency", "lt", "lt-weighted"])
def test_spread_runs_equal_oracle(eng, cfg1, case):
    g = cfg1
    thr = None
    dg = eng.upload(g)
    model = IC if case.startswith("ic") else LT
    if case == "ic-trivalency":
        thr = synth.random_thresholds(g.m, 61, choices=[synth.threshold_of(p) for p in synth.TRIVALENCY_P])
        eng.free(dg)
        dg = eng.upload(g, thr=thr)
    if case == "lt-weighted":
        thr = synth.random_lt_thresholds(g, 62)
        eng.set_lt_weights(dg, g, thr)
    S = _seeds(g, 50, 63)
    mean, total, counts = eng.spread(dg, model, 64, S, 3000, first=17, per_run=True)
    want = oracle.forward_spread(g, model, 64, 17, 3000, S, thr=thr)
    got = counts.cpu().numpy().astype(np.uint64)
    _say(f"{case}: mean spread {mean:.1f}")
    assert np.array_equal(got, want)
    assert total == int(want.sum()) and mean == total / 3000
    eng.free(dg)


def test_spread_degenerate_seed_sets(eng, cfg1):
    dg = eng.upload(cfg1)
    assert eng.spread(dg, IC, 1, [], 10) == (0.0, 0)
    mean, total = eng.spread(dg, LT, 1, np.arange(cfg1.n), 10)
    assert total == 10 * cfg1.n
    a = eng.spread(dg, IC, 2, [5, 9, 5, 9, 5], 500)
    b = eng.spread(dg, IC, 2, [5, 9], 500)
    assert a == b
    eng.free(dg)


def test_spread_cfg2_sampled_runs(eng):
    g = synth.config_graph("cfg2")
    dg = eng.upload(g)
    S = _seeds(g, 50, 65)
    for model in (IC, LT):
        _, _, counts = eng.spread(dg, model, 66, S, 40, first=1000, per_run=True)
        want = oracle.forward_spread(g, model, 66, 1000, 40, S)
        assert np.array_equal(counts.cpu().numpy().astype(np.uint64), want)
    eng.free(dg)


def test_forward_spread_agrees_with_rr_estimate(eng, cfg1):
    """Corollary 1: n * Pr[R meets S] = E[I(S)]; the RR estimate and the forward mean agree statistically."""
    dg = eng.upload(cfg1)
    S = _seeds(cfg1, 20, 67)
    for model in (IC, LT):
        runs = 20000
        _, _, counts = eng.spread(dg, model, 68, S, runs, per_run=True)
        c = counts.cpu().numpy().astype(np.float64)
        sets = 400000
        st = eng.sample_cover(dg, model, 69, 65, 0, sets, S)
        p = st.covered / sets
        rr = cfg1.n * p
        sd = math.sqrt(c.var() / runs + cfg1.n ** 2 * p * (1 - p) / sets)
        _say(f"model {model}: forward {c.mean():.2f}, RR {rr:.2f}, sd {sd:.2f}")
        assert abs(c.mean() - rr) <= 5 * sd
    eng.free(dg)
