"""TIM+ under device-memory budgets from a geometric sweep, with the real kernels (row A10: a
collection and its index that do not fit are kept in part and regenerated in chunks; the last
KptEstimation round is kept for RefineKPT only where its index fits).  A larger budget must never
fail where a smaller one ran every query, and every run must give the results of the run without a
budget, which for one query is checked against the oracle as well.  The graph is a Chung-Lu graph
with per-edge trivalency probabilities: its RR sets vary widely in size, so that rounds and
collections come out larger or smaller than the previous round predicts."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _key(res):
    seeds, gains, rep = res
    return (tuple(int(x) for x in seeds), tuple(int(x) for x in gains), rep.kpt.i_last, rep.kpt.kpt_star,
            rep.refine.theta_prime, rep.refine.covered_prime, rep.refine.kpt_plus, rep.select.theta,
            rep.select.nodes, rep.select.width)


def test_budget_sweep_equals_unbudgeted():
    import paper_1404_0900_amd as tim
    g = synth.chung_lu(20_000, 400_000, 2.1, seed=5, name="chung_lu_20k")
    thr = synth.random_thresholds(g.m, 7, [synth.threshold_of(p) for p in synth.TRIVALENCY_P])
    # (graph with per-edge thresholds?, model, k, eps, seed)
    queries = [(False, tim.IC, 1, 0.3, 11), (True, tim.IC, 10, 0.3, 12), (False, tim.LT, 25, 0.4, 13),
               (True, tim.IC, 40, 0.5, 14)]

    def run_all(budget):
        out = []
        with tim.Engine(0, budget_bytes=budget) as e:
            dgs = {False: e.upload(g), True: e.upload(g, thr=thr)}
            for with_thr, model, k, eps, seed in queries:
                try:
                    out.append(_key(e.run(dgs[with_thr], model, k, eps, 1.0, seed)))
                except tim.TimError as err:
                    assert err.status == tim.EBUDGET, str(err)
                    out.append(None)
            if budget:
                assert e.device_bytes() <= budget
        return out

    _say("budget sweep: unbudgeted reference")
    ref = run_all(0)
    # the reference of the second query against the oracle
    want = oracle.tim_run(g, tim.IC, 10, 0.3, 1.0, 12, thr=thr)
    assert list(ref[1][0]) == list(want["seeds"]) and list(ref[1][1]) == list(want["gains"])
    assert ref[1][7] == want["theta"]
    all_ok = False
    failed = []  # queries that did not fit, per budget
    budget = 1 << 17
    while budget <= 1 << 30:
        got = run_all(budget)
        ok = [r is not None for r in got]
        failed.append(len(ok) - sum(ok))
        _say(f"budget sweep: {budget} bytes, {sum(ok)} of {len(ok)} queries ran")
        for i, r in enumerate(got):
            if r is not None:
                assert r == ref[i], (budget, i)
        if all(ok):
            all_ok = True
        else:
            assert not all_ok, f"budget {budget} failed a query that a smaller budget ran"
        budget = int(budget * 1.6)
    # the sweep spans budgets too small for some query and budgets that run every one
    assert all_ok and failed[0] > 0
