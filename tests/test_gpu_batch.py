"""Batches of TIM+ queries (tim_run_batch) against the same queries run alone.

Every query of a batch must return exactly what tim_run returns for it alone
(seeds, gains, every round sum, KPT*, KPT', KPT+, theta', theta and the
collection's totals): its RR sets are functions of its own keys, whatever
else shares the launches.  A few small batches are also checked against the
CPU oracle directly.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
IC, LT = 0, 1

KEYS = ("ell_used", "lambda", "i_max", "i_last", "c_last", "kpt_star", "round_sums", "round_c", "round_width",
        "round_nodes", "theta", "ns_nodes", "ns_width", "ns_covered", "eps_prime", "lambda_prime", "theta_prime",
        "covered_prime", "kpt_prime", "kpt_plus")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def eng():
    import paper_1404_0900_amd as tim
    e = tim.Engine(0)
    yield e
    e.close()


def _mixed_queries():
    """16 queries of the batched workload's recipe at test sizes, plus two weighted-cascade IC queries."""
    qs = synth.batch_queries(16, base_seed=2000, n_range=(2_000, 40_000), deg_range=(4.0, 40.0), k_max=20,
                             eps_choices=(0.3, 0.5))
    out = [(q, *synth.batch_graph(q)) for q in qs]
    for j, (n, m) in enumerate(((8_000, 40_000), (25_000, 200_000))):
        q = dict(name=f"wc{j}", n=n, m=m, alpha=2.1, graph_seed=2100 + j, model=IC, k=7 + j, eps=0.4, ell=1.0,
                 seed=2100 + j, thr_seed=None)
        out.append((q, synth.chung_lu(n, m, 2.1, 2100 + j, name=q["name"]), None))
    return out


@pytest.fixture(scope="module")
def mixed(eng):
    """The mixed queries, uploaded, with their results when run alone."""
    import paper_1404_0900_amd as tim
    items = _mixed_queries()
    up, alone = [], []
    for q, g, thr in items:
        dg = eng.upload(g, thr=thr)
        seeds, gains, rep = eng.run(dg, q["model"], q["k"], q["eps"], q["ell"], q["seed"])
        up.append((q, g, thr, dg))
        alone.append((seeds, gains, tim.report_dict(rep, q["k"])))
    _say(f"mixed: {len(items)} queries run alone")
    return up, alone


def _as_batch(up):
    return [(dg, q["model"], q["k"], q["eps"], q["ell"], q["seed"]) for q, _, _, dg in up]


def _same(got, want, name):
    import paper_1404_0900_amd as tim
    seeds, gains, rep = got
    k = len(seeds)
    r = tim.report_dict(rep, k)
    assert np.array_equal(seeds, want[0]), name
    assert np.array_equal(gains, want[1]), name
    for key in KEYS:
        assert r[key] == want[2][key], (name, key)
    assert np.array_equal(r["s_prime"], want[2]["s_prime"]), name


def test_batch_equals_queries_alone(eng, mixed):
    up, alone = mixed
    res, info = eng.run_batch(_as_batch(up))
    _say(f"batch: rounds={info.rounds} jobs={info.jobs} launches={info.launches} max_jobs={info.max_jobs} "
         f"wall={info.ms_wall:.1f} ms")
    assert info.rounds > 0 and info.jobs >= len(up) and info.max_jobs > 1
    for (q, *_), got, want in zip(up, res, alone):
        _same(got, want, q["name"])


def test_batch_device_kpt_granularity_keeps_results(eng, mixed):
    """The batch's KptEstimation runs on the device in chunks of at most the work-queue granularity; the
    autotuner times each candidate (2^16 .. 2^22 sets per query and step) and the results stay those of
    every query alone, whichever it keeps."""
    up, alone = mixed
    batch = _as_batch(up)
    tune = eng.autotune_batch(batch)
    _say(f"batch autotune: caps {list(tune.caps)} ms {[round(x, 2) for x in tune.ms_kpt]} kept {tune.job_cap}")
    assert tune.job_cap in list(tune.caps) and all(x > 0 for x in tune.ms_kpt)
    res, info = eng.run_batch(batch)
    assert info.kpt_job_cap == tune.job_cap and info.kpt_steps > 0 and info.kpt_graph_launches > 0
    for (q, *_), got, want in zip(up, res, alone):
        _same(got, want, q["name"])


def test_batch_with_few_workers(eng, mixed):
    up, alone = mixed
    res, info = eng.run_batch(_as_batch(up), max_concurrent=3)
    assert info.workers == 3
    for (q, *_), got, want in zip(up, res, alone):
        _same(got, want, q["name"])


def test_batch_under_a_budget_with_regenerated_chunks(mixed):
    """Four queries at a time, each with a quarter of a 1 GiB budget and at most 2000 resident sets:
    larger collections are regenerated in chunks inside the batch, with the same results."""
    import paper_1404_0900_amd as tim
    up, alone = mixed
    with tim.Engine(0, budget_bytes=1 << 30) as e:
        e.set_resident_limit(2000)
        dgs = [e.upload(g, thr=thr) for _, g, thr, _ in up]
        batch = [(dg, q["model"], q["k"], q["eps"], q["ell"], q["seed"]) for dg, (q, *_) in zip(dgs, up)]
        res, info = e.run_batch(batch, max_concurrent=4)
        assert info.budget_bytes <= 1 << 30 and info.member_budget_bytes <= info.budget_bytes // 4
        chunked = [rep.select.resident_sets for _, _, rep in res if rep.select.theta > 2000]
        _say(f"budget batch: {len(chunked)} of {len(res)} queries regenerated part of their collection")
        assert chunked and all(r <= 2000 for r in chunked)
        for (q, *_), got, want in zip(up, res, alone):
            _same(got, want, q["name"])


def test_batch_of_more_than_64_queries(eng, monkeypatch):
    """70 LT queries with a long gathering window: rounds hold more jobs of one kind than one launch
    takes (64), so they are split over several launches."""
    import paper_1404_0900_amd as tim
    qs = [q for q in synth.batch_queries(140, base_seed=3000, n_range=(500, 3_000), deg_range=(3.0, 12.0), k_max=6,
                                         eps_choices=(0.5,)) if q["model"] == LT]
    monkeypatch.setenv("TIM_BATCH_WINDOW_US", "200000")
    up, alone = [], []
    for q in qs:
        g, thr = synth.batch_graph(q)
        dg = eng.upload(g, thr=thr)
        up.append((q, g, thr, dg))
        seeds, gains, rep = eng.run(dg, q["model"], q["k"], q["eps"], q["ell"], q["seed"])
        alone.append((seeds, gains, tim.report_dict(rep, q["k"])))
    res, info = eng.run_batch(_as_batch(up))
    _say(f"70-query batch: rounds={info.rounds} launches={info.launches} max_jobs={info.max_jobs}")
    assert info.max_jobs > 64 and info.launches > info.rounds
    for (q, *_), got, want in zip(up, res, alone):
        _same(got, want, q["name"])
    for _, _, _, dg in up:
        eng.free(dg)


def test_batch_equals_oracle(eng):
    """Small queries, including a supercritical trivalency graph whose RR sets reach most nodes."""
    import paper_1404_0900_amd as tim
    items = []
    for q in synth.batch_queries(4, base_seed=4000, n_range=(1_000, 4_000), deg_range=(4.0, 12.0), k_max=8,
                                 eps_choices=(0.5,)):
        items.append((q, *synth.batch_graph(q)))
    q = dict(name="supercritical", n=2_000, m=80_000, alpha=2.1, graph_seed=4100, model=IC, k=4, eps=0.5, ell=1.0,
             seed=4100, thr_seed=4100)
    items.append((q, *synth.batch_graph(q)))
    q = dict(name="wc", n=3_000, m=15_000, alpha=2.1, graph_seed=4101, model=IC, k=5, eps=0.5, ell=1.0, seed=4101,
             thr_seed=None)
    items.append((q, synth.chung_lu(q["n"], q["m"], 2.1, q["graph_seed"]), None))
    dgs = [eng.upload(g, thr=thr) for _, g, thr in items]
    res, info = eng.run_batch([(dg, q["model"], q["k"], q["eps"], q["ell"], q["seed"])
                               for dg, (q, _, _) in zip(dgs, items)])
    for (q, g, thr), (seeds, gains, rep) in zip(items, res):
        _say(f"oracle: {q['name']} model={q['model']} n={g.n} m={g.m} k={q['k']}")
        want = oracle.tim_run(g, q["model"], q["k"], q["eps"], q["ell"], q["seed"], thr=thr)
        r = tim.report_dict(rep, q["k"])
        assert np.array_equal(seeds, want["seeds"]) and np.array_equal(gains, want["gains"]), q["name"]
        for key in KEYS:
            assert r[key] == want[key], (q["name"], key)
    big = tim.report_dict(res[4][2], 4)
    # a mean of about 100 nodes per set: the sets that reach the giant component hold far more than the
    # first tier's 128-node queue, so the later tiers ran inside the batched launches
    assert big["ns_nodes"] > 50 * big["theta"]
    for dg in dgs:
        eng.free(dg)


def test_batch_rejects_a_bad_query(eng, mixed):
    import paper_1404_0900_amd as tim
    up, _ = mixed
    batch = _as_batch(up[:3])
    dg, model, k, eps, ell, seed = batch[1]
    batch[1] = (dg, model, k, 1.5, ell, seed)  # eps outside (0, 1]
    with pytest.raises(tim.TimError) as ei:
        eng.run_batch(batch)
    assert ei.value.status == tim.EINVAL and "query 1" in str(ei.value)
