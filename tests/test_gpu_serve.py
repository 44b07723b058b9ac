"""The request loop (tim_server_*): queries submitted over time give the results of tim_run alone."""
import sys
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KEYS = ("lambda", "i_last", "c_last", "kpt_star", "round_sums", "theta", "ns_nodes", "ns_width", "ns_covered",
        "theta_prime", "covered_prime", "kpt_plus")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    import paper_1404_0900_amd as tim
    e = tim.Engine(0)
    graphs = synth.serve_graphs(scale=0.005)
    dgs = [e.upload(g) for g in graphs]
    qs = synth.serve_queries(24, 400.0, 11, k_max=30, eps_choices=(0.3, 0.5))
    alone = []
    for q in qs:
        seeds, gains, rep = e.run(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"])
        alone.append((seeds, gains, tim.report_dict(rep, q["k"])))
    _say(f"serve: {len(qs)} queries run alone on graphs of {[g.n for g in graphs]} nodes")
    yield e, dgs, qs, alone
    e.close()


def _same(got, want, i):
    import paper_1404_0900_amd as tim
    seeds, gains, rep = got[:3]
    r = tim.report_dict(rep, len(seeds))
    assert np.array_equal(seeds, want[0]) and np.array_equal(gains, want[1]), i
    for key in KEYS:
        assert r[key] == want[2][key], (i, key)


def test_served_queries_equal_queries_alone(setup):
    e, dgs, qs, alone = setup
    with e.serve(slots=6) as srv:
        t0 = time.perf_counter()
        tickets = []
        for q in qs:  # Poisson arrivals: submit each query at its arrival time
            delay = q["arrival"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"]))
        results = [srv.wait(t) for t in tickets]
        info = srv.stop()
    lat = np.array([r[3] for r in results])
    _say(f"served: rounds={info.rounds} launches={info.launches} max_jobs={info.max_jobs} "
         f"latency p50={np.median(lat):.1f} ms max={lat.max():.1f} ms")
    assert info.rounds > 0 and np.all(lat > 0)
    for i, (got, want) in enumerate(zip(results, alone)):
        _same(got, want, i)


def test_stop_finishes_queued_queries(setup):
    e, dgs, qs, alone = setup
    srv = e.serve(slots=2)
    outs = []
    for i, q in enumerate(qs[:8]):
        t = srv.submit(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"])
        outs.append(srv._pending[t])
    srv.stop()  # no wait: the queued queries still run to the end
    for i, (qstruct, seeds, gains, rep) in enumerate(outs):
        assert qstruct.status == 0
        _same((seeds, gains, rep), alone[i], i)


def test_server_rejects_bad_queries_and_other_calls(setup):
    import paper_1404_0900_amd as tim
    e, dgs, qs, _ = setup
    with e.serve(slots=2) as srv:
        with pytest.raises(tim.TimError) as ei:
            srv.submit(dgs[0], tim.IC, 0, 0.5, 1.0, 1)  # k = 0
        assert ei.value.status == tim.EINVAL
        q = qs[0]
        with pytest.raises(tim.TimError):  # the context runs a server: no batch meanwhile
            e.run_batch([(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"])])
        t = srv.submit(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"])
        srv.wait(t)


def test_served_queries_equal_the_oracle():
    """Queries served over time on small resident graphs against the CPU oracle directly."""
    import oracle

    import paper_1404_0900_amd as tim
    graphs = synth.serve_graphs(scale=0.02)  # 2K, 20K, 80K and 200K nodes, average degree 16
    qs = synth.serve_queries(10, 300.0, 21, k_max=12, eps_choices=(0.5,))
    with tim.Engine(0) as e:
        dgs = [e.upload(g) for g in graphs]
        with e.serve(slots=4) as srv:
            tickets = [srv.submit(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"]) for q in qs]
            results = [srv.wait(t) for t in tickets]
            srv.stop()
    for i, (q, (seeds, gains, rep, _)) in enumerate(zip(qs, results)):
        g = graphs[q["graph"]]
        _say(f"served vs oracle: query {i} n={g.n} model={q['model']} k={q['k']}")
        want = oracle.tim_run(g, q["model"], q["k"], q["eps"], q["ell"], q["seed"])
        r = tim.report_dict(rep, q["k"])
        assert np.array_equal(seeds, want["seeds"]) and np.array_equal(gains, want["gains"]), i
        for key in KEYS:
            assert r[key] == want[key], (i, key)


def test_admission_by_theta_bytes_holds_queries_and_keeps_results(setup, monkeypatch):
    """An RR pool of 8 MB (TIM_RR_POOL_BYTES) under a 512 MB budget fits few collections at once:
    NodeSelections wait for memory in request order (none is refused; one larger than the pool gets the
    whole pool and regenerates its collection in chunks), the pool is never over-granted, and every
    result stays that of the query alone."""
    import paper_1404_0900_amd as tim
    _, _, qs, alone = setup
    graphs = synth.serve_graphs(scale=0.005)
    monkeypatch.setenv("TIM_RR_POOL_BYTES", str(8 << 20))
    with tim.Engine(0, budget_bytes=512 << 20) as e:
        dgs = [e.upload(g) for g in graphs]
        with e.serve(slots=8) as srv:
            tickets = [srv.submit(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"]) for q in qs]
            results = [srv.wait(t) for t in tickets]
            info = srv.stop()
    _say(f"admission: pool {info.rr_pool_bytes >> 20} MB, peak {info.rr_peak_bytes >> 20} MB, "
         f"{info.held_queries} held for {info.held_ms:.1f} ms")
    assert info.rr_pool_bytes == 8 << 20 and 0 < info.rr_peak_bytes <= info.rr_pool_bytes
    assert info.held_queries > 0
    for i, (got, want) in enumerate(zip(results, alone)):
        _same(got, want, i)
