"""The general triggering model (Section 4.2) on the GPU against the CPU oracle.

Every node's triggering set is drawn from an explicit distribution over subsets of its in-edges
(synth.random_triggering; reading R11 of the oracle).  Every RR set, width, size, exact kappa sum,
covered count, forward spread and the whole TIM+ run (rounds, KPT*, KPT+, theta, seeds, gains) must be
identical to the oracle's.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TRIG = 2


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


def _sorted_sets(set_off, nodes):
    so = np.asarray(set_off, dtype=np.int64)
    nd = np.asarray(nodes, dtype=np.int32)
    sid = np.repeat(np.arange(len(so) - 1), np.diff(so))
    return so, nd[np.lexsort((nd, sid))]


def _upload(eng, g, trig):
    dg = eng.upload(g)
    eng.set_triggering(dg, g, trig)
    return dg


def _cases():
    cfg1 = synth.config_graph("cfg1")
    small = synth.chung_lu(2000, 16000, 2.1, 31)
    giant = synth.chung_lu(8000, 120000, 2.1, 72)
    return [("cfg1 mass 0.3-0.8", cfg1, synth.random_triggering(cfg1, 61)),
            # total probability 1 and up to 5 members per outcome: sets of up to about 400 nodes, so
            # some outgrow the first tier's 128 nodes and finish in the one-set-per-wavefront tier
            ("cfg1 mass 1", cfg1, synth.random_triggering(cfg1, 62, max_outcomes=3, max_size=5, p_full=1.0)),
            ("dense 2K", small, synth.random_triggering(small, 63, max_outcomes=6, max_size=3, p_full=0.5)),
            # a giant reverse-reachable component: most sets have about 3000 nodes and finish in the block
            # tier after passing through the other two
            ("giant 8K", giant, synth.random_triggering(giant, 72, max_outcomes=2, max_size=6, p_full=1.0))]


@pytest.mark.parametrize("case", range(4))
def test_trigger_sets_widths_kappa_and_cover(eng, case):
    name, g, trig = _cases()[case]
    dg = _upload(eng, g, trig)
    count, first = (3000 if case == 3 else 12000), 5
    _say(f"triggering sets: {name}")
    so, nodes, widths, st = eng.sample_rr(dg, TRIG, 17, 64, first, count)
    so, nd = _sorted_sets(so.cpu().numpy(), nodes.cpu().numpy())
    wso, wnd, ww = oracle.sample_sets(g, TRIG, 17, 64, first, count, thr=trig)
    assert np.array_equal(so, wso) and np.array_equal(nd, wnd)
    assert np.array_equal(widths.cpu().numpy().astype(np.uint64), ww)
    sizes = np.diff(wso)
    _say(f"  set sizes mean {sizes.mean():.2f} max {sizes.max()}, deferred {st.deferred}")
    if case == 1:
        assert sizes.max() > 128 and st.deferred > 0  # the second tier took part
    if case == 3:
        assert sizes.max() > 1024 and sizes.min() <= 128 and st.deferred > 0  # every tier took part
    w, sz, wst = eng.sample_widths(dg, TRIG, 17, 64, first, count, 7)
    assert np.array_equal(w.cpu().numpy().astype(np.uint64), ww)
    assert np.array_equal(sz.cpu().numpy(), sizes.astype(np.int32))
    assert wst.kappa_sum == sum(oracle.kappa_fixed(int(x), g.m, 7) for x in ww)
    seeds = np.unique(wnd[:: max(1, len(wnd) // 50)])[:40].astype(np.int32)
    cst = eng.sample_cover(dg, TRIG, 17, 64, first, count, seeds)
    sid = np.repeat(np.arange(count), sizes)
    hit = np.zeros(count, dtype=bool)
    hit[sid[np.isin(wnd, seeds)]] = True
    assert cst.covered == int(hit.sum())
    eng.free(dg)


@pytest.mark.parametrize("case", [0, 1])
def test_trigger_tim_plus_equals_oracle(eng, case):
    import paper_1404_0900_amd as tim
    name, g, trig = _cases()[case]
    dg = _upload(eng, g, trig)
    k, eps, ell, seed = 25, 0.5, 1.0, 71
    _say(f"triggering TIM+: {name}")
    seeds, gains, rep = eng.run(dg, TRIG, k, eps, ell, seed)
    r = tim.report_dict(rep, k)
    want = oracle.tim_run(g, TRIG, k, eps, ell, seed, thr=trig)
    assert np.array_equal(seeds, want["seeds"]) and np.array_equal(gains, want["gains"])
    for key in ("i_last", "c_last", "kpt_star", "round_sums", "round_width", "round_nodes", "theta_prime",
                "covered_prime", "kpt_prime", "kpt_plus", "theta", "ns_nodes", "ns_width", "ns_covered"):
        assert r[key] == want[key], key
    eng.free(dg)


def test_trigger_spread_equals_oracle(eng, cfg1):
    trig = synth.random_triggering(cfg1, 64)
    dg = _upload(eng, cfg1, trig)
    seeds = np.array([3, 77, 1500, 9000, 14999], dtype=np.int32)
    mean, total, per = eng.spread(dg, TRIG, 9, seeds, 3000, first=11, per_run=True)
    want = oracle.forward_spread(cfg1, TRIG, 9, 11, 3000, seeds, thr=trig)
    assert np.array_equal(per.cpu().numpy().astype(np.uint64), want)
    assert total == int(want.sum())
    eng.free(dg)


def test_trigger_distribution_is_checked_and_can_be_removed(eng, cfg1):
    import paper_1404_0900_amd as tim
    dg = eng.upload(cfg1)
    with pytest.raises(tim.TimError):  # no distribution yet
        eng.run(dg, TRIG, 5, 0.5, 1.0, 1)
    good = synth.random_triggering(cfg1, 65)
    v = int(np.flatnonzero(np.diff(good.toff) >= 2)[0])
    bad = synth.Triggering(good.toff, good.tthr.copy(), good.tset, good.tmem)
    bad.tthr[good.toff[v]], bad.tthr[good.toff[v] + 1] = 100, 50  # decreasing within node v
    with pytest.raises(tim.TimError) as ei:
        eng.set_triggering(dg, cfg1, bad)
    assert ei.value.status == tim.EINVAL
    j = int(good.toff[v])
    bad = synth.Triggering(good.toff, good.tthr, good.tset, good.tmem.copy())
    bad.tmem[good.tset[j]] = np.diff(cfg1.off)[v]  # not an in-edge of v
    with pytest.raises(tim.TimError):
        eng.set_triggering(dg, cfg1, bad)
    eng.set_triggering(dg, cfg1, good)
    eng.set_triggering(dg, cfg1, None)
    with pytest.raises(tim.TimError):
        eng.run(dg, TRIG, 5, 0.5, 1.0, 1)
    # not in batches
    eng.set_triggering(dg, cfg1, good)
    with pytest.raises(tim.TimError):
        eng.run_batch([(dg, TRIG, 5, 0.5, 1.0, 1)])
    eng.free(dg)
