"""LT with random normalized in-weights (Section 7.1) on the GPU against the CPU oracle.

The weights are uint32 cumulative thresholds per in-edge (synth.random_lt_thresholds); the walk at v
takes the first in-edge whose threshold is at least word 0 of v's pick draw, and stops when the word
exceeds them all (weights summing below 1).  Every set, width, kappa sum, covered count, KPT*, KPT+,
theta, seed and gain must be identical.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
LT = 1


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


def _upload(eng, g, lthr):
    dg = eng.upload(g)
    eng.set_lt_weights(dg, g, lthr)
    return dg


def _graphs():
    cfg1 = synth.config_graph("cfg1")
    dense = synth.chung_lu(300_000, 9_000_000, 2.1, 22)  # walks of up to about 140 nodes: both LT tiers
    return [("cfg1 normalized", cfg1, synth.random_lt_thresholds(cfg1, 41)),
            ("cfg1 total 0.6", cfg1, synth.random_lt_thresholds(cfg1, 42, total=0.6)),
            ("dense normalized", dense, synth.random_lt_thresholds(dense, 43))]


@pytest.mark.parametrize("case", range(3))
def test_weighted_lt_sets_widths_kappa_and_cover(eng, case):
    name, g, lthr = _graphs()[case]
    dg = _upload(eng, g, lthr)
    count, first = 20000, 7
    _say(f"weighted LT sets: {name}")
    so, nodes, widths, st = eng.sample_rr(dg, LT, 13, 64, first, count)
    so, nd = _sorted_sets(so.cpu().numpy(), nodes.cpu().numpy())
    wso, wnd, ww = oracle.sample_sets(g, LT, 13, 64, first, count, thr=lthr)
    assert np.array_equal(so, wso) and np.array_equal(nd, wnd)
    assert np.array_equal(widths.cpu().numpy().astype(np.uint64), ww)
    sizes = np.diff(wso)
    _say(f"  set sizes mean {sizes.mean():.2f} max {sizes.max()}, deferred {st.deferred}")
    w, sz, wst = eng.sample_widths(dg, LT, 13, 64, first, count, 11)
    assert np.array_equal(w.cpu().numpy().astype(np.uint64), ww)
    assert np.array_equal(sz.cpu().numpy(), sizes.astype(np.int32))
    assert wst.kappa_sum == sum(oracle.kappa_fixed(int(x), g.m, 11) for x in ww)
    seeds = np.unique(wnd[:: max(1, len(wnd) // 50)])[:40].astype(np.int32)
    cst = eng.sample_cover(dg, LT, 13, 64, first, count, seeds)
    sid = np.repeat(np.arange(count), sizes)
    hit = np.zeros(count, dtype=bool)
    hit[sid[np.isin(wnd, seeds)]] = True
    assert cst.covered == int(hit.sum())
    if case == 2:
        assert sizes.max() > 64 and st.deferred > 0  # the long-chain tier took part
    eng.free(dg)


@pytest.mark.parametrize("total", [None, 0.8])
def test_weighted_lt_tim_plus_equals_oracle(eng, cfg1, total):
    import paper_1404_0900_amd as tim
    lthr = synth.random_lt_thresholds(cfg1, 44, total=total)
    dg = _upload(eng, cfg1, lthr)
    k, eps, ell, seed = 20, 0.5, 1.0, 45
    seeds, gains, rep = eng.run(dg, LT, k, eps, ell, seed)
    r = tim.report_dict(rep, k)
    want = oracle.tim_run(cfg1, LT, k, eps, ell, seed, thr=lthr)
    assert np.array_equal(seeds, want["seeds"]) and np.array_equal(gains, want["gains"])
    for key in ("i_last", "c_last", "kpt_star", "round_sums", "theta_prime", "covered_prime", "kpt_plus", "theta",
                "ns_nodes", "ns_width", "ns_covered"):
        assert r[key] == want[key], key
    eng.free(dg)


def test_weighted_lt_in_a_batch(eng, cfg1):
    """Queries on the same graph with and without weights in one batch equal their runs alone."""
    import paper_1404_0900_amd as tim
    lthr = synth.random_lt_thresholds(cfg1, 46)
    dw = _upload(eng, cfg1, lthr)
    du = eng.upload(cfg1)
    batch = [(dw, LT, 10, 0.5, 1.0, 50), (du, LT, 10, 0.5, 1.0, 50), (dw, LT, 3, 0.4, 1.0, 51),
             (du, 0, 7, 0.5, 1.0, 52)]
    res, info = eng.run_batch(batch)
    for b, (seeds, gains, rep) in zip(batch, res):
        s2, g2, r2 = eng.run(*b)
        assert np.array_equal(seeds, s2) and np.array_equal(gains, g2)
        assert rep.select.theta == r2.select.theta and rep.refine.kpt_plus == r2.refine.kpt_plus
    # the weights change the answer
    assert not np.array_equal(res[0][0], res[1][0])
    eng.free(dw)
    eng.free(du)


def test_lt_weights_are_checked_and_can_be_removed(eng, cfg1):
    import paper_1404_0900_amd as tim
    dg = eng.upload(cfg1)
    bad = synth.random_lt_thresholds(cfg1, 47)
    v = int(np.flatnonzero(np.diff(cfg1.off) >= 2)[0])
    bad[cfg1.off[v]], bad[cfg1.off[v] + 1] = 100, 50  # decreasing within node v
    with pytest.raises(tim.TimError) as ei:
        eng.set_lt_weights(dg, cfg1, bad)
    assert ei.value.status == tim.EINVAL
    eng.set_lt_weights(dg, cfg1, synth.random_lt_thresholds(cfg1, 48))
    eng.set_lt_weights(dg, cfg1, None)  # back to 1/indeg
    so, nodes, _, _ = eng.sample_rr(dg, LT, 3, 64, 0, 3000)
    so, nd = _sorted_sets(so.cpu().numpy(), nodes.cpu().numpy())
    wso, wnd, _ = oracle.sample_sets(cfg1, LT, 3, 64, 0, 3000)
    assert np.array_equal(so, wso) and np.array_equal(nd, wnd)
    eng.free(dg)
