"""The sampler-shape autotuner (tim_autotune): it times the candidates and keeps one; results stay the
oracle's."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
IC, LT = 0, 1


@pytest.mark.parametrize("model", [IC, LT])
def test_autotune_keeps_results(model):
    import paper_1404_0900_amd as tim
    g = synth.config_graph("cfg1")
    with tim.Engine(0) as e:
        dg = e.upload(g)
        r = e.autotune(dg, model, 1 << 16)
        assert r.seg_lanes in (4, 8, 16, 32, 64) and r.slice_cap in (512, 1024, 2048, 4096)
        assert all(x > 0 for x in r.ms_emit)
        if model == IC:
            assert all(x > 0 for x in r.ms_width) and all(x > 0 for x in r.ms_lanes_emit)
            # the chosen shape is the current one or one at least 3% faster than it on a width launch plus a
            # stored-set launch
            times = {lanes: w + e for lanes, w, e in zip((4, 8, 16, 32, 64), r.ms_width, r.ms_lanes_emit)}
            assert r.seg_lanes == 8 or times[r.seg_lanes] < 0.97 * times[8]
        else:
            assert all(x == 0 for x in r.ms_width) and all(x == 0 for x in r.ms_lanes_emit) and r.seg_lanes == 8
        seeds, gains, rep = e.run(dg, model, 30, 0.5, 1.0, 3)
        want = oracle.tim_run(g, model, 30, 0.5, 1.0, 3)
        assert np.array_equal(seeds, want["seeds"]) and np.array_equal(gains, want["gains"])
        assert rep.select.theta == want["theta"] and rep.select.nodes == want["ns_nodes"]


def test_autotune_rejects_bad_sizes():
    import paper_1404_0900_amd as tim
    g = synth.config_graph("cfg1")
    with tim.Engine(0) as e:
        dg = e.upload(g)
        with pytest.raises(tim.TimError):
            e.autotune(dg, IC, 100)
