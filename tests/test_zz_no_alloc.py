"""tim_max_coverage_noalloc (the greedy with the library's fixed work area, no
allocation) against tim_max_coverage through the C ABI: two calls in a row,
the second on a smaller collection, and the limits of the fixed area."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _collection(rng, n, nsets, maxlen):
    sets = [rng.choice(n, size=int(rng.integers(1, min(n, maxlen) + 1)), replace=False) for _ in range(nsets)]
    off = np.zeros(nsets + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(s) for s in sets])
    nodes = np.concatenate(sets).astype(np.int32) if nsets else np.zeros(0, dtype=np.int32)
    return off, nodes


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.asarray(a), dtype=dtype, device="cuda")


@pytest.fixture(scope="module")
def eng():
    import paper_1404_0900_amd as tim
    e = tim.Engine(0)
    yield e
    e.close()


def test_noalloc_greedy_equals_the_allocating_one_twice_in_a_row(eng):
    import torch
    rng = np.random.default_rng(11)
    # a large collection first, then a smaller one: the second call must not see the first's state
    for n, nsets, maxlen, k in ((200_000, 300_000, 40, 50), (3_000, 20_000, 12, 17)):
        _say(f"noalloc greedy: n={n} nsets={nsets} k={k}")
        off, nodes = _collection(rng, n, nsets, maxlen)
        d_off, d_nodes = _dev(off, torch.int64), _dev(nodes, torch.int32)
        want_s, want_g = eng.max_coverage(n, d_off, d_nodes, k)
        got_s, got_g = eng.max_coverage_noalloc(n, d_off, d_nodes, k)
        assert np.array_equal(got_s, want_s) and np.array_equal(got_g, want_g)


def test_noalloc_greedy_small_cases(eng):
    import torch
    rng = np.random.default_rng(5)
    for trial in range(12):
        n = int(rng.integers(2, 300))
        nsets = int(rng.integers(0, 2000))
        off, nodes = _collection(rng, n, nsets, 20)
        k = int(rng.integers(1, min(n, 40) + 1))
        d_off, d_nodes = _dev(off, torch.int64), _dev(nodes, torch.int32)
        want = eng.max_coverage(n, d_off, d_nodes, k)
        got = eng.max_coverage_noalloc(n, d_off, d_nodes, k)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), trial


def test_noalloc_greedy_rejects_inputs_beyond_its_area(eng):
    import torch

    import paper_1404_0900_amd as tim
    off = _dev([0, 1], torch.int64)
    nodes = _dev([0], torch.int32)
    with pytest.raises(tim.TimError):
        eng.max_coverage_noalloc((1 << 20) + 1, off, nodes, 1)   # n above 2^20
    with pytest.raises(tim.TimError):
        eng.max_coverage_noalloc(2000, off, nodes, 1025)         # k above 1024
    with pytest.raises(tim.TimError):
        eng.max_coverage_noalloc(3, _dev([0, 2], torch.int64), _dev([0, 5], torch.int32), 1)  # id out of range
    # still usable afterwards
    s, g = eng.max_coverage_noalloc(4, _dev([0, 2, 3, 4, 5], torch.int64), _dev([0, 3, 1, 2, 3], torch.int32), 1)
    assert list(s) == [3] and list(g) == [2]
