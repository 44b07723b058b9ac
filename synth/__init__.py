"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

Only input data is produced here: graphs as canonical in-edge CSR arrays
(int64 offsets, int32 sources sorted by (dst, src)), small hand-made graphs,
and per-edge threshold arrays drawn at random.  Nothing here computes RR sets,
coins, widths or any other step of the influence-maximisation method.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build() -> str:
    """Compile the Chung-Lu generator into synth/libsynth.so (gcc)."""
    src = os.path.join(_HERE, "chunglu.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_chung_lu.restype = ctypes.c_int
        lib.synth_chung_lu.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_set_verbose.restype = None
        lib.synth_set_verbose.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """In-edge CSR of a directed graph: in-edges of v are src[off[v]:off[v+1]]."""
    n: int
    m: int
    off: np.ndarray  # int64[n+1]
    src: np.ndarray  # int32[m]
    name: str = ""

    def indeg(self) -> np.ndarray:
        return np.diff(self.off)


def chung_lu(n: int, m: int, alpha: float = 2.1, seed: int = 1, name: str = "") -> Graph:
    """Directed Chung-Lu power-law graph with exactly m distinct edges, no self-loops."""
    lib = _load()
    lib.synth_set_verbose(1 if m >= 100_000_000 else 0)  # progress lines on stderr for large graphs
    off = np.empty(n + 1, dtype=np.int64)
    src = np.empty(m, dtype=np.int32)
    i0 = ctypes.c_int64(0)
    rc = lib.synth_chung_lu(n, m, float(alpha), seed & 0xFFFFFFFFFFFFFFFF, off.ctypes.data, src.ctypes.data,
                            ctypes.byref(i0))
    if rc != 0:
        raise RuntimeError(f"synth_chung_lu(n={n}, m={m}) failed with code {rc}")
    return Graph(n, m, off, src, name or f"chunglu_n{n}_m{m}_s{seed}")


def from_edges(n: int, edges, name: str = "") -> Graph:
    """Canonical in-CSR from a list of directed (u, v) edges; rejects self-loops and repeats."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("node id out of range")
    if np.any(e[:, 0] == e[:, 1]):
        raise ValueError("self-loop")
    order = np.lexsort((e[:, 0], e[:, 1]))
    e = e[order]
    if len(e) > 1 and np.any(np.all(e[1:] == e[:-1], axis=1)):
        raise ValueError("repeated edge")
    off = np.zeros(n + 1, dtype=np.int64)
    np.add.at(off, e[:, 1] + 1, 1)
    off = np.cumsum(off).astype(np.int64)
    return Graph(n, len(e), off, e[:, 0].astype(np.int32).copy(), name)


def edge_list(g: Graph) -> np.ndarray:
    """(m, 2) array of (src, dst) in CSR order."""
    dst = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.off))
    return np.stack([g.src.astype(np.int64), dst], axis=1)


def random_thresholds(m: int, seed: int, choices=None) -> np.ndarray:
    """Per-edge uint32 thresholds drawn from `choices` (or uniformly over uint32)."""
    rng = np.random.default_rng(seed)
    if choices is None:
        return rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32)
    c = np.asarray(choices, dtype=np.uint32)
    return c[rng.integers(0, len(c), size=m)]


def random_lt_thresholds(g: Graph, seed: int, total=None) -> np.ndarray:
    """LT in-weights drawn at random and normalized per node, as uint32 cumulative thresholds.

    Every in-edge of v gets an integer weight uniform in [1, 2^16]; with S_j the sum of the first j+1
    weights of v's list (CSR order) and S the sum of all of them, t_j = floor(S_j * 2^32 / S) - 1
    (exact integer arithmetic; the last is 2^32 - 1, so the weights sum to 1), clamped to >= 0.
    `total` (a float in (0, 1], or None for 1) scales the cumulative weights so that they sum to
    `total` instead: the walk then stops at v with probability about 1 - total.
    """
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 2**16 + 1, size=g.m, dtype=np.uint64)
    cum = np.cumsum(w, dtype=np.uint64)
    indeg = np.diff(g.off)
    first = np.repeat(g.off[:-1], indeg)  # first edge of each edge's node
    before = np.where(first > 0, cum[np.maximum(first - 1, 0)], 0).astype(np.uint64)
    s_j = cum - before  # prefix within the node's list, <= 2^16 * indeg < 2^48
    last = (g.off[1:] - 1)[indeg > 0]
    s_tot = np.zeros(g.n, dtype=np.uint64)
    s_tot[indeg > 0] = cum[last] - np.where(g.off[:-1][indeg > 0] > 0,
                                            cum[np.maximum(g.off[:-1][indeg > 0] - 1, 0)], 0)
    den = np.repeat(s_tot, indeg)
    if total is not None:  # scale the numerator by total in 2^-16 steps
        s_j = (s_j * np.uint64(int(round(total * 65536)))) >> np.uint64(16)
    # floor(s_j * 2^32 / den) in two 16-bit steps (no product exceeds 2^64)
    hi = (s_j << np.uint64(16)) // den
    rem = (s_j << np.uint64(16)) % den
    q = (hi << np.uint64(16)) + ((rem << np.uint64(16)) // den)
    t = q.astype(np.int64) - 1
    return np.clip(t, 0, 0xFFFFFFFF).astype(np.uint32)


@dataclass
class Triggering:
    """An explicit triggering distribution per node (general triggering model, Section 4.2): the outcomes of v
    are j in [toff[v], toff[v+1]) with uint32 cumulative thresholds tthr[j] (t_j = floor(C_j * 2^32) - 1 for
    the cumulative probability C_j), and outcome j's triggering set is the in-edges off[v] + tmem[i] for i in
    [tset[j], tset[j+1]) (local in-edge indices, increasing).  Probability left over is the empty set."""
    toff: np.ndarray  # int64[n+1]
    tthr: np.ndarray  # uint32[J]
    tset: np.ndarray  # int64[J+1]
    tmem: np.ndarray  # uint32[total]


def random_triggering(g: Graph, seed: int, max_outcomes: int = 4, max_size: int = 3, mass=(0.3, 0.8),
                      p_full: float = 0.25) -> Triggering:
    """A random triggering distribution for every node of g.

    A node of in-degree d >= 1 gets 1..max_outcomes outcomes (uniform); each outcome is a uniformly drawn
    subset of 1..min(d, max_size) of its in-edges (outcomes may repeat a subset).  Outcome weights are
    integers uniform in [1, 2^16]; the node's total probability F / 2^16 is 1 with probability p_full,
    else F is uniform in [mass[0] * 2^16, mass[1] * 2^16].  With S_j the sum of the first j+1 weights and
    S their sum, t_j = floor(S_j * F * 2^16 / S) - 1 in exact integers (clamped to >= 0)."""
    rng = np.random.default_rng(seed)
    d = np.diff(g.off).astype(np.int64)
    nout = np.where(d > 0, rng.integers(1, max_outcomes + 1, size=g.n), 0).astype(np.int64)
    toff = np.zeros(g.n + 1, dtype=np.int64)
    toff[1:] = np.cumsum(nout)
    J = int(toff[-1])
    od = np.repeat(d, nout)  # in-degree of each outcome's node
    size = 1 + (rng.integers(0, 2**31, size=J) % np.minimum(od, max_size))
    # up to max_size distinct local indices per outcome: draw c-th pick uniformly among the od - c
    # indices not taken yet (skip past the taken ones in increasing order)
    big = np.iinfo(np.int64).max
    picks = np.full((J, max_size), big, dtype=np.int64)
    r = rng.integers(0, 2**62, size=(J, max_size))
    for c in range(max_size):
        x = r[:, c] % np.maximum(od - c, 1)
        taken = np.sort(picks[:, :c], axis=1)
        for t in range(c):
            x = np.where(x >= taken[:, t], x + 1, x)
        picks[:, c] = np.where(c < size, x, big)
    keep = np.arange(max_size)[None, :] < size[:, None]
    picks.sort(axis=1)
    tset = np.zeros(J + 1, dtype=np.int64)
    tset[1:] = np.cumsum(size)
    tmem = picks[keep].astype(np.uint32) if J else np.zeros(0, dtype=np.uint32)
    # cumulative thresholds (S_j * F * 2^16 < 2^(16 + log2(max_outcomes)) * 2^32: exact in int64 up to 2^14
    # outcomes per node)
    assert max_outcomes <= 2**14
    w = rng.integers(1, 2**16 + 1, size=J).astype(np.int64)
    full = rng.random(g.n) < p_full
    F = np.where(full, 2**16, rng.integers(int(mass[0] * 2**16), int(mass[1] * 2**16) + 1, size=g.n)).astype(np.int64)
    cum = np.cumsum(w)
    first = np.repeat(toff[:-1], nout)  # first outcome of each outcome's node
    before = np.where(first > 0, cum[np.maximum(first - 1, 0)], 0)
    s_j = cum - before
    S = np.repeat(np.where(nout > 0, cum[np.maximum(toff[1:] - 1, 0)] - np.where(toff[:-1] > 0,
                                                                                  cum[np.maximum(toff[:-1] - 1, 0)],
                                                                                  0), 1), nout)
    Fo = np.repeat(F, nout)
    tthr = np.maximum((s_j * Fo * 2**16) // S - 1, 0).astype(np.uint32)
    return Triggering(toff, tthr, tset, tmem)


def random_small_graph(n: int, m: int, seed: int) -> Graph:
    """Uniform random simple digraph with exactly m edges (tiny sizes, for exhaustive tests)."""
    rng = np.random.default_rng(seed)
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    pick = rng.choice(len(pairs), size=m, replace=False)
    return from_edges(n, [pairs[i] for i in pick], name=f"small_n{n}_m{m}_s{seed}")


# Trivalency edge probabilities: IC where each edge's p is one of three values.
TRIVALENCY_P = (0.1, 0.01, 0.001)


def threshold_of(p: float) -> int:
    """uint32 threshold t = floor(p * 2^32) - 1 of an edge probability p in (0, 1] (exact in p's binary value)."""
    from fractions import Fraction
    t = int(Fraction(p) * 2**32) - 1
    if not 0 <= t <= 0xFFFFFFFF:
        raise ValueError(f"p={p} has no uint32 threshold")
    return t


def batch_queries(count: int = 64, base_seed: int = 1000, n_range=(10_000, 2_000_000), deg_range=(4.0, 40.0),
                  k_max: int = 50, eps_choices=(0.1, 0.2, 0.5)) -> list:
    """Parameters of a batch of independent TIM+ queries, each on a graph of its own.

    Query j draws from numpy's default_rng(base_seed + j), in this order: n log-uniform in n_range
    (rounded), the average degree uniform in deg_range (m = round(n * degree)), k uniform in
    [1, k_max], eps from eps_choices.  Even j use IC with per-edge probabilities drawn uniformly from
    TRIVALENCY_P (thresholds seeded with base_seed + j), odd j LT with in-weights 1/indeg.  The graph is
    the directed Chung-Lu graph (alpha 2.1) seeded with base_seed + j; ell = 1; the algorithm seed is
    base_seed + j.
    """
    import math
    out = []
    for j in range(count):
        r = np.random.default_rng(base_seed + j)
        n = int(round(math.exp(r.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        deg = float(r.uniform(deg_range[0], deg_range[1]))
        m = int(round(n * deg))
        k = int(r.integers(1, k_max + 1))
        eps = float(r.choice(np.asarray(eps_choices, dtype=np.float64)))
        model = 0 if j % 2 == 0 else 1
        out.append(dict(name=f"q{j}", n=n, m=m, alpha=2.1, graph_seed=base_seed + j, model=model, k=k, eps=eps,
                        ell=1.0, seed=base_seed + j, thr_seed=(base_seed + j) if model == 0 else None))
    return out


def batch_graph(q: dict):
    """(Graph, thresholds or None) of one query of batch_queries()."""
    g = chung_lu(q["n"], q["m"], q["alpha"], q["graph_seed"], name=q["name"])
    thr = None
    if q["thr_seed"] is not None:
        thr = random_thresholds(g.m, q["thr_seed"], choices=[threshold_of(p) for p in TRIVALENCY_P])
    return g, thr


def batch_graphs(queries, workers: int = 8) -> list:
    """batch_graph() of every query, generated by `workers` threads (the generator releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    _load()
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        return list(ex.map(batch_graph, queries))


# Serving workload: resident graphs and a seeded stream of queries arriving over time.
SERVE_GRAPHS = ((100_000, 1601), (1_000_000, 1602), (4_000_000, 1603), (10_000_000, 1604))  # (n, seed)
SERVE_DEGREE = 16


def serve_graphs(scale: float = 1.0, workers: int = 4) -> list:
    """The serving workload's resident graphs: directed Chung-Lu (alpha 2.1), average degree 16, with
    n = 10^5, 10^6, 4*10^6 and 10^7 (times `scale`, for tests), generated by `workers` threads."""
    from concurrent.futures import ThreadPoolExecutor
    _load()
    specs = [(max(1000, int(n * scale)), seed) for n, seed in SERVE_GRAPHS]
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        return list(ex.map(lambda a: chung_lu(a[0], SERVE_DEGREE * a[0], 2.1, a[1], name=f"serve_n{a[0]}"), specs))


def serve_queries(count: int, rate: float, seed: int, ngraphs: int = 4, k_max: int = 100,
                  eps_choices=(0.1, 0.2, 0.3)) -> list:
    """A seeded stream of `count` queries with Poisson arrivals at `rate` per second.

    From numpy's default_rng(seed), per query in order: the gap to the previous arrival (exponential,
    mean 1/rate; the first query arrives at its gap), the graph (uniform over ngraphs), the model (IC
    with p = 1/indeg, or LT, uniform), k uniform in [1, k_max], eps from eps_choices; ell = 1 and the
    algorithm seed is seed * 100000 + the query's index.
    """
    r = np.random.default_rng(seed)
    out, t = [], 0.0
    for i in range(count):
        t += float(r.exponential(1.0 / rate))
        out.append(dict(arrival=t, graph=int(r.integers(0, ngraphs)), model=int(r.integers(0, 2)),
                        k=int(r.integers(1, k_max + 1)), eps=float(r.choice(np.asarray(eps_choices))),
                        ell=1.0, seed=seed * 100_000 + i))
    return out


# Configurations of the synthetic workloads (graph part only).
CONFIGS = {
    "cfg1": dict(n=15_000, m=60_000, alpha=2.1, seed=1),
    "cfg2": dict(n=1_000_000, m=10_000_000, alpha=2.1, seed=2),
    "cfg5": dict(n=41_600_000, m=1_470_000_000, alpha=2.1, seed=5),
}


def config_graph(name: str) -> Graph:
    c = CONFIGS[name]
    return chung_lu(c["n"], c["m"], c["alpha"], c["seed"], name=name)
