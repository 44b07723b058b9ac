"""CPU oracle for TIM / TIM+ — test infrastructure, not part of the product.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps the plain single-threaded C implementation in
tim_oracle.c (RR sets, kappa, KptEstimation, RefineKPT, greedy NodeSelection,
TIM/TIM+) and the exhaustive checker in brute.c.  It shares no code with the
HIP path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

IC, LT, TRIGGER = 0, 1, 2
PHASE_REFINE, PHASE_SELECT = 63, 64
FLAG_PLAIN, FLAG_ELL_ADJUST = 1, 2
_MAX_ROUNDS = 64


def build() -> str:
    """Compile oracle/liboracle.so with gcc (no FMA contraction, no fast-math)."""
    srcs = [os.path.join(_HERE, f) for f in ("tim_oracle.c", "brute.c")]
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-o", tmp, *srcs, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Report(ctypes.Structure):
    _fields_ = [
        ("i_max", ctypes.c_int32), ("i_last", ctypes.c_int32), ("c_last", ctypes.c_uint64),
        ("kpt_star", ctypes.c_double),
        ("round_c", ctypes.c_uint64 * _MAX_ROUNDS),
        ("round_sum_lo", ctypes.c_uint64 * _MAX_ROUNDS), ("round_sum_hi", ctypes.c_uint64 * _MAX_ROUNDS),
        ("round_width", ctypes.c_uint64 * _MAX_ROUNDS), ("round_nodes", ctypes.c_uint64 * _MAX_ROUNDS),
        ("eps_prime", ctypes.c_double), ("lambda_prime", ctypes.c_double), ("kpt_prime", ctypes.c_double),
        ("kpt_plus", ctypes.c_double),
        ("theta_prime", ctypes.c_uint64), ("covered_prime", ctypes.c_uint64),
        ("lambda_", ctypes.c_double), ("ell_used", ctypes.c_double),
        ("theta", ctypes.c_uint64), ("ns_nodes", ctypes.c_uint64), ("ns_width", ctypes.c_uint64),
        ("ns_covered", ctypes.c_uint64),
    ]

    def round_sums(self) -> dict:
        out = {}
        last = self.i_last if self.i_last > 0 else 0
        for i in range(1, last + 1):
            out[i] = (int(self.round_sum_hi[i]) << 64) | int(self.round_sum_lo[i])
        return out

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_ if not name.startswith("round_")}
        d["lambda"] = d.pop("lambda_")
        d["round_sums"] = self.round_sums()
        d["round_c"] = {i: int(self.round_c[i]) for i in d["round_sums"]}
        d["round_width"] = {i: int(self.round_width[i]) for i in d["round_sums"]}
        d["round_nodes"] = {i: int(self.round_nodes[i]) for i in d["round_sums"]}
        return d


_P = ctypes.c_void_p
_G = [ctypes.c_int64, ctypes.c_int64, _P, _P, _P]  # n, m, off, src, thr


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "orc_philox4x32_10": (None, [_P, _P, _P]),
        "orc_draw": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, _P]),
        "orc_root": (ctypes.c_int64, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64]),
        "orc_coin_word": (ctypes.c_uint32, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64]),
        "orc_wc_threshold": (ctypes.c_uint32, [ctypes.c_int64]),
        "orc_lt_pick": (ctypes.c_int64, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64,
                                         ctypes.c_int64]),
        "orc_trig_pick": (ctypes.c_int64, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, _P,
                                           _P]),
        "orc_lt_pick_cumulative": (ctypes.c_int64, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                                    ctypes.c_int64, _P, ctypes.c_int64]),
        "orc_forward_spread": (ctypes.c_int, _G + [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                                   _P, ctypes.c_int, _P]),
        "orc_sample_sets": (ctypes.c_int64, _G + [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                                  ctypes.c_uint64, _P, _P, ctypes.c_int64, _P]),
        "orc_rr_single": (ctypes.c_int64, _G + [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, _P,
                                                _P]),
        "orc_round_sum": (ctypes.c_int, _G + [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                              ctypes.c_uint64, ctypes.c_int, _P]),
        "orc_kappa": (ctypes.c_double, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int]),
        "orc_kappa_fixed": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int]),
        "orc_ln_binom": (ctypes.c_double, [ctypes.c_int64, ctypes.c_int]),
        "orc_lambda": (ctypes.c_double, [ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
        "orc_eps_prime": (ctypes.c_double, [ctypes.c_int, ctypes.c_double, ctypes.c_double]),
        "orc_lambda_prime": (ctypes.c_double, [ctypes.c_int64, ctypes.c_double, ctypes.c_double]),
        "orc_i_max": (ctypes.c_int, [ctypes.c_int64]),
        "orc_c_i": (ctypes.c_uint64, [ctypes.c_int64, ctypes.c_double, ctypes.c_int]),
        "orc_greedy": (ctypes.c_int, [ctypes.c_int64, ctypes.c_uint64, _P, _P, ctypes.c_int, _P, _P]),
        "orc_kpt_estimate": (ctypes.c_int, _G + [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, _P]),
        "orc_refine_kpt": (ctypes.c_int, _G + [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_uint64, _P,
                                               _P]),
        "orc_node_select": (ctypes.c_int, _G + [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, _P, _P,
                                                _P]),
        "orc_tim_run": (ctypes.c_int, _G + [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_uint64, ctypes.c_uint32, _P, _P, _P, _P]),
        "orc_report_size": (ctypes.c_size_t, []),
        "brute_all_spreads": (ctypes.c_int, _G + [ctypes.c_int, _P]),
        "brute_rr_stats": (ctypes.c_int, _G + [ctypes.c_int, ctypes.c_int, _P, _P, _P, _P]),
        "brute_max_coverage": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_uint64, _P, _P, ctypes.c_int, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if lib.orc_report_size() != ctypes.sizeof(Report):
        raise RuntimeError("oracle report layout mismatch")
    _lib = lib
    return lib


class _TriggerC(ctypes.Structure):
    """orc_trigger: the explicit triggering distribution of reading R11 (model 2)."""
    _fields_ = [("toff", ctypes.c_void_p), ("tthr", ctypes.c_void_p), ("tset", ctypes.c_void_p),
                ("tmem", ctypes.c_void_p)]


class _TriggerArg:
    """A triggering distribution handed to the C code in place of a threshold array."""

    def __init__(self, t):
        arrs = [np.ascontiguousarray(t.toff, dtype=np.int64), np.ascontiguousarray(t.tthr, dtype=np.uint32),
                np.ascontiguousarray(t.tset, dtype=np.int64), np.ascontiguousarray(t.tmem, dtype=np.uint32)]
        self.arrays = tuple(a if a.size else np.zeros(1, dtype=a.dtype) for a in arrs)
        self.c = _TriggerC(*(a.ctypes.data for a in self.arrays))
        self.address = ctypes.addressof(self.c)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, _TriggerArg):
        return a.address
    return a.ctypes.data


def _garr(g, thr):
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    src = np.ascontiguousarray(g.src, dtype=np.int32)
    if thr is None:
        t = None
    elif hasattr(thr, "tmem"):  # a triggering distribution (model 2, reading R11)
        t = _TriggerArg(thr)
    else:
        t = np.ascontiguousarray(thr, dtype=np.uint32)
    return off, src, t


def _gargs(g, off, src, t):
    return [g.n, g.m, off.ctypes.data, src.ctypes.data, _ptr(t)]


# ---- random-number stream -------------------------------------------------
def philox(ctr, key) -> tuple:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return tuple(int(x) for x in o)


def draw(seed, phase, kind, idx, set_id) -> tuple:
    o = np.zeros(4, dtype=np.uint32)
    _load().orc_draw(seed, phase, kind, idx, set_id, o.ctypes.data)
    return tuple(int(x) for x in o)


def root(seed, phase, set_id, n) -> int:
    return int(_load().orc_root(seed, phase, set_id, n))


def coin_word(seed, phase, set_id, e) -> int:
    return int(_load().orc_coin_word(seed, phase, set_id, e))


def wc_threshold(d) -> int:
    return int(_load().orc_wc_threshold(d))


def lt_pick(seed, phase, set_id, v, d) -> int:
    return int(_load().orc_lt_pick(seed, phase, set_id, v, d))


def trig_pick(seed, phase, set_id, v, trig) -> int:
    """Outcome index (into trig.tthr / trig.tset) that node v draws under reading R11, or -1 (empty set)."""
    a = _TriggerArg(trig)
    return int(_load().orc_trig_pick(seed, phase, set_id, v, a.arrays[0].ctypes.data, a.arrays[1].ctypes.data))


def lt_pick_cumulative(seed, phase, set_id, v, t) -> int:
    """In-edge index the LT walk takes at v under cumulative thresholds t (uint32 over v's in-edges), or -1."""
    t = np.ascontiguousarray(t, dtype=np.uint32)
    return int(_load().orc_lt_pick_cumulative(seed, phase, set_id, v, t.ctypes.data, len(t)))


# ---- spread evaluation -----------------------------------------------------
PHASE_EVAL = 65


def forward_spread(g, model, seed, first, count, seeds, thr=None) -> np.ndarray:
    """Spread of `seeds` in the live-edge worlds of runs [first, first+count) (uint64 per run)."""
    off, src, t = _garr(g, thr)
    s = np.ascontiguousarray(seeds, dtype=np.int32)
    out = np.zeros(count, dtype=np.uint64)
    rc = _load().orc_forward_spread(*_gargs(g, off, src, t), model, seed, first, count, s.ctypes.data, len(s),
                                     out.ctypes.data)
    if rc:
        raise RuntimeError(f"orc_forward_spread failed ({rc})")
    return out


# ---- RR sets ---------------------------------------------------------------
def sample_sets(g, model, seed, phase, first, count, thr=None, cap=None):
    """Sets [first, first+count): (set_off int64[count+1], nodes int32 sorted per set, widths uint64[count])."""
    off, src, t = _garr(g, thr)
    cap = cap or max(1024, count * 64)
    while True:
        so = np.zeros(count + 1, dtype=np.int64)
        nodes = np.zeros(cap, dtype=np.int32)
        widths = np.zeros(max(count, 1), dtype=np.uint64)
        r = _load().orc_sample_sets(*_gargs(g, off, src, t), model, seed, phase, first, count, so.ctypes.data,
                                    nodes.ctypes.data, cap, widths.ctypes.data)
        if r == -1:
            cap *= 4
            continue
        if r < 0:
            raise RuntimeError("orc_sample_sets failed")
        return so, nodes[:r].copy(), widths[:count].copy()


def rr_set(g, model, seed, phase, set_id, thr=None):
    """One RR set: (sorted node array, width)."""
    off, src, t = _garr(g, thr)
    nodes = np.zeros(g.n, dtype=np.int32)
    w = ctypes.c_uint64(0)
    r = _load().orc_rr_single(*_gargs(g, off, src, t), model, seed, phase, set_id, nodes.ctypes.data, ctypes.byref(w))
    if r < 0:
        raise RuntimeError("orc_rr_single failed")
    return nodes[:r].copy(), int(w.value)


# ---- kappa and scalars -----------------------------------------------------
def round_sum(g, model, seed, phase, first, count, k, thr=None) -> dict:
    """One KptEstimation round over set ids [first, first+count) (Algorithm 2; Equation (8)):
    exact sum S of kappa(R) * 2^53, total width and total size."""
    lib = _load()
    off, src, t = _garr(g, thr)
    out = np.zeros(4, dtype=np.uint64)
    rc = lib.orc_round_sum(*_gargs(g, off, src, t), model, seed, phase, first, count, k, _ptr(out))
    if rc != 0:
        raise RuntimeError(f"orc_round_sum failed ({rc})")
    return dict(sum=(int(out[1]) << 64) | int(out[0]), width=int(out[2]), nodes=int(out[3]))


def kappa(w, m, k) -> float:
    return float(_load().orc_kappa(w, m, k))


def kappa_fixed(w, m, k) -> int:
    return int(_load().orc_kappa_fixed(w, m, k))


def ln_binom(n, k) -> float:
    return float(_load().orc_ln_binom(n, k))


def lam(n, k, eps, ell) -> float:
    return float(_load().orc_lambda(n, k, eps, ell))


def eps_prime(k, eps, ell) -> float:
    return float(_load().orc_eps_prime(k, eps, ell))


def lambda_prime(n, eps_p, ell) -> float:
    return float(_load().orc_lambda_prime(n, eps_p, ell))


def i_max(n) -> int:
    return int(_load().orc_i_max(n))


def c_i(n, ell, i) -> int:
    return int(_load().orc_c_i(n, ell, i))


# ---- greedy and the phases -------------------------------------------------
def greedy(n, set_off, set_nodes, k):
    so = np.ascontiguousarray(set_off, dtype=np.int64)
    sn = np.ascontiguousarray(set_nodes, dtype=np.int32)
    if sn.size == 0:
        sn = np.zeros(1, dtype=np.int32)
    seeds = np.zeros(k, dtype=np.int32)
    gains = np.zeros(k, dtype=np.uint64)
    rc = _load().orc_greedy(n, len(so) - 1, so.ctypes.data, sn.ctypes.data, k, seeds.ctypes.data, gains.ctypes.data)
    if rc:
        raise RuntimeError(f"orc_greedy failed ({rc})")
    return seeds, gains


def kpt_estimate(g, model, seed, k, ell, thr=None) -> dict:
    off, src, t = _garr(g, thr)
    rep = Report()
    rc = _load().orc_kpt_estimate(*_gargs(g, off, src, t), model, seed, k, ell, ctypes.byref(rep))
    if rc:
        raise RuntimeError(f"orc_kpt_estimate failed ({rc})")
    return rep.as_dict()


def refine_kpt(g, model, seed, k, eps, ell, kpt_star, i_last, c_last, thr=None):
    off, src, t = _garr(g, thr)
    rep = Report()
    sp = np.zeros(k, dtype=np.int32)
    rc = _load().orc_refine_kpt(*_gargs(g, off, src, t), model, seed, k, eps, ell, kpt_star, i_last, c_last,
                                sp.ctypes.data, ctypes.byref(rep))
    if rc:
        raise RuntimeError(f"orc_refine_kpt failed ({rc})")
    d = rep.as_dict()
    d["s_prime"] = sp
    return d


def node_select(g, model, seed, k, theta, thr=None):
    off, src, t = _garr(g, thr)
    rep = Report()
    seeds = np.zeros(k, dtype=np.int32)
    gains = np.zeros(k, dtype=np.uint64)
    rc = _load().orc_node_select(*_gargs(g, off, src, t), model, seed, k, theta, seeds.ctypes.data, gains.ctypes.data,
                                 ctypes.byref(rep))
    if rc:
        raise RuntimeError(f"orc_node_select failed ({rc})")
    d = rep.as_dict()
    d["seeds"], d["gains"] = seeds, gains
    return d


def tim_run(g, model, k, eps, ell, seed, flags=0, thr=None) -> dict:
    off, src, t = _garr(g, thr)
    rep = Report()
    seeds = np.zeros(k, dtype=np.int32)
    gains = np.zeros(k, dtype=np.uint64)
    sp = np.zeros(k, dtype=np.int32)
    rc = _load().orc_tim_run(*_gargs(g, off, src, t), model, k, eps, ell, seed, flags, seeds.ctypes.data,
                             gains.ctypes.data, sp.ctypes.data, ctypes.byref(rep))
    if rc:
        raise RuntimeError(f"orc_tim_run failed ({rc})")
    d = rep.as_dict()
    d["seeds"], d["gains"], d["s_prime"] = seeds, gains, sp
    return d


# ---- exhaustive checker ----------------------------------------------------
def brute_all_spreads(g, model, thr=None) -> np.ndarray:
    """E[I(S)] for every S (index = bit mask of S), by enumerating live-edge worlds."""
    off, src, t = _garr(g, thr)
    out = np.zeros(1 << g.n, dtype=np.float64)
    rc = _load().brute_all_spreads(*_gargs(g, off, src, t), model, out.ctypes.data)
    if rc:
        raise RuntimeError(f"brute_all_spreads failed ({rc})")
    return out


def brute_rr_stats(g, model, k, thr=None) -> dict:
    """Exact Pr[u in R], E[w(R)], E[kappa(R)], E[|R|] of a random RR set."""
    off, src, t = _garr(g, thr)
    p_in = np.zeros(g.n, dtype=np.float64)
    ew, ek, es = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = _load().brute_rr_stats(*_gargs(g, off, src, t), model, k, p_in.ctypes.data, ctypes.byref(ew),
                                ctypes.byref(ek), ctypes.byref(es))
    if rc:
        raise RuntimeError(f"brute_rr_stats failed ({rc})")
    return dict(p_in=p_in, ept=ew.value, ekappa=ek.value, esize=es.value)


def brute_max_coverage(n, set_off, set_nodes, k):
    so = np.ascontiguousarray(set_off, dtype=np.int64)
    sn = np.ascontiguousarray(set_nodes, dtype=np.int32)
    if sn.size == 0:
        sn = np.zeros(1, dtype=np.int32)
    mask = ctypes.c_uint32(0)
    r = _load().brute_max_coverage(n, len(so) - 1, so.ctypes.data, sn.ctypes.data, k, ctypes.byref(mask))
    if r < 0:
        raise RuntimeError("brute_max_coverage failed")
    return int(r), int(mask.value)
