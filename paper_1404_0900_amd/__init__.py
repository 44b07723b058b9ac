"""Python binding of libtim.so — the MI355X (gfx950) TIM / TIM+ engine.

Argument marshalling only: every RR set, kappa sum, index and greedy step is
computed by the HIP kernels behind the C ABI of include/tim.h.  PyTorch
provides device memory (output tensors) and the stream.  Importing works
without a GPU; constructing an Engine needs the built library and a GPU and
raises if either is missing (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtim.so")

IC, LT, TRIGGER = 0, 1, 2
PHASE_REFINE, PHASE_SELECT = 63, 64
FLAG_PLAIN, FLAG_ELL_ADJUST = 1, 2
MAX_ROUNDS = 64

OK, EINVAL, ENOMEM, EBUDGET, EDEVICE, ECAPACITY = range(6)
_STATUS = {1: "TIM_EINVAL", 2: "TIM_ENOMEM", 3: "TIM_EBUDGET", 4: "TIM_EDEVICE", 5: "TIM_ECAPACITY"}

EXPORTED = ("tim_ctx_create", "tim_ctx_destroy", "tim_last_error", "tim_ctx_device_bytes", "tim_set_resident_limit",
            "tim_graph_upload", "tim_graph_set_lt_weights", "tim_graph_set_triggering",
            "tim_graph_free", "tim_sample_rr", "tim_sample_widths", "tim_sample_cover", "tim_max_coverage",
            "tim_max_coverage_noalloc",
            "tim_kpt_estimate", "tim_refine_kpt", "tim_node_select", "tim_run", "tim_profile_enable",
            "tim_profile_read", "tim_autotune", "tim_spread_mc", "tim_run_batch", "tim_autotune_batch", "tim_server_start", "tim_server_submit", "tim_server_wait",
            "tim_server_stop")

U64, I64, U32, I32, DBL, P = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_double,
                              ctypes.c_void_p)


class TimError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class BatchStats(ctypes.Structure):
    _fields_ = [("count", U64), ("kappa_sum_lo", U64), ("kappa_sum_hi", U64), ("width_sum", U64),
                ("node_sum", U64), ("covered", U64), ("deferred", U64)]

    @property
    def kappa_sum(self) -> int:
        return (int(self.kappa_sum_hi) << 64) | int(self.kappa_sum_lo)


class KptResult(ctypes.Structure):
    _fields_ = [("i_max", I32), ("i_last", I32), ("c_last", U64), ("kpt_star", DBL),
                ("round_c", U64 * MAX_ROUNDS), ("round_sum_lo", U64 * MAX_ROUNDS), ("round_sum_hi", U64 * MAX_ROUNDS),
                ("round_width", U64 * MAX_ROUNDS), ("round_nodes", U64 * MAX_ROUNDS)]

    def round_sums(self) -> dict:
        return {i: (int(self.round_sum_hi[i]) << 64) | int(self.round_sum_lo[i]) for i in range(1, self.i_last + 1)}


class RefineResult(ctypes.Structure):
    _fields_ = [("eps_prime", DBL), ("lambda_prime", DBL), ("theta_prime", U64), ("covered_prime", U64),
                ("kpt_prime", DBL), ("kpt_plus", DBL)]


class SelectResult(ctypes.Structure):
    _fields_ = [("theta", U64), ("nodes", U64), ("width", U64), ("covered", U64), ("store_bytes", U64),
                ("resident_sets", U64), ("chunk_sets", U64), ("regenerated_sets", U64)]


class Report(ctypes.Structure):
    _fields_ = [("ell_used", DBL), ("lambda_", DBL), ("kpt", KptResult), ("refine", RefineResult),
                ("select", SelectResult), ("s_prime", I32 * 128),
                ("ms_kpt", DBL), ("ms_refine", DBL), ("ms_select_sample", DBL), ("ms_select_index", DBL),
                ("ms_select_greedy", DBL), ("ms_total", DBL), ("sets_total", U64), ("width_total", U64)]


class TuneResult(ctypes.Structure):
    _fields_ = [("seg_lanes", I32), ("slice_cap", U32), ("ms_width", DBL * 5), ("ms_emit", DBL * 4), ("ms_lanes_emit", DBL * 5)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("launches", U64), ("kernel_ms", DBL), ("sets", U64), ("nodes", U64), ("edges", U64),
                ("bytes", U64), ("large_launches", U64), ("large_ms", DBL), ("deferred", U64)]


class Profile(ctypes.Structure):
    _fields_ = [("sampler", (KernelProfile * 3) * 2), ("index_calls", U64), ("index_ms", DBL), ("greedy_ms", DBL),
                ("ic_wide", KernelProfile * 3), ("grouped", KernelProfile * 2)]


class Query(ctypes.Structure):
    _fields_ = [("graph", P), ("model", ctypes.c_int), ("k", ctypes.c_int), ("eps", DBL), ("ell", DBL),
                ("seed", U64), ("flags", U32), ("seeds", P), ("gains", P), ("report", P), ("status", ctypes.c_int)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("rounds", U64), ("jobs", U64), ("launches", U64), ("max_jobs", U64), ("workers", U64),
                ("budget_bytes", U64), ("member_budget_bytes", U64), ("ms_wall", DBL), ("ms_kpt", DBL),
                ("kpt_job_cap", U64), ("kpt_steps", U64), ("kpt_graph_launches", U64),
                ("rr_pool_bytes", U64), ("rr_peak_bytes", U64), ("held_queries", U64), ("held_ms", DBL)]


class BatchTune(ctypes.Structure):
    _fields_ = [("job_cap", U64), ("caps", U64 * 4), ("ms_kpt", DBL * 4)]


MODE_NAMES = ("widths", "store", "cover")
MODEL_NAMES = ("ic", "lt")

_lib = None


def load_library():
    """Loads libtim.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1404_0900_amd/build.py "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "tim_ctx_create": (ctypes.c_int, [ctypes.c_int, P, U64, ctypes.POINTER(P)]),
        "tim_ctx_destroy": (None, [P]),
        "tim_last_error": (ctypes.c_char_p, []),
        "tim_ctx_device_bytes": (U64, [P]),
        "tim_set_resident_limit": (ctypes.c_int, [P, U64]),
        "tim_graph_upload": (ctypes.c_int, [P, I64, I64, P, P, P, ctypes.POINTER(P)]),
        "tim_graph_free": (None, [P]),
        "tim_graph_set_lt_weights": (ctypes.c_int, [P, P, P, P]),
        "tim_graph_set_triggering": (ctypes.c_int, [P, P, P, P, P, P, P]),
        "tim_sample_rr": (ctypes.c_int, [P, P, ctypes.c_int, U64, U32, U64, U64, P, P, U64, P,
                                         ctypes.POINTER(U64), ctypes.POINTER(BatchStats)]),
        "tim_sample_widths": (ctypes.c_int, [P, P, ctypes.c_int, U64, U32, U64, U64, ctypes.c_int, P, P,
                                             ctypes.POINTER(BatchStats)]),
        "tim_sample_cover": (ctypes.c_int, [P, P, ctypes.c_int, U64, U32, U64, U64, P, ctypes.c_int,
                                            ctypes.POINTER(BatchStats)]),
        "tim_max_coverage": (ctypes.c_int, [P, I64, U64, P, P, ctypes.c_int, P, P]),
        "tim_max_coverage_noalloc": (ctypes.c_int, [P, I64, U64, P, P, ctypes.c_int, P, P]),
        "tim_kpt_estimate": (ctypes.c_int, [P, P, ctypes.c_int, U64, ctypes.c_int, DBL, ctypes.POINTER(KptResult)]),
        "tim_refine_kpt": (ctypes.c_int, [P, P, ctypes.c_int, U64, ctypes.c_int, DBL, DBL, DBL, ctypes.c_int, U64, P,
                                          ctypes.POINTER(RefineResult)]),
        "tim_node_select": (ctypes.c_int, [P, P, ctypes.c_int, U64, ctypes.c_int, U64, P, P,
                                           ctypes.POINTER(SelectResult)]),
        "tim_run": (ctypes.c_int, [P, P, ctypes.c_int, ctypes.c_int, DBL, DBL, U64, U32, P, P,
                                   ctypes.POINTER(Report)]),
        "tim_profile_enable": (ctypes.c_int, [P, ctypes.c_int]),
        "tim_profile_read": (ctypes.c_int, [P, ctypes.POINTER(Profile)]),
        "tim_autotune": (ctypes.c_int, [P, P, ctypes.c_int, U64, ctypes.POINTER(TuneResult)]),
        "tim_spread_mc": (ctypes.c_int, [P, P, ctypes.c_int, U64, U64, U64, P, ctypes.c_int, P,
                                         ctypes.POINTER(DBL), ctypes.POINTER(U64)]),
        "tim_run_batch": (ctypes.c_int, [P, ctypes.POINTER(Query), ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(BatchInfo)]),
        "tim_autotune_batch": (ctypes.c_int, [P, ctypes.POINTER(Query), ctypes.c_int, ctypes.POINTER(BatchTune)]),
        "tim_server_start": (ctypes.c_int, [P, ctypes.c_int, ctypes.POINTER(P)]),
        "tim_server_submit": (ctypes.c_int, [P, ctypes.POINTER(Query), ctypes.POINTER(U64)]),
        "tim_server_wait": (ctypes.c_int, [P, U64, ctypes.POINTER(DBL)]),
        "tim_server_stop": (ctypes.c_int, [P, ctypes.POINTER(BatchInfo)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st):
    if st != OK:
        raise TimError(st, load_library().tim_last_error().decode())


def _np_ptr(a):
    return None if a is None else a.ctypes.data


def _dev_ptr(t):
    return None if t is None else t.data_ptr()


@dataclass
class DeviceGraph:
    handle: int
    n: int
    m: int
    weighted_cascade: bool


class Engine:
    """A context on one GPU (one per thread); frees its device memory on close()."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm GPU visible: the TIM engine runs only on the GPU")
        self._torch = torch
        self.lib = load_library()
        self.device = device
        torch.cuda.set_device(device)
        stream = torch.cuda.current_stream(device).cuda_stream
        h = P()
        _check(self.lib.tim_ctx_create(device, stream or None, budget_bytes, ctypes.byref(h)))
        self.ctx = h.value
        self._graphs = []

    # ---- lifetime ----
    def close(self):
        if getattr(self, "ctx", None):
            for g in self._graphs:
                self.lib.tim_graph_free(g.handle)
            self._graphs = []
            self.lib.tim_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def device_bytes(self) -> int:
        return int(self.lib.tim_ctx_device_bytes(self.ctx))

    def set_resident_limit(self, max_sets: int | None):
        """Most RR sets a greedy keeps resident (None: no limit); the rest is regenerated in chunks."""
        _check(self.lib.tim_set_resident_limit(self.ctx, (1 << 64) - 1 if max_sets is None else int(max_sets)))

    def profile(self, on: bool = True):
        """Turns per-kernel timing on/off and clears the counters."""
        _check(self.lib.tim_profile_enable(self.ctx, 1 if on else 0))

    def read_profile(self) -> Profile:
        p = Profile()
        _check(self.lib.tim_profile_read(self.ctx, ctypes.byref(p)))
        return p

    def _sync_torch(self):
        self._torch.cuda.current_stream(self.device).synchronize()

    # ---- graph ----
    def upload(self, graph, thr=None) -> DeviceGraph:
        off = np.ascontiguousarray(graph.off, dtype=np.int64)
        src = np.ascontiguousarray(graph.src, dtype=np.int32)
        t = None if thr is None else np.ascontiguousarray(thr, dtype=np.uint32)
        h = P()
        _check(self.lib.tim_graph_upload(self.ctx, graph.n, graph.m, off.ctypes.data, src.ctypes.data, _np_ptr(t),
                                         ctypes.byref(h)))
        g = DeviceGraph(h.value, graph.n, graph.m, thr is None)
        self._graphs.append(g)
        return g

    def set_lt_weights(self, g: DeviceGraph, graph, lt_thr):
        """LT in-weights of g as uint32 cumulative thresholds per edge (None: back to 1/indeg)."""
        off = np.ascontiguousarray(graph.off, dtype=np.int64)
        t = None if lt_thr is None else np.ascontiguousarray(lt_thr, dtype=np.uint32)
        _check(self.lib.tim_graph_set_lt_weights(self.ctx, g.handle, _np_ptr(t), off.ctypes.data))

    def set_triggering(self, g: DeviceGraph, graph, trig):
        """The general triggering model's distribution of every node of g (toff, tthr, tset, tmem arrays as in
        include/tim.h), or None to remove it."""
        off = np.ascontiguousarray(graph.off, dtype=np.int64)
        if trig is None:
            _check(self.lib.tim_graph_set_triggering(self.ctx, g.handle, None, None, None, None, off.ctypes.data))
            return
        arrs = [np.ascontiguousarray(trig.toff, dtype=np.int64), np.ascontiguousarray(trig.tthr, dtype=np.uint32),
                np.ascontiguousarray(trig.tset, dtype=np.int64), np.ascontiguousarray(trig.tmem, dtype=np.uint32)]
        arrs = [a if a.size else np.zeros(1, dtype=a.dtype) for a in arrs]
        _check(self.lib.tim_graph_set_triggering(self.ctx, g.handle, *(a.ctypes.data for a in arrs),
                                                 off.ctypes.data))

    def free(self, g: DeviceGraph):
        self.lib.tim_graph_free(g.handle)
        self._graphs.remove(g)

    # ---- RR sets ----
    def sample_rr(self, g: DeviceGraph, model: int, seed: int, phase: int, first: int, count: int,
                  with_widths: bool = True, capacity: int | None = None):
        """Sets [first, first+count): (set_off int64[count+1], nodes int32, widths int64[count]) on the GPU."""
        torch = self._torch
        dev = torch.device("cuda", self.device)
        set_off = torch.empty(count + 1, dtype=torch.int64, device=dev)
        widths = torch.empty(max(count, 1), dtype=torch.int64, device=dev) if with_widths else None
        cap = capacity if capacity is not None else max(1024, 16 * count)
        nodes = torch.empty(cap, dtype=torch.int32, device=dev)
        total = U64(0)
        st = BatchStats()
        self._sync_torch()
        rc = self.lib.tim_sample_rr(self.ctx, g.handle, model, seed, phase, first, count, _dev_ptr(set_off),
                                    _dev_ptr(nodes), cap, _dev_ptr(widths), ctypes.byref(total), ctypes.byref(st))
        if rc == ECAPACITY:
            cap = int(total.value)
            nodes = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            rc = self.lib.tim_sample_rr(self.ctx, g.handle, model, seed, phase, first, count, _dev_ptr(set_off),
                                        _dev_ptr(nodes), cap, _dev_ptr(widths), ctypes.byref(total),
                                        ctypes.byref(st))
        _check(rc)
        return set_off, nodes[: int(total.value)], (widths[:count] if widths is not None else None), st

    def sample_widths(self, g: DeviceGraph, model: int, seed: int, phase: int, first: int, count: int, k: int,
                      per_set: bool = True):
        torch = self._torch
        dev = torch.device("cuda", self.device)
        widths = torch.empty(max(count, 1), dtype=torch.int64, device=dev) if per_set else None
        sizes = torch.empty(max(count, 1), dtype=torch.int32, device=dev) if per_set else None
        st = BatchStats()
        self._sync_torch()
        _check(self.lib.tim_sample_widths(self.ctx, g.handle, model, seed, phase, first, count, k, _dev_ptr(widths),
                                          _dev_ptr(sizes), ctypes.byref(st)))
        if per_set:
            return widths[:count], sizes[:count], st
        return None, None, st

    def sample_cover(self, g: DeviceGraph, model: int, seed: int, phase: int, first: int, count: int, seeds):
        s = np.ascontiguousarray(seeds, dtype=np.int32)
        st = BatchStats()
        _check(self.lib.tim_sample_cover(self.ctx, g.handle, model, seed, phase, first, count, _np_ptr(s), len(s),
                                         ctypes.byref(st)))
        return st

    # ---- greedy ----
    def max_coverage(self, n: int, set_off, nodes, k: int):
        """Greedy on a device CSR collection (torch tensors int64 / int32)."""
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        nsets = int(set_off.numel()) - 1
        self._sync_torch()
        _check(self.lib.tim_max_coverage(self.ctx, n, nsets, _dev_ptr(set_off), _dev_ptr(nodes) if nodes.numel() else
                                         None, k, seeds.ctypes.data, gains.ctypes.data))
        return seeds, gains

    def max_coverage_noalloc(self, n: int, set_off, nodes, k: int):
        """tim_max_coverage_noalloc: the same greedy with the library's fixed work area (no allocation)."""
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        nsets = int(set_off.numel()) - 1
        self._sync_torch()
        _check(self.lib.tim_max_coverage_noalloc(self.ctx, n, nsets, _dev_ptr(set_off),
                                                 _dev_ptr(nodes) if nodes.numel() else None, k,
                                                 seeds.ctypes.data, gains.ctypes.data))
        return seeds, gains

    # ---- phases ----
    def kpt_estimate(self, g: DeviceGraph, model: int, seed: int, k: int, ell: float) -> KptResult:
        out = KptResult()
        _check(self.lib.tim_kpt_estimate(self.ctx, g.handle, model, seed, k, ell, ctypes.byref(out)))
        return out

    def refine_kpt(self, g, model, seed, k, eps, ell, kpt_star, i_last, c_last):
        sp = np.zeros(k, dtype=np.int32)
        out = RefineResult()
        _check(self.lib.tim_refine_kpt(self.ctx, g.handle, model, seed, k, eps, ell, kpt_star, i_last, c_last,
                                       sp.ctypes.data, ctypes.byref(out)))
        return sp, out

    def node_select(self, g, model, seed, k, theta):
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        out = SelectResult()
        _check(self.lib.tim_node_select(self.ctx, g.handle, model, seed, k, theta, seeds.ctypes.data,
                                        gains.ctypes.data, ctypes.byref(out)))
        return seeds, gains, out

    def run(self, g: DeviceGraph, model: int, k: int, eps: float, ell: float, seed: int, flags: int = 0):
        """TIM+ (or TIM with FLAG_PLAIN): (seeds int32[k], gains uint64[k], Report)."""
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        rep = Report()
        _check(self.lib.tim_run(self.ctx, g.handle, model, k, eps, ell, seed, flags, seeds.ctypes.data,
                                gains.ctypes.data, ctypes.byref(rep)))
        return seeds, gains, rep

    def autotune(self, g: DeviceGraph, model: int, sets: int = 1 << 20) -> TuneResult:
        """Times the sampler shapes on g and keeps the fastest for this engine (results do not change)."""
        out = TuneResult()
        _check(self.lib.tim_autotune(self.ctx, g.handle, model, sets, ctypes.byref(out)))
        return out

    def spread(self, g: DeviceGraph, model: int, seed: int, seeds, runs: int, first: int = 0,
               per_run: bool = False):
        """E[I(S)] by forward Monte-Carlo runs: (mean, total[, spreads per run as a uint32 tensor])."""
        torch = self._torch
        s = np.ascontiguousarray(seeds, dtype=np.int32)
        counts = torch.empty(max(runs, 1), dtype=torch.int32, device=torch.device("cuda", self.device)) \
            if per_run else None
        mean, total = DBL(0.0), U64(0)
        self._sync_torch()
        _check(self.lib.tim_spread_mc(self.ctx, g.handle, model, seed, first, runs, _np_ptr(s) if len(s) else None,
                                      len(s), _dev_ptr(counts), ctypes.byref(mean), ctypes.byref(total)))
        if per_run:
            return mean.value, int(total.value), counts[:runs]
        return mean.value, int(total.value)

    def serve(self, slots: int) -> "Server":
        """Starts a request loop with `slots` queries at a time (upload the graphs first)."""
        return Server(self, slots)

    def run_batch(self, queries, max_concurrent: int = 0):
        """Runs queries [(graph, model, k, eps, ell, seed[, flags]), ...] as one batch.

        Returns ([(seeds, gains, Report) per query], BatchInfo)."""
        nq = len(queries)
        arr = (Query * max(nq, 1))()
        keep = []
        for i, q in enumerate(queries):
            g, model, k, eps, ell, seed = q[:6]
            flags = q[6] if len(q) > 6 else 0
            seeds = np.zeros(k, dtype=np.int32)
            gains = np.zeros(k, dtype=np.uint64)
            rep = Report()
            keep.append((seeds, gains, rep))
            arr[i] = Query(g.handle, model, k, eps, ell, seed, flags, seeds.ctypes.data, gains.ctypes.data,
                           ctypes.addressof(rep), 0)
        info = BatchInfo()
        _check(self.lib.tim_run_batch(self.ctx, arr, nq, max_concurrent, ctypes.byref(info)))
        return keep, info

    def autotune_batch(self, queries) -> BatchTune:
        """Times the batch's device KptEstimation with each work-queue granularity and keeps the fastest."""
        nq = len(queries)
        arr = (Query * max(nq, 1))()
        keep = []
        for i, q in enumerate(queries):
            g, model, k, eps, ell, seed = q[:6]
            flags = q[6] if len(q) > 6 else 0
            seeds = np.zeros(k, dtype=np.int32)
            keep.append(seeds)
            arr[i] = Query(g.handle, model, k, eps, ell, seed, flags, seeds.ctypes.data, None, None, 0)
        out = BatchTune()
        _check(self.lib.tim_autotune_batch(self.ctx, arr, nq, ctypes.byref(out)))
        return out


class Server:
    """A request loop on an Engine (tim_server_*): submit() queues a query, wait() returns its result."""

    def __init__(self, engine: "Engine", slots: int):
        self.engine = engine
        self.lib = engine.lib
        h = P()
        _check(self.lib.tim_server_start(engine.ctx, slots, ctypes.byref(h)))
        self.handle = h.value
        self._pending = {}

    def submit(self, g: DeviceGraph, model: int, k: int, eps: float, ell: float, seed: int, flags: int = 0) -> int:
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        rep = Report()
        q = Query(g.handle, model, k, eps, ell, seed, flags, seeds.ctypes.data, gains.ctypes.data,
                  ctypes.addressof(rep), 0)
        t = U64(0)
        _check(self.lib.tim_server_submit(self.handle, ctypes.byref(q), ctypes.byref(t)))
        self._pending[int(t.value)] = (q, seeds, gains, rep)
        return int(t.value)

    def wait(self, ticket: int):
        """(seeds, gains, Report, latency in ms) of a submitted query."""
        lat = DBL(0.0)
        _check(self.lib.tim_server_wait(self.handle, ticket, ctypes.byref(lat)))
        _, seeds, gains, rep = self._pending.pop(ticket)
        return seeds, gains, rep, lat.value

    def stop(self) -> BatchInfo:
        info = BatchInfo()
        if self.handle:
            _check(self.lib.tim_server_stop(self.handle, ctypes.byref(info)))
            self.handle = None
            self._pending.clear()
        return info

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()


def report_dict(rep: Report, k: int) -> dict:
    """The fields of a Report in the vocabulary of the paper."""
    kp = rep.kpt
    return dict(
        ell_used=rep.ell_used, **{"lambda": rep.lambda_},
        i_max=kp.i_max, i_last=kp.i_last, c_last=int(kp.c_last), kpt_star=kp.kpt_star, round_sums=kp.round_sums(),
        round_c={i: int(kp.round_c[i]) for i in range(1, kp.i_last + 1)},
        round_width={i: int(kp.round_width[i]) for i in range(1, kp.i_last + 1)},
        round_nodes={i: int(kp.round_nodes[i]) for i in range(1, kp.i_last + 1)},
        eps_prime=rep.refine.eps_prime, lambda_prime=rep.refine.lambda_prime,
        theta_prime=int(rep.refine.theta_prime), covered_prime=int(rep.refine.covered_prime),
        kpt_prime=rep.refine.kpt_prime, kpt_plus=rep.refine.kpt_plus,
        theta=int(rep.select.theta), ns_nodes=int(rep.select.nodes), ns_width=int(rep.select.width),
        ns_covered=int(rep.select.covered), s_prime=np.array(rep.s_prime[:min(k, 128)], dtype=np.int32),
        ms_kpt=rep.ms_kpt, ms_refine=rep.ms_refine, ms_select_sample=rep.ms_select_sample,
        ms_select_greedy=rep.ms_select_greedy, ms_total=rep.ms_total, sets_total=int(rep.sets_total),
        width_total=int(rep.width_total))
