#!/usr/bin/env python3
"""Benchmark of the TIM+ hot path on one MI355X.

Workload: a directed Chung-Lu power-law graph with n = 1,000,000 nodes and
m = 10,000,000 edges (alpha = 2.1, seed 2), independent cascade with
p(u,v) = 1/indeg(v), TIM+ with eps = 0.2, ell = 1.  One step runs TIM+ for
k = 1, 10 and 50 (KptEstimation, RefineKPT, NodeSelection: every RR set is
generated on the GPU).  The graph is resident in device memory before timing.

Prints one JSON line: RR sets generated per second over the timed steps
(value; RefineKPT takes the sets of the last KptEstimation round without
generating them again, as Algorithm 3 prescribes, so they count once), edges
examined per second, TIM+ seconds per k, the roofline of the dominant sampler
kernel (algorithmic bytes over its event-timed duration), and the CPU oracle
timed on the host on one TIM+ run of the same graph (k = 50), whose result the
last timed k = 50 run must equal ("parity").  Outside the timed steps it also
reports LT (1/indeg and random in-weights), the general triggering model, and
("batched") the 64-query mixed workload below as one batch against the same
queries one by one (--no-batch skips it).

--workload batch64: 64 independent TIM+ queries, each on a Chung-Lu graph of
its own (n log-uniform in [10^4, 2*10^6], average degree uniform in [4, 40];
even queries IC with per-edge p from {0.1, 0.01, 0.001}, odd ones LT; k
uniform in [1, 50], eps from {0.1, 0.2, 0.5}, ell = 1), all graphs resident.
A step runs the 64 queries one after the other (tim_run) and then as one
batch (tim_run_batch); value is the batch's queries per second, beside the
sequential rate, and the two must return identical results.

--workload serve: a request loop (tim_server_*, 16 slots, 200 GB budget) over
4 resident Chung-Lu graphs (n = 10^5, 10^6, 4*10^6, 10^7, average degree 16).
Queries from a seeded stream (graph and model uniform, IC with p = 1/indeg or
LT, k uniform in [1, 100], eps from {0.1, 0.2, 0.3}, ell = 1) arrive as a
Poisson process at 1, 5, 20, 50 and 200 per second; each rate reports p50 and
p99 latency (submission to result) and the queries per second completed.
value is the rate sustained at 200 arrivals per second; the same queries run
one by one (tim_run) give the plain rate, and must give the same results.

--workload sweep: quality and time of TIM and TIM+ on the 1M-node graph
(IC with p = 1/indeg, and LT), a k sweep (eps = 0.2) and an eps sweep
(k = 50): TIM+ and TIM seconds, theta, KPT*, KPT+ and their ratio, and the
expected spread of the seeds by 10^4 forward Monte-Carlo runs (tim_spread_mc).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import hashlib

KS = (1, 10, 50)
EPS, ELL, SEED = 0.2, 1.0, 2
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per RR entry of the inverted index and greedy: the entry read by the counts pass, read and
# written by the scatter, and read by the cover pass that decrements the counts of a chosen node's sets (4 B each).
GREEDY_BYTES_PER_ENTRY = 20
SEG_GROUPS = 1  # 4-edge groups per lane and step of the IC segment kernels (kSegGroups)
MODES = ("widths", "store", "cover")
# HBM bytes per launch of the first-tier IC kernels that can be the dominant
# one (stored sets; widths of the large rounds), from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs of this benchmark (scaled by a plain-copy calibration; see
# profiles/ic_seg_kernel_chunglu_n1e6_m1e7.md), for the shapes the autotuner
# picks on this graph.  Valid only for the kernel sources they were taken on.
TRAFFIC = {
    "ic_seg_kernel<1, true, 8, 128, 0, 512, 1> (store)": {
        "sources_sha256_16": "f04a4aa503ad565e", "taken": "2026-12-03", "fetch_bytes": 2906637862, "write_bytes": 571520432},
    "ic_seg_kernel<0, true, 8, 128, 0, 512, 1> (widths)": {
        "sources_sha256_16": "f04a4aa503ad565e", "taken": "2026-12-03", "fetch_bytes": 2645093577, "write_bytes": 104174699},
}
KERNEL_SOURCES = ("paper_1404_0900_amd/csrc/sample.hip", "paper_1404_0900_amd/csrc/rng.hpp",
                  "paper_1404_0900_amd/csrc/pick.hpp", "paper_1404_0900_amd/csrc/engine.hpp")


def sources_sha():
    """Hash of the kernel sources' code: comments and blank lines do not count."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(line.rstrip() for line in text.splitlines() if line.strip()).encode())
    return h.hexdigest()[:16]


def kernel_name(model, mode, lanes=None):
    """Tier-0 sampler kernel of (model, mode) as rocprofv3 lists it (template arguments: mode, WC, lanes per set,
    queue length, log2 of the hash size, group limit, groups per lane)."""
    if model == 1:
        return f"lt_lane_kernel<{mode}> ({MODES[mode]})"
    if lanes is None:
        lanes = int(os.environ.get("TIM_IC_SEG_LANES", "8"))
    lanes = lanes if lanes in (4, 8, 16, 32, 64) else 8
    q = {4: 64, 8: 128, 16: 128, 32: 256, 64: 512}[lanes]
    hlog = {4: 0, 8: 0, 16: 8, 32: 9, 64: 10}[lanes]
    gmax = {4: 256, 8: 512, 16: 512, 32: 1024, 64: 2048}[lanes]
    return f"ic_seg_kernel<{mode}, true, {lanes}, {q}, {hlog}, {gmax}, {SEG_GROUPS}> ({MODES[mode]})"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain leg of the default line")
    ap.add_argument("--workload", choices=("timplus", "batch64", "serve", "sweep"), default="timplus")
    ap.add_argument("--mc-runs", type=int, default=10_000, help="forward Monte-Carlo runs per seed set (sweep)")
    ap.add_argument("--rates", type=str, default="1,5,20,50,200", help="arrival rates per second (serve)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the context's sampler shapes (TIM_IC_SEG_LANES) instead of timing them first")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        return batch_main(args)
    if args.workload == "serve":
        return serve_main(args)
    if args.workload == "sweep":
        return sweep_main(args)

    import torch

    import paper_1404_0900_amd as tim
    import synth

    log("generating the 1M-node / 10M-edge Chung-Lu graph")
    g = synth.config_graph("cfg2")
    eng = tim.Engine(0)
    dg = eng.upload(g)
    log(f"graph resident: n={g.n} m={g.m}")
    if args.no_autotune:
        tune = tim.TuneResult()
        tune.seg_lanes = int(os.environ.get("TIM_IC_SEG_LANES", "8"))
        tune.slice_cap = 0
    else:
        # the sampler shapes for this graph, before timing, on launches about the size of its large rounds
        tune = eng.autotune(dg, tim.IC, 1 << 22)
    log(f"sampler shape: {tune.seg_lanes} lanes per set, slice cap {tune.slice_cap}")

    last = {}  # per k: seeds, gains and report of the last run (compared with the oracle below)

    def step():
        out = []
        for k in KS:
            t0 = time.perf_counter()
            seeds, gains, rep = eng.run(dg, tim.IC, k, EPS, ELL, SEED)
            out.append((k, time.perf_counter() - t0, rep))
            last[k] = (seeds, gains, rep)
        return out

    phases = {}  # per k: GPU milliseconds of each phase and the collection sizes (last timed step)

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    eng.profile(True)
    sets = width = 0
    greedy_entries = greedy_argmax_bytes = 0  # RR entries the greedy runs index, and their argmax passes' bytes
    per_k = {k: 0.0 for k in KS}
    t0 = time.perf_counter()
    for i in range(args.steps):
        for k, dt, rep in step():
            sets += rep.sets_total
            width += rep.width_total
            # two greedy runs per query: RefineKPT's on R' (the last KptEstimation round) and NodeSelection's
            greedy_entries += int(rep.kpt.round_nodes[rep.kpt.i_last]) + int(rep.select.nodes)
            greedy_argmax_bytes += 2 * k * 4 * g.n
            per_k[k] += dt
            phases[str(k)] = {"kpt_ms": round(rep.ms_kpt, 3), "refine_ms": round(rep.ms_refine, 3),
                              "select_sample_ms": round(rep.ms_select_sample, 3),
                              "select_greedy_ms": round(rep.ms_select_greedy, 3),
                              "c_last": int(rep.kpt.c_last), "theta_prime": int(rep.refine.theta_prime),
                              "theta": int(rep.select.theta), "rr_entries": int(rep.select.nodes)}
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = eng.read_profile()
    eng.profile(False)

    # dominant sampler kernel: the one with the most GPU time in the timed steps
    def name_of(model, mode):
        return kernel_name(model, mode, tune.seg_lanes)

    def traffic_of(model, mode):
        t = TRAFFIC.get(name_of(model, mode))
        if t and sources_sha() == t["sources_sha256_16"]:
            return t["fetch_bytes"] + t["write_bytes"]
        return None
    roofline = dominant_roofline(prof, name_of, traffic_of)
    t = TRAFFIC.get(roofline["kernel"])
    roofline["traffic_source"] = (
        f"stored figure: rocprofv3 FETCH_SIZE and WRITE_SIZE runs of {t['taken']} on kernel sources "
        f"{t['sources_sha256_16']} (profiles/), scaled by a plain-copy calibration"
        if roofline["traffic"] is not None else
        "null: no counter run on the current kernel sources " + sources_sha())
    sampler_ms = sum(prof.sampler[a][b].kernel_ms + prof.sampler[a][b].large_ms for a in (0, 1) for b in (0, 1, 2))
    sampler_ms += sum(prof.ic_wide[b].kernel_ms + prof.ic_wide[b].large_ms for b in (0, 1, 2))
    sampler_ms += sum(prof.grouped[a].kernel_ms + prof.grouped[a].large_ms for a in (0, 1))
    by_phase = sampler_by_mode(prof, 0)
    roofline_widths = kernel_roofline(prof, 0, 0, name_of, traffic_of)
    ig_ms = prof.index_ms + prof.greedy_ms
    ig_bytes = GREEDY_BYTES_PER_ENTRY * greedy_entries + greedy_argmax_bytes
    ig_gbs = ig_bytes / (ig_ms * 1e-3) / 1e9 if ig_ms > 0 else 0.0
    roofline_index_greedy = {
        "bound": "hbm", "achieved": round(ig_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(ig_gbs / HBM_PEAK_GBS, 5), "traffic": None,
        "kernels": "inverted index (counts, scan, scatter) and greedy (argmax, cover) of every query",
        "entries_per_step": greedy_entries // args.steps, "bytes_per_entry": GREEDY_BYTES_PER_ENTRY,
        "argmax_bytes_per_step": greedy_argmax_bytes // args.steps, "gpu_ms_per_step": round(ig_ms / args.steps, 3)}

    line = {
        "metric": "RR sets/s (IC, 1 GPU, TIM+ on 1M-node Chung-Lu, k in {1,10,50})",
        "value": round(sets / elapsed, 1),
        "unit": "RR sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 integer, f64 kappa",
        "data": "synthetic (seeded directed Chung-Lu, alpha=2.1)",
        "config": {"workload": "chunglu_n1e6_m1e7_ic_wc_timplus_k1_10_50", "n": g.n, "m": g.m, "alpha": 2.1,
                   "graph_seed": 2, "model": "IC p=1/indeg", "k": list(KS), "eps": EPS, "ell": ELL, "seed": SEED},
        "edges_per_s": round(width / elapsed, 1),
        "tim_plus_s": {str(k): round(per_k[k] / args.steps, 6) for k in KS},
        "phases": phases,
        "sets_per_step": sets // args.steps,
        "sampler_gpu_ms_per_step": round(sampler_ms / args.steps, 3),
        "index_greedy_gpu_ms_per_step": round((prof.index_ms + prof.greedy_ms) / args.steps, 3),
        "sampler_by_phase": by_phase,
        "roofline": roofline,
        "roofline_widths": roofline_widths,
        "roofline_index_greedy": roofline_index_greedy,
        "autotune": None if args.no_autotune else {
            "seg_lanes": int(tune.seg_lanes), "slice_cap": int(tune.slice_cap),
            "ms_width_4_8_16_32_64": [round(x, 3) for x in tune.ms_width],
            "ms_stored_4_8_16_32_64": [round(x, 3) for x in tune.ms_lanes_emit],
            "ms_emit_512_1024_2048_4096": [round(x, 3) for x in tune.ms_emit]},
    }

    # the same TIM+ runs under LT (one uniform in-edge per node), outside the timed steps
    lt_sets, t0 = 0, time.perf_counter()
    lt_per_k = {}
    for k in KS:
        t1 = time.perf_counter()
        _, _, rep = eng.run(dg, tim.LT, k, EPS, ELL, SEED)
        lt_per_k[str(k)] = round(time.perf_counter() - t1, 6)
        lt_sets += rep.sets_total
    line["lt"] = {"sets_per_s": round(lt_sets / (time.perf_counter() - t0), 1), "tim_plus_s": lt_per_k}

    # LT with random in-weights normalized per node (the paper's LT setting), also outside the timed steps
    eng.set_lt_weights(dg, g, synth.random_lt_thresholds(g, SEED))
    for k in KS:  # warm-up
        eng.run(dg, tim.LT, k, EPS, ELL, SEED)
    lw_sets, t0 = 0, time.perf_counter()
    lw_per_k = {}
    for k in KS:
        t1 = time.perf_counter()
        _, _, rep = eng.run(dg, tim.LT, k, EPS, ELL, SEED)
        lw_per_k[str(k)] = round(time.perf_counter() - t1, 6)
        lw_sets += rep.sets_total
    line["lt_weighted"] = {"sets_per_s": round(lw_sets / (time.perf_counter() - t0), 1), "tim_plus_s": lw_per_k}
    eng.set_lt_weights(dg, g, None)

    # the general triggering model (explicit per-node distributions over in-edge subsets), outside the timed steps
    log("general triggering model: drawing the distributions")
    eng.set_triggering(dg, g, synth.random_triggering(g, SEED))
    for k in KS:  # warm-up
        eng.run(dg, tim.TRIGGER, k, EPS, ELL, SEED)
    tr_sets, t0 = 0, time.perf_counter()
    tr_per_k = {}
    for k in KS:
        t1 = time.perf_counter()
        _, _, rep = eng.run(dg, tim.TRIGGER, k, EPS, ELL, SEED)
        tr_per_k[str(k)] = round(time.perf_counter() - t1, 6)
        tr_sets += rep.sets_total
    line["trigger"] = {"sets_per_s": round(tr_sets / (time.perf_counter() - t0), 1), "tim_plus_s": tr_per_k,
                       "distribution": "synth.random_triggering(seed 2): 1-4 outcomes per node, 1-3 in-edges each, "
                                       "total probability 1 (a quarter of the nodes) or uniform in [0.3, 0.8]"}
    eng.set_triggering(dg, g, None)

    line["parity"] = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the CPU oracle: one TIM+ run, IC, k=50")
        t0 = time.perf_counter()
        r = oracle.tim_run(g, 0, 50, EPS, ELL, SEED)
        dt = time.perf_counter() - t0
        osets = sum(r["round_c"].values()) + r["c_last"] + r["theta_prime"] + r["theta"]
        line["cpu_baseline"] = {
            "value": round(osets / dt, 1), "unit": "RR sets/s", "cores": 1, "kind": "oracle",
            "sample": f"one oracle TIM+ run (IC, k=50) on the same graph: {osets} RR sets in {dt:.2f} s",
            "cpu_model": cpu_model(), "host_cpus": host_cpus(),
        }
        line["parity"] = parity_with_oracle(tim, last[50], r, 50)
        log(f"parity of the last timed k=50 run with the oracle: {line['parity']}")
    eng.close()
    if not args.no_batch:
        # batched vs plain queries/s on the 64-query mixed workload (its own graphs; outside the timed steps)
        b = batch_measure(2, 1)
        line["batched"] = {"metric": "TIM+ queries/s, 64 mixed queries, batched vs one by one",
                           "queries_per_s": b["queries_per_s"], "plain_queries_per_s": b["sequential"]["value"],
                           "speedup": b["speedup_vs_sequential"], "identical_outputs": b["identical_outputs"],
                           "device_kpt_ms": b["device_kpt"]["ms"], "job_cap": b["device_kpt"]["job_cap"],
                           "workload": b["config"]["workload"], "steps": 2}
    print(json.dumps(line), flush=True)


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_cpus():
    """CPUs this process may run on, and the machine's count."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"usable": usable, "online": os.cpu_count()}


def parity_with_oracle(tim, gpu, want, k):
    """Bit-exact comparison of one GPU TIM+ run (seeds, gains, report) with the oracle's."""
    import numpy as np
    seeds, gains, rep = gpu
    r = tim.report_dict(rep, k)
    fields = ["i_last", "c_last", "kpt_star", "round_sums", "theta_prime", "covered_prime", "kpt_prime", "kpt_plus",
              "theta", "ns_nodes", "ns_width", "ns_covered"]
    bad = [f for f in fields if r[f] != want[f]]
    if not np.array_equal(seeds, want["seeds"]):
        bad.append("seeds")
    if not np.array_equal(gains, want["gains"]):
        bad.append("gains")
    return {"run": f"IC k={k} eps={EPS} ell={ELL} seed={SEED}, last timed step", "identical": not bad,
            "compared": fields + ["seeds", "gains"], "mismatch": bad}


def sampler_by_mode(prof, model):
    """RR sets/s of one model's sampler per kind of launch: the width-only KptEstimation rounds, the stored
    sets (the last round kept as R' and NodeSelection's theta sets) and RefineKPT's coverage sets.  Sets and
    GPU time cover every tier of the launches (the HIP events bracket them), including IC launches of few sets
    that run the 64-lane first tier and the multi-job launches of the early rounds (whose sets include those of
    rounds past the stopping one); edges/s is the first tier's, over the sets it finished."""
    out = {}
    for mode, name in ((0, "kpt_widths"), (1, "stored_sets"), (2, "refine_coverage")):
        parts = [prof.sampler[model][mode]] + ([prof.ic_wide[mode]] if model == 0 else [])
        if mode == 0:
            parts.append(prof.grouped[model])
        launches = sum(int(p.launches) for p in parts)
        if not launches:
            continue
        sets = sum(int(p.sets + p.deferred) for p in parts)
        ms = sum(p.kernel_ms + p.large_ms for p in parts)
        out[name] = {"launches": launches, "sets": sets, "gpu_ms": round(ms, 3),
                     "sets_per_s": round(sets / (ms * 1e-3), 1),
                     "tier0_edges_per_s": round(sum(p.edges for p in parts) / (sum(p.kernel_ms for p in parts) * 1e-3), 1)}
        wide = prof.ic_wide[mode] if model == 0 else None
        if wide is not None and wide.launches:
            out[name]["wide_launches"] = int(wide.launches)
        if mode == 0 and prof.grouped[model].launches:
            out[name]["grouped_launches"] = int(prof.grouped[model].launches)
    return out


def profiled_kernel_ms(prof):
    """Kernel time a tim_profile holds: every IC and LT sampler launch (all tiers), the index builds
    and the greedy runs. Of a sequential run it is the GPU's busy time, which no batching can beat
    unless its launches themselves run faster."""
    ms = sum(prof.sampler[a][b].kernel_ms + prof.sampler[a][b].large_ms for a in (0, 1) for b in (0, 1, 2))
    ms += sum(prof.ic_wide[b].kernel_ms + prof.ic_wide[b].large_ms for b in (0, 1, 2))
    ms += sum(prof.grouped[a].kernel_ms + prof.grouped[a].large_ms for a in (0, 1))
    return ms + prof.index_ms + prof.greedy_ms


def dominant_roofline(prof, name_of, traffic_of=lambda model, mode: None):
    """Roofline object of the sampler kernel with the most event time in a profile."""
    best = None
    for model in (0, 1):
        for mode in (0, 1, 2):
            kp = prof.sampler[model][mode]
            if kp.launches and (best is None or kp.kernel_ms > best[2].kernel_ms):
                best = (model, mode, kp)
    return kernel_roofline(prof, best[0], best[1], name_of, traffic_of)


def kernel_roofline(prof, model, mode, name_of, traffic_of=lambda model, mode: None):
    """Roofline object of one first-tier sampler kernel (algorithmic bytes over its event time), or None."""
    kp = prof.sampler[model][mode]
    if not kp.launches:
        return None
    achieved = kp.bytes / (kp.kernel_ms * 1e-3) / 1e9
    return {
        "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic_of(model, mode),
        "kernel": name_of(model, mode), "launches": int(kp.launches),
        "avg_launch_us": round(kp.kernel_ms * 1e3 / kp.launches, 3),
        "bytes_per_launch": int(kp.bytes // kp.launches),
        "edges_per_s": round(kp.edges / (kp.kernel_ms * 1e-3), 1),
    }


def batch_kernel_name(model, mode):
    """Tier-0 kernel of the batched launches as rocprofv3 lists it."""
    if model == 1:
        return f"lt_lane_batch_kernel<{mode}> ({MODES[mode]})"
    return f"ic_seg_batch_kernel<{mode}, false, 8, 128, 0, 512, {SEG_GROUPS}> ({MODES[mode]})"


def batch_main(args):
    res = batch_measure(args.steps, args.warmup)
    line = {
        "metric": "TIM+ queries/s, 64 mixed queries batched on 1 GPU (vs the same queries run one by one)",
        "value": res["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_batch"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 integer, f64 kappa",
        "data": "synthetic (64 seeded directed Chung-Lu graphs, alpha=2.1)",
        "config": res.pop("config"),
    }
    line.update(res)
    print(json.dumps(line), flush=True)


def batch_measure(steps, warmup):
    """The 64-query batched workload: the queries one by one (tim_run) and as one batch (tim_run_batch),
    `steps` times each after `warmup` untimed rounds; medians, identity of the outputs, and the batch's
    device KptEstimation figures."""
    import statistics

    import numpy as np
    import torch

    import paper_1404_0900_amd as tim
    import synth

    queries = synth.batch_queries(64)
    log("generating the 64 graphs of the batched workload")
    graphs = synth.batch_graphs(queries, workers=16)
    eng = tim.Engine(0)
    dgs = [eng.upload(g, thr=thr) for g, thr in graphs]
    batch = [(dg, q["model"], q["k"], q["eps"], q["ell"], q["seed"]) for dg, q in zip(dgs, queries)]
    log(f"64 graphs resident: {sum(g.m for g, _ in graphs)} edges")

    def sequential():
        return [eng.run(*b) for b in batch]

    def same(seq, bat):
        for (s1, g1, r1), (s2, g2, r2) in zip(seq, bat):
            if not (np.array_equal(s1, s2) and np.array_equal(g1, g2) and r1.select.theta == r2.select.theta
                    and r1.kpt.kpt_star == r2.kpt.kpt_star and r1.refine.kpt_plus == r2.refine.kpt_plus
                    and r1.select.nodes == r2.select.nodes and r1.select.width == r2.select.width):
                return False
        return True

    for i in range(warmup):
        sequential()
        eng.run_batch(batch)
        log(f"batch warmup {i + 1}/{warmup} done")
    # the granularity of the batch's device KptEstimation work queue, timed before the steps
    tune = eng.autotune_batch(batch)
    log(f"batch autotune: {[int(c) for c in tune.caps]} sets per query and step -> "
        f"{[round(x, 2) for x in tune.ms_kpt]} ms; kept {int(tune.job_cap)}")
    t_seq, t_bat, identical, info = [], [], True, None
    sets = 0
    for i in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seq = sequential()
        t_seq.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        bat, info = eng.run_batch(batch)
        t_bat.append(time.perf_counter() - t0)
        identical = identical and same(seq, bat)
        sets = sum(int(r.sets_total) for _, _, r in bat)
        log(f"batch step {i + 1}/{steps}: sequential {t_seq[-1]:.3f} s, batched {t_bat[-1]:.3f} s "
            f"(device KptEstimation {info.ms_kpt:.1f} ms in {info.kpt_steps} steps / {info.kpt_graph_launches} "
            f"graph launches; then {info.rounds} rounds, {info.launches} launches, up to {info.max_jobs} jobs), "
            f"identical={identical}")
    ts, tb = statistics.median(t_seq), statistics.median(t_bat)

    # the queries one by one once more with per-launch timing: the GPU's busy time of the sequential run
    eng.profile(True)
    sequential()
    seq_kernel_ms = profiled_kernel_ms(eng.read_profile())
    eng.profile(False)
    # one more batch with per-launch timing, for the roofline of the dominant batched kernel
    eng.profile(True)
    eng.run_batch(batch)
    prof = eng.read_profile()
    eng.profile(False)
    roofline = dominant_roofline(prof, batch_kernel_name)

    slow = sorted(((r.ms_total, q["name"]) for (_, _, r), q in zip(seq, queries)), reverse=True)[:5]
    out = {
        "queries_per_s": round(64 / tb, 3),
        "ms_per_batch": round(tb * 1e3, 3),
        "config": {"workload": "batch64_chunglu_ic_trivalency_lt", "queries": 64, "n_range": [10_000, 2_000_000],
                   "avg_degree_range": [4, 40], "ic_p": list(synth.TRIVALENCY_P), "k_range": [1, 50],
                   "eps": [0.1, 0.2, 0.5], "ell": 1.0, "seeds": "1000+j",
                   "edges_total": int(sum(g.m for g, _ in graphs))},
        "sequential": {"value": round(64 / ts, 3), "unit": "queries/s", "ms_per_step": round(ts * 1e3, 3),
                       "kernel_ms": round(seq_kernel_ms, 3)},
        "speedup_vs_sequential": round(ts / tb, 3),
        "identical_outputs": identical,
        "device_kpt": {"ms": round(info.ms_kpt, 3), "steps": int(info.kpt_steps),
                       "graph_launches": int(info.kpt_graph_launches), "job_cap": int(info.kpt_job_cap),
                       "autotune_caps": [int(c) for c in tune.caps],
                       "autotune_ms": [round(x, 3) for x in tune.ms_kpt]},
        "rounds": int(info.rounds), "launches": int(info.launches), "max_jobs": int(info.max_jobs),
        "rr_sets_per_step": sets,
        "rr_sets_per_s": round(sets / tb, 1),
        "slowest_alone_ms": {name: round(ms, 3) for ms, name in slow},
        "roofline": roofline,
    }
    eng.close()
    return out


def serve_main(args):
    import numpy as np
    import torch

    import paper_1404_0900_amd as tim
    import synth

    slots, budget = 16, 200 << 30
    log("generating the 4 resident graphs of the serving workload")
    graphs = synth.serve_graphs()
    eng = tim.Engine(0, budget_bytes=budget)
    dgs = [eng.upload(g) for g in graphs]
    log(f"graphs resident: {[g.n for g in graphs]} nodes, {sum(g.m for g in graphs)} edges")
    for q in synth.serve_queries(8, 100.0, 99):  # warm-up: buffers of the plain path
        eng.run(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"])

    def serve(qs):
        with eng.serve(slots) as srv:
            t0 = time.perf_counter()
            tickets = []
            for q in qs:
                delay = q["arrival"] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                tickets.append((time.perf_counter() - t0,
                                srv.submit(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"])))
            res = [(t_sub,) + srv.wait(t) for t_sub, t in tickets]
            info = srv.stop()
        return res, info

    serve(synth.serve_queries(16, 200.0, 98))  # warm-up: member contexts and their buffers
    sweep, last = [], None
    for idx, rate in enumerate(float(r) for r in args.rates.split(",")):
        count = int(min(60, max(10, rate * 10)))
        qs = synth.serve_queries(count, rate, 7 + idx)
        res, info = serve(qs)
        lat = np.array([r[4] for r in res])
        first = qs[0]["arrival"]
        done = max(r[0] + r[4] / 1e3 for r in res)
        point = {"rate_per_s": rate, "queries": count, "completed_per_s": round(count / (done - first), 3),
                 "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                 "rounds": int(info.rounds), "max_jobs": int(info.max_jobs),
                 "rr_pool_gb": round(info.rr_pool_bytes / 1e9, 3), "rr_peak_gb": round(info.rr_peak_bytes / 1e9, 3),
                 "held_queries": int(info.held_queries), "held_ms": round(info.held_ms, 3)}
        sweep.append(point)
        last = (qs, res)
        log(f"rate {rate:g}/s: {point}")

    # the last point's queries one by one: the plain rate, and the same results
    qs, res = last
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    identical = True
    for q, r in zip(qs, res):
        seeds, gains, rep = eng.run(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"])
        identical = identical and np.array_equal(seeds, r[1]) and np.array_equal(gains, r[2]) and \
            rep.select.theta == r[3].select.theta and rep.refine.kpt_plus == r[3].refine.kpt_plus
    plain = time.perf_counter() - t0
    log(f"plain: {len(qs)} queries one by one in {plain:.3f} s, identical={identical}")
    # once more with per-launch timing: the GPU's busy time of the plain run
    eng.profile(True)
    for q in qs:
        eng.run(dgs[q["graph"]], q["model"], q["k"], q["eps"], q["ell"], q["seed"])
    plain_kernel_s = profiled_kernel_ms(eng.read_profile()) * 1e-3
    eng.profile(False)
    log(f"plain: kernel time {plain_kernel_s:.3f} s")
    top = sweep[-1]
    line = {
        "metric": "served TIM+ queries/s at 200 Poisson arrivals/s (1 GPU, continuous batching), p50/p99 latency",
        "value": top["completed_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": len(sweep),
        "warmup": 1,
        "ms_per_step": round(1e3 * top["queries"] / top["completed_per_s"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 integer, f64 kappa",
        "data": "synthetic (4 seeded directed Chung-Lu graphs, alpha=2.1; seeded Poisson query stream)",
        "config": {"workload": "serve_chunglu_4graphs_deg16_poisson", "graphs_n": [g.n for g in graphs],
                   "avg_degree": synth.SERVE_DEGREE, "models": ["IC p=1/indeg", "LT"], "k_range": [1, 100],
                   "eps": [0.1, 0.2, 0.3], "ell": 1.0, "slots": slots, "budget_bytes": budget},
        "p50_ms": top["p50_ms"],
        "p99_ms": top["p99_ms"],
        "sweep": sweep,
        "plain": {"value": round(len(qs) / plain, 3), "unit": "queries/s", "queries": len(qs),
                  "seconds": round(plain, 3), "kernel_s": round(plain_kernel_s, 3),
                  "kernel_bound_queries_per_s": round(len(qs) / plain_kernel_s, 3)},
        "identical_outputs": identical,
    }
    eng.close()
    print(json.dumps(line), flush=True)


def sweep_main(args):
    import math

    import paper_1404_0900_amd as tim
    import synth

    log("generating the 1M-node / 10M-edge Chung-Lu graph")
    g = synth.config_graph("cfg2")
    eng = tim.Engine(0)
    dg = eng.upload(g)
    for model in (tim.IC, tim.LT):  # warm-up
        eng.run(dg, model, 10, 0.5, ELL, SEED)
        eng.spread(dg, model, SEED, [0], 10)
    points = [("k", k, 0.2) for k in (1, 10, 20, 30, 40, 50)] + [("eps", 50, e) for e in (0.1, 0.2, 0.3, 0.5)]
    rows = []
    for model in (tim.IC, tim.LT):
        for sweep, k, eps in points:
            t0 = time.perf_counter()
            seeds, gains, rep = eng.run(dg, model, k, eps, ELL, SEED)
            t_plus = time.perf_counter() - t0
            plain = eps >= 0.2  # TIM at eps = 0.1 needs billions of sets here (theta = lambda / KPT*)
            if plain:
                t0 = time.perf_counter()
                seeds_p, _, rep_p = eng.run(dg, model, k, eps, ELL, SEED, tim.FLAG_PLAIN)
                t_plain = time.perf_counter() - t0
            t0 = time.perf_counter()
            spread, _ = eng.spread(dg, model, SEED + 1, seeds, args.mc_runs)
            spread_p = eng.spread(dg, model, SEED + 1, seeds_p, args.mc_runs)[0] if plain else None
            t_mc = time.perf_counter() - t0
            row = {"model": "IC" if model == tim.IC else "LT", "sweep": sweep, "k": k, "eps": eps,
                   "tim_plus_s": round(t_plus, 5), "tim_s": round(t_plain, 5) if plain else None,
                   "theta_plus": int(rep.select.theta),
                   "theta_tim": int(rep_p.select.theta) if plain else int(math.ceil(rep.lambda_ / rep.kpt.kpt_star)),
                   "kpt_star": round(rep.kpt.kpt_star, 3), "kpt_plus": round(rep.refine.kpt_plus, 3),
                   "kpt_ratio": round(rep.refine.kpt_plus / rep.kpt.kpt_star, 3),
                   "spread_plus": round(spread, 2), "spread_tim": round(spread_p, 2) if plain else None,
                   "mc_runs": args.mc_runs, "mc_s": round(t_mc, 3)}
            rows.append(row)
            log(f"{row}")
    eng.close()
    line = {
        "metric": "TIM/TIM+ quality and time sweeps (1 GPU, 1M-node Chung-Lu): seconds, theta, KPT+/KPT*, E[I(S)]",
        "value": round(sum(r["tim_plus_s"] for r in rows), 5),
        "unit": "s (sum of TIM+ runs over the sweep)",
        "n_gpus": 1, "steps": len(rows), "warmup": 1,
        "ms_per_step": round(1e3 * sum(r["tim_plus_s"] for r in rows) / len(rows), 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32/u64 integer, f64 kappa", "data": "synthetic (seeded directed Chung-Lu, alpha=2.1)",
        "config": {"workload": "sweep_chunglu_n1e6_m1e7", "n": g.n, "m": g.m, "ell": ELL, "seed": SEED,
                   "mc_runs": args.mc_runs},
        "rows": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
