"""Writes the oracle's TIM+ results on the 1M-node / 10M-edge Chung-Lu graph
(alpha 2.1, graph seed 2) for k = 1 and k = 10, eps = 0.2, ell = 1, seed 2,
under IC (weighted cascade) and LT (1/indeg in-weights).

Only the CPU oracle computes these values: the k = 1 runs take minutes on one
core, too long to repeat inside every GPU test session.  The file records a
hash of the graph so that a test can refuse values of another graph.

    python tests/golden/make_timplus_golden.py      (about 5 minutes, 4 threads)
"""
import hashlib
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "timplus_chunglu_n1e6_m1e7_k1_k10.json")
RUNS = [(0, 1), (1, 1), (0, 10), (1, 10)]
EPS, ELL, SEED = 0.2, 1.0, 2


def graph_hash(g) -> str:
    h = hashlib.sha256()
    h.update(g.off.astype("<i8").tobytes())
    h.update(g.src.astype("<i4").tobytes())
    return h.hexdigest()


def encode(r: dict) -> dict:
    out = {}
    for key, v in r.items():
        if key in ("seeds", "gains", "s_prime"):
            out[key] = [int(x) for x in v]
        elif isinstance(v, dict):
            out[key] = {str(i): int(x) for i, x in v.items()}
        elif isinstance(v, float):
            out[key] = v.hex()
        else:
            out[key] = int(v)
    return out


def main() -> None:
    g = synth.config_graph("cfg2")

    def run(mk):
        model, k = mk
        print(f"oracle TIM+ model={model} k={k} ...", flush=True)
        return mk, oracle.tim_run(g, model, k, EPS, ELL, SEED)

    with ThreadPoolExecutor(len(RUNS)) as ex:
        results = list(ex.map(run, RUNS))
    doc = {"graph": {"name": "cfg2", "n": g.n, "m": g.m, "sha256": graph_hash(g)},
           "eps": EPS, "ell": ELL, "seed": SEED,
           "runs": [{"model": model, "k": k, "result": encode(r)} for (model, k), r in results]}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
