"""Evaluation of the shipped warm-start network on the 100 unseen N = 24
deployments (J = 500, load ~ U[0.5, 0.9)), with every final answer checked
by the CPU oracle.

    python tests/warm_start_oracle_eval.py [--count 100] [--out FILE]

For each deployment: iterations and solve seconds to a 1e-8 balance
residual from the cold start of Algorithm 1 (p_n = 1 / C(N, n)), the
heuristic product-form seed and the learned seed, and the seconds of
hq_create for the cold and the learned start (the latter includes feature
extraction and inference); then the oracle's relative L1 balance residual
of (1), with its own Algorithm-3 coefficients, on the learned answer.  The
summary is merged, under "oracle_check", into a copy of
paper_2603_03019_amd/weights/warm_mlp_eval.json written to --out (by
default that file itself).  Test infrastructure: it loads the oracle.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import cpu  # noqa: E402
from paper_2603_03019_amd import hq, warmstart  # noqa: E402
from paper_2603_03019_amd.instances import config_instance  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=100)
    ap.add_argument("--weights", default="", help="network parameters (default: the shipped ones)")
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2603_03019_amd", "weights", "warm_mlp_eval.json"))
    a = ap.parse_args()
    src = a.out if os.path.exists(a.out) else os.path.join(ROOT, "paper_2603_03019_amd", "weights",
                                                           "warm_mlp_eval.json")
    net = warmstart.load_network(a.weights) if a.weights else warmstart.load_network()
    rows = []
    for idx in range(50000, 50000 + a.count):
        inst = config_instance(6, idx)
        res = {}
        for name, kw in (("cold", {}), ("heuristic", dict(init_rho=warmstart.heuristic_rho(inst))),
                         ("learned", dict(mlp=net))):
            t0 = time.perf_counter()
            ctx = hq.create_from_instance(inst, inner=hq.HQ_INNER_ONE, **kw)
            create_s = time.perf_counter() - t0
            info = hq.hq_solve(ctx, 1e-8)
            # seconds of hq_create (tables, programs, and for the learned
            # start its features and inference) and of hq_solve
            res[name] = (info["iterations"], info["seconds"], info["residual"], info["warm_used"], create_s)
            if name == "learned":
                P = hq.hq_state(ctx)
            hq.hq_destroy(ctx)
        r = cpu.residual(inst, P)
        rows.append({"index": idx, "load": inst.load, "cold": res["cold"][0], "heuristic": res["heuristic"][0],
                     "learned": res["learned"][0], "cold_s": res["cold"][1], "learned_s": res["learned"][1],
                     "cold_create_s": res["cold"][4], "learned_create_s": res["learned"][4],
                     "kept": res["learned"][3], "gpu_residual": res["learned"][2], "oracle_residual": r})
        print(f"eval {idx}: cold {res['cold'][0]} heuristic {res['heuristic'][0]} learned {res['learned'][0]} "
              f"(kept {res['learned'][3]}), oracle residual of the learned answer {r:.3e}", flush=True)
    summ = {
        "instances": len(rows),
        "tolerance": 1e-8,
        "cold_iterations_mean": float(np.mean([x["cold"] for x in rows])),
        "heuristic_iterations_mean": float(np.mean([x["heuristic"] for x in rows])),
        "learned_iterations_mean": float(np.mean([x["learned"] for x in rows])),
        "cold_solve_seconds_mean": float(np.mean([x["cold_s"] for x in rows])),
        "learned_solve_seconds_mean": float(np.mean([x["learned_s"] for x in rows])),
        "cold_create_seconds_mean": float(np.mean([x["cold_create_s"] for x in rows])),
        "learned_create_seconds_mean": float(np.mean([x["learned_create_s"] for x in rows])),
        "learned_kept_fraction": float(np.mean([x["kept"] for x in rows])),
        "oracle_residual_max": float(max(x["oracle_residual"] for x in rows)),
        "gpu_residual_max": float(max(x["gpu_residual"] for x in rows)),
        "oracle_threads": cpu.threads(),
        "rows": [{k: x[k] for k in ("index", "cold", "learned", "kept", "oracle_residual")} for x in rows],
    }
    print(json.dumps(summ), flush=True)
    with open(src) as f:
        d = json.load(f)
    d["oracle_check"] = summ
    with open(a.out, "w") as f:
        json.dump(d, f, indent=1)
    hq.hq_mlp_destroy(net)


if __name__ == "__main__":
    main()
