"""Benchmark: time-to-1e-8 residual and state-updates/s of the hypercube
solver at N=26 on one MI355X.

A step is one full solve (init, Gauss-Seidel layer sweeps, residual checks,
until the relative L1 balance residual <= 1e-8) of the N=26 / J=1000
clustered-demand deployment at load 0.7.  Inputs (rates, preference lists,
per-tile dispatch tables) are resident in HBM before timing: hq_create is
setup and is not timed.

Prints one JSON line (rank 0).  Besides value / ms_per_step it carries:
  roofline      the layer-sweep kernels' algorithmic HBM bytes per outer
                iteration over their device time per iteration (HIP events
                on the library's stream around the sweeps);
  cpu_baseline  the CPU FP64 oracle's Algorithm 1 on the same deployment,
                timed on a block of middle-layer states (coefficient step
                and outer-iteration updates) at one thread and at every
                host thread, scaled to the full state space.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 L1 residual & state-updates/s at N=26; warm/batched vs plain"
HBM_PEAK_GBS = 8000.0
# sources that decide what the sweep launches do: the kernels, their tables,
# and the host code that builds the dispatch programs and picks the stored
# layers
KERNEL_SRCS = [os.path.join(ROOT, "paper_2603_03019_amd", "csrc", f)
               for f in ("hq_kernels.hip", "hq_sweep.hip", "hq_sweeptab.h", "hq_api.cpp", "hq_tables.h",
                         "hq_layout.h")]


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(hashlib.sha256(f.read()).digest())
    return h.hexdigest()


def measured_traffic(N: int, precision: str):
    """HBM bytes per outer iteration of the layer kernels, from the committed
    counter summary; None when the sweep's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"sweep_n{N}_{precision}_hbm_bytes.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_iteration"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes_per_iteration(N: int, s: int) -> float:
    """Each swept layer n = 1..N-1 reads layers n-1 and n+1 and writes layer n once."""
    C = math.comb
    return float(s * sum(C(N, n - 1) + C(N, n) + C(N, n + 1) for n in range(1, N)))


def _sample_layer_states(rng, N: int, n: int, k: int):
    """k uniformly drawn states of layer n (n of the N bits set)."""
    import numpy as np

    bits = np.argsort(rng.random((k, N)), axis=1)[:, :n].astype(np.uint32)
    return np.bitwise_or.reduce(np.left_shift(np.uint32(1), bits), axis=1).astype(np.uint32)


def _oracle_rates(cpu, inst, n: int, threads: int, coef_target_s: float, update_target_s: float):
    """Per-state seconds of Algorithm 1's step 2 (coefficients by Algorithm
    3) and of one outer-iteration update, timed by the oracle on a block of
    consecutive layer-n states, the block sized to take about the target times."""
    first = math.comb(inst.N, n) // 3
    probe = cpu.time_sample(inst, n, first, 2000, 2, threads)
    per_coef = max(probe["coef_s"] / 2000, 1e-9)
    count = int(min(math.comb(inst.N, n) - first, max(2000, coef_target_s / per_coef)))
    per_upd = max(probe["update_s"] / 2000, 1e-10)
    reps = int(max(1, min(50, update_target_s / (per_upd * count))))
    r = cpu.time_sample(inst, n, first, count, reps, threads)
    return r["coef_s"] / count, r["update_s"] / count, r["threads"], count, reps


def cpu_baseline(inst, iterations: int, checks: int):
    """The CPU oracle's Algorithm 1 on the same deployment, at one thread and
    at every host thread.  A full oracle solve at 2^26 states takes about an
    hour, so the oracle times its own code on a block of middle-layer states
    (step 2's coefficient generation, then outer-iteration updates: the
    same functions its solve runs) and the figures are scaled to the whole
    state space and to the iteration count the GPU solve needed."""
    from oracle import cpu

    cpu.build(force=False)
    N = inst.N
    n = N // 2
    S = (1 << N) - 2
    legs = {}
    for threads in (1, cpu.threads()):
        if threads in legs:
            continue
        per_coef, per_upd, used, count, reps = _oracle_rates(cpu, inst, n, threads, 4.0, 3.0)
        coef_s = per_coef * (1 << N)
        iter_s = per_upd * S
        legs[used] = {
            "value": 1.0 / per_upd,
            "unit": "state-updates/s",
            "cores": used,
            "coef_s": coef_s,
            "iter_s": iter_s,
            "time_to_tol_s": coef_s + (iterations + checks) * iter_s,
            "sample": f"{count} consecutive layer-{n} states, {reps} update reps",
        }
    top = legs[max(legs)]
    one = legs[min(legs)]
    # the old figure: one update (12) of sampled states with the coefficients
    # generated per state (what a solve pays when it stores no coefficients)
    import numpy as np

    rng = np.random.default_rng(0)
    states = _sample_layer_states(rng, N, n, 200000)
    p = np.full(1 << N, 1.0 / math.comb(N, n))
    t = time.perf_counter()
    cpu.update_states(inst, states, p, p, 1.0, 1.0)
    on_demand = len(states) / (time.perf_counter() - t)
    del p
    return {
        "value": top["value"],
        "unit": "state-updates/s",
        "cores": top["cores"],
        "kind": "oracle",
        "sample": f"Algorithm 1 of the FP64 oracle on the same N={N}, J={inst.J} deployment, timed on "
                  f"{top['sample']} (coefficient step and outer-iteration updates, the functions its "
                  f"solve runs) and scaled to 2^{N} states; time_to_tol_s = coef_s + (iterations + "
                  f"residual checks of the GPU solve = {iterations} + {checks}) x iter_s",
        "time_to_tol_s": top["time_to_tol_s"],
        "coef_s": top["coef_s"],
        "iter_s": top["iter_s"],
        "single_thread": one,
        "on_demand_update": {"value": on_demand, "unit": "state-updates/s", "cores": cpu.threads(),
                             "note": "one update (12) of 200000 sampled layer states with the "
                                     "coefficients generated per state (no step 2)"},
    }


def copy_probe(mib: int, reps: int):
    """A plain device copy of known size (calibrates the HBM byte counters)."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "reps": reps}), flush=True)


def batched_leg(hq, config_instance, tol: float, count: int = 256):
    """The batch of uneven deployments in one persistent launch vs one plain
    solve after the other (same contexts, same tolerance)."""
    import torch

    insts = [config_instance(4, i) for i in range(count)]
    ctxs = [hq.create_from_instance(i, inner=hq.HQ_INNER_ONE) for i in insts]
    hq.hq_solve_batch(ctxs, tol)  # first call: work-group size autotune and graph capture
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, infos = hq.hq_solve_batch(ctxs, tol)
    batch_s = time.perf_counter() - t
    block = hq.hq_batch_last_block()
    t = time.perf_counter()
    seq = [hq.hq_solve(c, tol) for c in ctxs]
    seq_s = time.perf_counter() - t
    updates = sum(((1 << i.N) - 2) * x["iterations"] for i, x in zip(insts, infos))
    for c in ctxs:
        hq.hq_destroy(c)
    return {
        "workload": f"{count} deployments, N~U{{12..18}} (total {sum(1 << i.N for i in insts)} states), "
                    f"J=100 uniform, mu_i~U[0.8,1.2], load 0.6, tol {tol:g}",
        "tile_low_bits": 10,
        "work_group_threads": block,
        "batched_s": batch_s,
        "sequential_s": seq_s,
        "speedup_vs_sequential": seq_s / batch_s,
        "state_updates_per_s": updates / batch_s,
        "iterations_mean": sum(x["iterations"] for x in infos) / count,
        "max_residual": max(x["residual"] for x in infos),
        "sequential_max_residual": max(x["residual"] for x in seq),
    }


def warm_leg(hq, inst, tol: float, plain_s: float, plain_iters: float, steps: int):
    """Learned product-form start (shipped network) on the same instance;
    the timed region also covers feature extraction and inference."""
    import torch

    from paper_2603_03019_amd import warmstart

    net = warmstart.load_network()
    ctx = hq.create_from_instance(inst, inner=hq.HQ_INNER_ONE, mlp=net)
    hq.hq_solve(ctx, tol)
    torch.cuda.synchronize()
    total, iters, kept, res = 0.0, 0, 0, 0.0
    for _ in range(steps):
        t = time.perf_counter()
        X = hq.hq_mlp_features(inst.N, inst.J, inst.lam, inst.nu, inst.pref)
        hq.hq_mlp_forward(net, X)
        info = hq.hq_solve(ctx, tol)
        total += time.perf_counter() - t
        iters += info["iterations"]
        kept += info["warm_used"]
        res = max(res, info["residual"])
    hq.hq_destroy(ctx)
    hq.hq_mlp_destroy(net)
    return {
        "time_to_tol_s": total / steps,
        "iterations": iters / steps,
        "plain_time_to_tol_s": plain_s,
        "plain_iterations": plain_iters,
        "speedup_vs_plain": plain_s / (total / steps),
        "warm_start_kept": kept / steps,
        "final_residual": res,
    }


def fp32_leg(hq, inst, tol: float, P64, steps: int):
    """FP32 storage with per-layer scales (FP64 reductions), handed to FP64
    at the FP32 floor; error of the result against the FP64 solve."""
    import numpy as np
    import torch

    ctx = hq.create_from_instance(inst, inner=hq.HQ_INNER_ONE, precision=hq.HQ_FP32_POLISH64)
    hq.hq_solve(ctx, tol)
    torch.cuda.synchronize()
    t = time.perf_counter()
    infos = [hq.hq_solve(ctx, tol) for _ in range(steps)]
    wall = (time.perf_counter() - t) / steps
    P = hq.hq_state(ctx)
    hq.hq_destroy(ctx)
    it = infos[-1]
    return {
        "time_to_tol_s": wall,
        "iterations": it["iterations"],
        "fp64_iterations": it["fp64_iterations"],
        "sweep_state_updates_per_s": ((1 << inst.N) - 2) * it["iterations"] / max(it["sweep_seconds"], 1e-12),
        "final_residual": it["residual"],
        "l1_vs_fp64": float(np.abs(P - P64).sum()),
        # maximum percentage relative error over the states, eq. (15)
        "mpre_vs_fp64_percent": float(100.0 * np.max(np.abs(P - P64)[P64 > 0] / P64[P64 > 0])),
    }


def inner_leg(hq, inst, tol: float):
    """Outer iterations and time to tol for the readings of the inner loop:
    one update, the closed-form limit, and the literal loop at two
    tolerances (the same instance and stopping rule)."""
    import torch

    out = {}
    for name, kw in (("one", dict(inner=hq.HQ_INNER_ONE)), ("closed", dict(inner=hq.HQ_INNER_CLOSED)),
                     ("literal_1e-6", dict(inner=hq.HQ_INNER_LITERAL, delta=1e-6)),
                     ("literal_1e-10", dict(inner=hq.HQ_INNER_LITERAL, delta=1e-10))):
        ctx = hq.create_from_instance(inst, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = hq.hq_solve(ctx, tol)
        out[name] = {"iterations": info["iterations"], "time_to_tol_s": time.perf_counter() - t,
                     "sweep_ms_per_iteration": 1e3 * info["sweep_seconds"] / max(info["iterations"], 1)}
        hq.hq_destroy(ctx)
        # the exact crossing: the residual checked after every outer iteration
        ctx = hq.create_from_instance(inst, check_every=1, **kw)
        out[name]["iterations_checked_every_iteration"] = hq.hq_solve(ctx, tol)["iterations"]
        hq.hq_destroy(ctx)
    return out


def dispatch_leg(hq, ctx, inst):
    """Dispatch probabilities and mean travel time of the solved instance
    (superset-sum transform of P); synthetic travel times."""
    import numpy as np
    import torch

    d = np.linalg.norm(inst.atom_xy[:, None, :] - inst.unit_xy[None, :, :], axis=2)
    travel = 0.03 + d / 0.5
    hq.hq_dispatch(ctx, travel)  # first call allocates the transform buffer
    torch.cuda.synchronize()
    t = time.perf_counter()
    q, mt = hq.hq_dispatch(ctx, travel)
    dt = time.perf_counter() - t
    rho, _ = hq.hq_marginals(ctx)
    return {"seconds": dt, "mean_travel": mt,
            "max_flow_gap": float(np.abs((inst.lam[:, None] * q).sum(axis=0) - inst.nu * rho).max()),
            "note": "P export + 6 superset-sum passes over 2^26 doubles + per-node gather"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=26)
    ap.add_argument("--J", type=int, default=1000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--precision", choices=["fp64", "fp32", "polish"], default="fp64")
    ap.add_argument("--inner", choices=["closed", "one"], default="one")
    ap.add_argument("--tile-bits", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the batched, warm and FP32 forms")
    ap.add_argument("--profile-iters", type=int, default=0,
                    help="only set up and run this many outer iterations (for counter runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the solver runs each "
              "instance on one device and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2603_03019_amd import hq
    from paper_2603_03019_amd.instances import config_instance

    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe, 4)
        return
    inst = config_instance(3, 0, N=args.N, J=args.J)
    prec = {"fp64": hq.HQ_FP64, "fp32": hq.HQ_FP32, "polish": hq.HQ_FP32_POLISH64}[args.precision]
    inner = hq.HQ_INNER_ONE if args.inner == "one" else hq.HQ_INNER_CLOSED
    print(f"bench: create N={inst.N} J={inst.J} precision={args.precision} inner={args.inner}", flush=True)
    t = time.perf_counter()
    ctx = hq.create_from_instance(inst, precision=prec, inner=inner, tile_bits=args.tile_bits, device=0)
    create_s = time.perf_counter() - t
    if args.profile_iters:
        hq.hq_iterate(ctx, args.profile_iters)
        torch.cuda.synchronize()
        print(json.dumps({"profile_iters": args.profile_iters, "N": inst.N,
                          "bytes_per_iteration": algorithmic_bytes_per_iteration(
                              inst.N, 8 if args.precision == "fp64" else 4)}), flush=True)
        return
    for i in range(args.warmup):
        info = hq.hq_solve(ctx, args.tol)
        print(f"bench: warmup {i} iterations={info['iterations']} residual={info['residual']:.3e} "
              f"seconds={info['seconds']:.3f}", flush=True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        infos.append(hq.hq_solve(ctx, args.tol))
        print(f"bench: step {i} iterations={infos[-1]['iterations']} residual={infos[-1]['residual']:.3e}",
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iters = sum(x["iterations"] for x in infos)
    sweep_s = sum(x["sweep_seconds"] for x in infos)
    states = (1 << inst.N) - 2
    s = 8 if args.precision == "fp64" else 4
    bytes_it = algorithmic_bytes_per_iteration(inst.N, s)
    per_it = sweep_s / max(iters, 1)
    achieved = bytes_it / per_it / 1e9
    out = {
        "metric": METRIC,
        "value": states * iters / wall,
        "unit": "state-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "polish": "f32+f64"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"plain loss system N={inst.N} units, J={inst.J} demand nodes in 4 Gaussian "
                        f"clusters (sigma 0.1), mu_i~U[0.5,1.5], load 0.7, solve to relative L1 balance "
                        f"residual {args.tol:g}",
            "N": inst.N, "J": inst.J, "load": inst.load, "tol": args.tol,
            "precision": args.precision, "inner": args.inner,
            "iterations_per_solve": iters / args.steps,
        },
        "time_to_tol_s": wall / args.steps,
        "sweep_state_updates_per_s": states * iters / max(sweep_s, 1e-12),
        "create_s": create_s,
        "final_residual": infos[-1]["residual"],
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(inst.N, args.precision),
            "kernel": "layer sweep: sweep_kernel (short-program layers) and layer_kernel (long-program and "
                      f"stored layers){' with the look-ahead sums of the closed form' if args.inner == 'closed' else ''}, "
                      "per outer "
                      f"iteration of {inst.N - 1} layer launches and their finalize launches",
            "bytes_per_iteration": bytes_it,
            "us_per_iteration": per_it * 1e6,
        },
    }
    if not args.no_legs and args.precision == "fp64":
        plain_s, plain_iters = wall / args.steps, iters / args.steps
        print("bench: dispatch measures", flush=True)
        out["dispatch"] = dispatch_leg(hq, ctx, inst)
        P64 = hq.hq_state(ctx)
        hq.hq_destroy(ctx)
        print("bench: inner-loop readings", flush=True)
        out["inner_forms"] = inner_leg(hq, inst, args.tol)
        print("bench: fp32 form", flush=True)
        out["fp32_form"] = fp32_leg(hq, inst, args.tol, P64, 1)
        del P64
        from paper_2603_03019_amd import warmstart

        if os.path.exists(warmstart.WEIGHTS):
            print("bench: warm start", flush=True)
            out["warm_start"] = warm_leg(hq, inst, args.tol, plain_s, plain_iters, 1)
        print("bench: batched form", flush=True)
        out["batched"] = batched_leg(hq, config_instance, args.tol)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle sample)", flush=True)
        out["cpu_baseline"] = cpu_baseline(inst, round(iters / args.steps),
                                           round(sum(x["checks"] for x in infos) / args.steps))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
