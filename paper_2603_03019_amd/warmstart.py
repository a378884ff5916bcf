"""Learned warm start: training data from the solver itself, GPU training of
the network, and the cold / heuristic / learned comparison.

All arithmetic runs in libhq.so (batched solves, feature extraction, the
network's forward/backward/Adam kernels); this module only orchestrates.

* ``training_set``: solve a seeded pool of deployments (N ~ U{16..20},
  load ~ U[0.5, 0.9); uniform demand with J = 500, plus a share with four
  Gaussian demand clusters, J = 1000 and mu ~ U[0.5, 1.5]) with one batched
  launch per chunk and return the per-unit features with the solved busy
  probabilities as targets.
* ``train``: fit a fresh network on that set (Adam, minibatches, on the GPU).
* ``heuristic_rho``: the baseline product-form seed, each unit as an M/M/1/1
  queue fed by the demand that ranks it first: a / (1 + a), a = load / nu.
* ``evaluate``: iterations and time to the tolerance for the cold start
  (1/C(N,n), Algorithm 1 step 2), the heuristic seed and the learned seed.
"""
from __future__ import annotations

import argparse
import json
import os
import time
from typing import Dict, List, Optional

import numpy as np

from . import hq
from .instances import config_instance

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warm_mlp.npy")


def load_network(path: str = WEIGHTS, device: int = -1):
    """The shipped network (FP32 master parameters written by ``main``)."""
    params = np.load(path, allow_pickle=False)
    m = hq.hq_mlp_create(device=device, seed=0)
    hq.hq_mlp_set_params(m, params)
    return m


CLUSTERED = dict(clusters=4, sigma=0.1, J=1000, nu_range=(0.5, 1.5))


def pool_instance(i: int, count: int, clustered: float):
    """Deployment i of a training pool of ``count``: the last
    round(count * clustered) have clustered demand."""
    n_uniform = count - int(round(count * clustered))
    if i < n_uniform:
        return config_instance(5, 1000 + i)
    return config_instance(5, 200000 + i, **CLUSTERED)


def training_set(count: int, *, clustered: float = 0.0, tol: float = 1e-7, chunk: int = 512,
                 verbose: bool = False, targets: Optional[np.ndarray] = None):
    """Features X [rows, HQ_MLP_IN] and targets t [rows] (busy probabilities).
    With ``targets`` (the t of an earlier call on the same pool) nothing is
    solved again: the features are rebuilt from the seeded deployments."""
    X: List[np.ndarray] = []
    t: List[np.ndarray] = []
    if targets is not None:
        for i in range(count):
            inst = pool_instance(i, count, clustered)
            X.append(hq.hq_mlp_features(inst.N, inst.J, inst.lam, inst.nu, inst.pref))
        X = np.concatenate(X)
        if X.shape[0] != targets.shape[0]:
            raise ValueError("targets do not match this pool")
        return X, np.asarray(targets, dtype=np.float32)
    for c0 in range(0, count, chunk):
        insts = [pool_instance(i, count, clustered) for i in range(c0, min(count, c0 + chunk))]
        ctxs = [hq.create_from_instance(i, inner=hq.HQ_INNER_ONE) for i in insts]
        t0 = time.perf_counter()
        hq.hq_solve_batch(ctxs, tol)
        for inst, ctx in zip(insts, ctxs):
            rho, _ = hq.hq_marginals(ctx)
            X.append(hq.hq_mlp_features(inst.N, inst.J, inst.lam, inst.nu, inst.pref))
            t.append(rho.astype(np.float32))
            hq.hq_destroy(ctx)
        if verbose:
            print(f"warmstart: solved {min(count, c0 + chunk)}/{count} training deployments "
                  f"({time.perf_counter() - t0:.1f}s)", flush=True)
    return np.concatenate(X), np.concatenate(t)


def holdout_rmse(net, count: int) -> dict:
    """RMSE of the predicted utilisations on ``count`` uniform and ``count``
    clustered deployments outside the training pool (solved to 1e-8)."""
    out = {}
    for kind, base, kw in (("uniform", 900000, {}), ("clustered", 950000, CLUSTERED)):
        insts = [config_instance(5, base + i, **kw) for i in range(count)]
        ctxs = [hq.create_from_instance(i, inner=hq.HQ_INNER_ONE) for i in insts]
        hq.hq_solve_batch(ctxs, 1e-8)
        err = []
        for inst, ctx in zip(insts, ctxs):
            rho, _ = hq.hq_marginals(ctx)
            pred = hq.hq_mlp_forward(net, hq.hq_mlp_features(inst.N, inst.J, inst.lam, inst.nu, inst.pref))
            err.append(np.asarray(pred, float) - rho)
            hq.hq_destroy(ctx)
        e = np.concatenate(err)
        out[f"val_rmse_{kind}"] = float(np.sqrt(np.mean(e * e)))
    out["holdout_per_kind"] = count
    return out


def train(X: np.ndarray, t: np.ndarray, *, epochs: int = 40, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0, device: int = -1):
    """A fresh network fitted on (X, t); returns (network, per-epoch loss)."""
    m = hq.hq_mlp_create(device=device, seed=seed)
    losses = hq.hq_mlp_train(m, X, t, epochs=epochs, batch=batch, lr=lr, seed=seed + 1)
    return m, losses


def heuristic_rho(inst) -> np.ndarray:
    share0 = np.zeros(inst.N)
    np.add.at(share0, inst.pref[:, 0], inst.lam)
    a = share0 / inst.nu
    return a / (1.0 + a)


def evaluate(net, indices, *, tol: float = 1e-8, config: int = 6, verbose: bool = False,
             overrides: Optional[dict] = None) -> Dict[str, list]:
    """Per instance: iterations, seconds and final residual for the three starts."""
    out: Dict[str, list] = {"cold": [], "heuristic": [], "learned": [], "warm_kept": [], "N": []}
    for idx in indices:
        inst = config_instance(config, idx, **(overrides or {}))
        runs = {
            "cold": dict(),
            "heuristic": dict(init_rho=heuristic_rho(inst)),
            "learned": dict(mlp=net),
        }
        # the learned start also pays for its features and inference (done in hq_create)
        t0 = time.perf_counter()
        feats = hq.hq_mlp_features(inst.N, inst.J, inst.lam, inst.nu, inst.pref)
        hq.hq_mlp_forward(net, feats)
        infer_s = time.perf_counter() - t0
        for name, kw in runs.items():
            ctx = hq.create_from_instance(inst, inner=hq.HQ_INNER_ONE, **kw)
            info = hq.hq_solve(ctx, tol)
            sec = info["seconds"] + (infer_s if name == "learned" else 0.0)
            out[name].append((info["iterations"], sec, info["residual"]))
            if name == "learned":
                out["warm_kept"].append(info["warm_used"])
            hq.hq_destroy(ctx)
        out["N"].append(inst.N)
        if verbose:
            print(f"warmstart: eval {idx}: cold {out['cold'][-1][0]} it, heuristic "
                  f"{out['heuristic'][-1][0]} it, learned {out['learned'][-1][0]} it", flush=True)
    return out


def summarize(res: Dict[str, list]) -> dict:
    s = {}
    for name in ("cold", "heuristic", "learned"):
        it = np.array([r[0] for r in res[name]], float)
        sec = np.array([r[1] for r in res[name]], float)
        s[name] = {"iterations_mean": float(it.mean()), "seconds_mean": float(sec.mean()),
                   "max_residual": float(max(r[2] for r in res[name]))}
    s["learned_vs_cold_time"] = s["cold"]["seconds_mean"] / s["learned"]["seconds_mean"]
    s["learned_vs_cold_iterations"] = s["cold"]["iterations_mean"] / s["learned"]["iterations_mean"]
    s["warm_kept_fraction"] = float(np.mean(res["warm_kept"]))
    s["instances"] = len(res["N"])
    return s


def main(argv=None):
    """Train the shipped network on method-generated solves and evaluate it.

    python -m paper_2603_03019_amd.warmstart --train 20000 --clustered 0.2 --eval 100
    """
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000, help="training deployments to solve")
    ap.add_argument("--clustered", type=float, default=0.2, help="share of clustered-demand deployments")
    ap.add_argument("--eval", type=int, default=100, help="unseen N=24 deployments to evaluate")
    ap.add_argument("--epochs", type=int, default=120)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--summary", default="")
    ap.add_argument("--targets", default="", help="solved targets of the pool: reused if the file exists, "
                                                  "else written after solving")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--holdout", type=int, default=400,
                    help="uniform and clustered deployments outside the pool for the RMSE of the prediction")
    a = ap.parse_args(argv)
    t = time.perf_counter()
    cached = np.load(a.targets, allow_pickle=False) if a.targets and os.path.exists(a.targets) else None
    X, y = training_set(a.train, clustered=a.clustered, verbose=True, targets=cached)
    if a.targets and cached is None:
        np.save(a.targets, y, allow_pickle=False)
    print(f"warmstart: {X.shape[0]} rows from {a.train} solves in {time.perf_counter() - t:.1f}s", flush=True)
    t = time.perf_counter()
    net, losses = train(X, y, epochs=a.epochs, batch=a.batch, lr=a.lr)
    print(f"warmstart: trained in {time.perf_counter() - t:.1f}s, loss {losses[0]:.3e} -> {losses[-1]:.3e}",
          flush=True)
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    np.save(a.out, hq.hq_mlp_get_params(net).astype(np.float32), allow_pickle=False)
    s = {"train_solves": a.train, "train_clustered": a.clustered, "train_rows": int(X.shape[0]), "epochs": a.epochs,
         "batch": a.batch, "lr": a.lr,
         "loss_first": float(losses[0]), "loss_last": float(losses[-1])}
    if a.holdout:
        s["validation"] = holdout_rmse(net, a.holdout)
        print(f"warmstart: held-out RMSE {s['validation']}", flush=True)
    if a.eval:
        s.update(summarize(evaluate(net, range(50000, 50000 + a.eval), verbose=True)))
    print(json.dumps(s), flush=True)
    if a.summary:
        with open(a.summary, "w") as f:
            json.dump(s, f, indent=1)


if __name__ == "__main__":
    main()
