"""Time to 1e-2 relative error of v* for the SGD arms (plain, Hutchinson =
Algorithm 1, learned preconditioner, exact diagonal), on synthetic data.

Training recipe of the network: data sets at 64^3 and 128^3 with varied
defocus ranges, Hutchinson diagonals with 200 probes as targets, Adam on the
GPU kernels.  Evaluation: the mid (128^3, 50,000 images, batch 256) and
high-resolution (256^3, 200,000 images, batch 1024) workloads, noise-free
(see `experiment`), every arm from v = 0 with the same Armijo rule; the run
stops when the relative error over the ball (or over the high-frequency
half of it) reaches 1e-2.  Wall time = setup (the arm's own preparation)
+ iterations + error evaluations.
"""
from __future__ import annotations

import time

import torch

from . import experiment as E
from . import learned as L

# (grid side, images, blobs, defocus range in micrometres) of the training sets
TRAIN_SPECS = [(64, 10_000, 100, (0.5 + 0.25 * i, 2.0 + 0.25 * i)) for i in range(10)] + \
              [(128, 20_000, 200, (0.5 + 0.3 * i, 2.0 + 0.3 * i)) for i in range(10)]

EVAL_SPECS = {
    "mid_128": dict(M=128, N=50_000, n_blobs=200, batch=256, defocus_um=(0.8, 3.0), seed=2128),
    "hires_256": dict(M=256, N=200_000, n_blobs=1000, batch=1024, defocus_um=(1.0, 3.0), seed=3256),
    # ill-conditioned stress case: preferred orientations (von Mises-Fisher
    # viewing directions, kappa 10), 500,000 images regenerated per batch
    # (410 GB would not fit in device memory), deterministic adjoint
    "stress_320": dict(M=320, N=500_000, n_blobs=1000, batch=2048, defocus_um=(0.5, 4.0), seed=5320,
                       poses="vmf", kappa=10.0, stream=True, deterministic=True, cg_tol=1e-9, cg_max_iter=150, max_epochs=8,
                       time_limit=150.0),
}


def train_network(specs=TRAIN_SPECS, steps: int = 2000, n_probe: int = 200, log=print):
    t0 = time.perf_counter()
    sets = []
    for i, (M, N, nb, dfr) in enumerate(specs):
        ds = E.make_dataset(M, N, nb, 7000 + i, float("inf"), defocus_um=dfr)
        sets.append(L.training_set(ds, n_probe=n_probe, seed=i))
        del ds
    torch.cuda.empty_cache()
    params, hist = L.train(sets, steps=steps)
    if log:
        log("[tta] network trained on %d sets (%d samples) in %.1fs, final loss %.3e" % (
            len(sets), sum(s.X.shape[0] for s in sets), time.perf_counter() - t0, hist[-1][1]))
    return params, hist


MILESTONES = (0.1, 0.05, 0.02, 0.01)


def milestones(errors, col):
    """First (iteration, seconds) at which the error in column `col` of the
    recorded (iteration, seconds, ball error, high-band error) rows is at or
    below each milestone (None: not reached)."""
    out = {}
    for m in MILESTONES:
        hit = next(((it, round(t, 4)) for it, t, *e in errors if e[col - 2] <= m), None)
        out[str(m)] = hit
    return out


def fsc_summary(curve):
    """Lowest shell correlation over shells 1 .. M/2 - 1 and the first shell
    where it drops below 0.9 and 0.75 (None: never)."""
    c = curve[1:]
    first = lambda t: next((i + 1 for i, f in enumerate(c) if f < t), None)
    return {"min": round(min(c), 6), "below_0.9": first(0.9), "below_0.75": first(0.75)}


def evaluate(params, configs=("mid_128", "hires_256"), log=print, max_epochs: int = 6, time_limit: float = 60.0):
    out = {}
    for name in configs:
        spec = dict(EVAL_SPECS[name])
        batch = spec.pop("batch")
        seed = spec.pop("seed")
        ds = E.make_dataset(spec["M"], spec["N"], spec["n_blobs"], seed, float("inf"), defocus_um=spec["defocus_um"],
                            poses=spec.get("poses", "uniform"), kappa=spec.get("kappa", 10.0),
                            stream=spec.get("stream", False))
        res = {}
        stops = ("high",) if ds.streamed else ("ball", "high")
        for stop in stops:
            if log:
                log("[tta] %s stop_on=%s" % (name, stop))
            r = E.compare_arms(ds, batch, params=params, stop_on=stop, max_epochs=spec.get("max_epochs", max_epochs),
                               time_limit=spec.get("time_limit", time_limit), eval_every=10 if ds.M <= 128 else 5,
                               log=log, deterministic=spec.get("deterministic", False),
                               cg_tol=spec.get("cg_tol", 1e-6), cg_max_iter=spec.get("cg_max_iter", 500))
            res[stop] = {arm: {"reached": a.reached, "iterations": a.iterations, "run_s": round(a.seconds, 4),
                               "setup_s": round(a.setup_seconds, 4), "total_s": round(a.total_seconds, 4),
                               "gen_s": round(a.gen_seconds, 4), "note": a.note,
                               "final_error": {"ball": round(a.errors[-1][2], 6), "high": round(a.errors[-1][3], 6)}
                               if a.errors else None,
                               "fsc_final": fsc_summary(a.fsc[-1][1]) if a.fsc else None,
                               "milestones_ball": milestones(a.errors, 2), "milestones_high": milestones(a.errors, 3)}
                         for arm, a in r["arms"].items()}
            res["cg_iterations"] = r["cg_iterations"]
            res["cg_residual"] = r["cg_residual"]
        out[name] = dict(M=ds.M, N=ds.N, batch=batch, poses=spec.get("poses", "uniform"),
                         deterministic=spec.get("deterministic", False), streamed=ds.streamed, **res)
        del ds
        torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="time to 1e-2 of the SGD arms")
    ap.add_argument("--configs", default="mid_128,hires_256", help="comma-separated names of EVAL_SPECS")
    ap.add_argument("--out", default=None, help="write the JSON result here as well")
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    params, _ = train_network(log=log)
    res = evaluate(params, configs=tuple(args.configs.split(",")), log=log)
    txt = json.dumps(res)
    print(txt, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(txt + "\n")

