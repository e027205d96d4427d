"""Time to 1e-2 relative error of v* for the SGD arms (plain, Hutchinson =
Algorithm 1, learned preconditioner, exact diagonal), on synthetic data.

Training recipe of the network: data sets at 64^3 and 128^3 with varied
defocus ranges, Hutchinson diagonals with 200 probes as targets, Adam on the
GPU kernels.  Evaluation: the mid (128^3, 50,000 images, batch 256) and
high-resolution (256^3, 200,000 images, batch 1024) workloads, noise-free
(see `experiment`), and the mid workload at its SNR of 0.05 with a step-size
halving per epoch and iterate averaging in every arm; every arm from v = 0
with the same Armijo rule; the error is evaluated after every iteration and
the run stops when the relative error over the ball (or over the
high-frequency half of it) reaches 1e-2.  Wall time = setup (the arm's own
preparation) + iterations; the error evaluations are timed apart.  The
network's training is deterministic (seeded sampling, fixed-order gradient
sums), and its parameters can be saved and reused (--params-out/-in).
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
    # the mid workload at its own SNR (0.05), lambda = sigma^2 / tau^2: the
    # iterates are averaged from epoch 1 on (Polyak-Ruppert), identically in
    # every arm (Algorithm 1's constant-step iterates stall near relative
    # error 1 at this SNR); up to 40 epochs
    "mid_128_snr005": dict(M=128, N=50_000, n_blobs=200, batch=256, defocus_um=(0.8, 3.0), seed=2128, snr=0.05,
                           average_from_epoch=1, max_epochs=40, time_limit=200.0, stops=("ball",)),
    # the same data under the other schedules (16 epochs): Algorithm 1 as it
    # is (constant step cap), the step-size cap halved every epoch, and both
    # the halving and the averaging; the arms' error floors
    "mid_128_snr005_const": dict(M=128, N=50_000, n_blobs=200, batch=256, defocus_um=(0.8, 3.0), seed=2128,
                                 snr=0.05, max_epochs=16, time_limit=120.0, stops=("ball",)),
    "mid_128_snr005_decay": dict(M=128, N=50_000, n_blobs=200, batch=256, defocus_um=(0.8, 3.0), seed=2128,
                                 snr=0.05, decay_epochs=1, max_epochs=16, time_limit=120.0, stops=("ball",)),
    "mid_128_snr005_decay_avg": dict(M=128, N=50_000, n_blobs=200, batch=256, defocus_um=(0.8, 3.0), seed=2128,
                                     snr=0.05, decay_epochs=1, average_from_epoch=1, max_epochs=16,
                                     time_limit=120.0, stops=("ball",)),
    # ill-conditioned stress case: preferred orientations (von Mises-Fisher
    # viewing directions, kappa 10), 500,000 images regenerated per batch
    # (410 GB would not fit in device memory), deterministic adjoint
    "stress_320": dict(M=320, N=500_000, n_blobs=1000, batch=2048, defocus_um=(0.5, 4.0), seed=5320,
                       poses="vmf", kappa=10.0, stream=True, deterministic=True, cg_tol=1e-9, cg_max_iter=150, max_epochs=8,
                       time_limit=150.0, fsc_every=61),
    # the stress set at its own SNR (0.02), lambda = sigma^2 / tau^2, the
    # noise of each regenerated image made on the device from its index;
    # iterates averaged from epoch 1 on in every arm, as for the mid set
    "stress_320_snr002": dict(M=320, N=500_000, n_blobs=1000, batch=2048, defocus_um=(0.5, 4.0), seed=5320,
                              poses="vmf", kappa=10.0, stream=True, deterministic=True, snr=0.02, cg_tol=1e-7,
                              cg_max_iter=150, average_from_epoch=1, max_epochs=40, time_limit=150.0,
                              stops=("ball",)),
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


def fsc_epochs(fsc_rows, thresholds=(0.75, 0.9, 0.99)):
    """Per shell, the first recorded iteration (epoch ends and the stop) at
    which the shell correlation with v* reaches each threshold (None: never);
    and the shell x epoch table of the correlations (Sec. 4.2's FSC figures)."""
    nsh = len(fsc_rows[0][1]) if fsc_rows else 0
    first = {}
    for th in thresholds:
        first[str(th)] = [next((it for it, curve in fsc_rows if curve[s] >= th), None) for s in range(nsh)]
    return {"iterations": [it for it, _ in fsc_rows], "first_iteration_at": first,
            "table": [[round(c, 4) for c in curve] for _, curve in fsc_rows]}


def arm_record(a, with_fsc_table=False):
    rec = {"reached": a.reached, "iterations": a.iterations, "run_s": round(a.seconds, 4),
           "setup_s": round(a.setup_seconds, 4), "total_s": round(a.total_seconds, 4),
           "gen_s": round(a.gen_seconds, 4), "eval_s": round(a.eval_seconds, 4), "capped": a.capped, "note": a.note,
           "final_error": {"ball": round(a.errors[-1][2], 6), "high": round(a.errors[-1][3], 6)} if a.errors else None,
           "fsc_final": fsc_summary(a.fsc[-1][1]) if a.fsc else None,
           "milestones_ball": milestones(a.errors, 2), "milestones_high": milestones(a.errors, 3)}
    if with_fsc_table and a.fsc:
        rec["fsc_epochs"] = fsc_epochs(a.fsc)
    return rec


def evaluate(params, configs=("mid_128", "hires_256"), log=print, max_epochs: int = 6, time_limit: float = 60.0,
             precomputed_epochs=None, fsc_tables: bool = False):
    """precomputed_epochs: {config name: epochs} of the precomputed arm
    (default 1000, the paper's; 0 leaves the arm out)."""
    out = {}
    for name in configs:
        spec = dict(EVAL_SPECS[name])
        batch = spec.pop("batch")
        seed = spec.pop("seed")
        snr = spec.get("snr", float("inf"))
        ds = E.make_dataset(spec["M"], spec["N"], spec["n_blobs"], seed, snr, defocus_um=spec["defocus_um"],
                            poses=spec.get("poses", "uniform"), kappa=spec.get("kappa", 10.0),
                            stream=spec.get("stream", False))
        pe = 1000 if precomputed_epochs is None else precomputed_epochs.get(name, 1000)
        arms = ("plain", "hutchinson", "learned", "precomputed", "exact") if pe > 0 else \
            ("plain", "hutchinson", "learned", "exact")
        res = {}
        stops = spec.get("stops", ("high",) if ds.streamed else ("ball", "high"))
        v_star = E.ground_truth(ds, tol=spec.get("cg_tol", 1e-6), max_iter=spec.get("cg_max_iter", 500),
                                log=log if ds.N * ds.M ** 2 > 10 ** 10 else None)
        cache = {}
        for stop in stops:
            if log:
                log("[tta] %s stop_on=%s" % (name, stop))
            r = E.compare_arms(ds, batch, params=params, arms=arms, stop_on=stop, v_star=v_star,
                               max_epochs=spec.get("max_epochs", max_epochs),
                               time_limit=spec.get("time_limit", time_limit), eval_every=1, log=log,
                               deterministic=spec.get("deterministic", False), precomputed_epochs=pe, cache=cache,
                               decay_epochs=spec.get("decay_epochs", 0),
                               average_from_epoch=spec.get("average_from_epoch"),
                               fsc_every=spec.get("fsc_every", 0) if fsc_tables else 0)
            res[stop] = {arm: arm_record(a, fsc_tables) for arm, a in r["arms"].items()}
            res[stop + "_diagonals"] = r["diagonals"]
        res["cg_iterations"] = v_star[1]
        res["cg_residual"] = v_star[2]
        out[name] = dict(M=ds.M, N=ds.N, batch=batch, poses=spec.get("poses", "uniform"), snr=snr, lam=ds.lam,
                         deterministic=spec.get("deterministic", False), streamed=ds.streamed,
                         decay_epochs=spec.get("decay_epochs", 0), average_from_epoch=spec.get("average_from_epoch"),
                         **res)
        del ds
        torch.cuda.empty_cache()
    return out


def save_params(params, path):
    import numpy as np
    np.save(path, params.cpu().numpy())


def load_params(path, device="cuda"):
    import numpy as np
    return torch.from_numpy(np.load(path, allow_pickle=False)).to(device)


if __name__ == "__main__":
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="time to 1e-2 of the SGD arms")
    ap.add_argument("--configs", default="mid_128,hires_256", help="comma-separated names of EVAL_SPECS")
    ap.add_argument("--out", default=None, help="write the JSON result here as well")
    ap.add_argument("--params-in", default=None, help="use these trained network parameters (.npy)")
    ap.add_argument("--params-out", default=None, help="save the trained network parameters here (.npy)")
    ap.add_argument("--precomputed-epochs", default="", help="name=epochs,... for the precomputed arm (default 1000)")
    ap.add_argument("--fsc-tables", action="store_true", help="record the shell x epoch FSC tables")
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.params_in:
        params = load_params(args.params_in)
    else:
        params, _ = train_network(log=log)
    if args.params_out:
        save_params(params, args.params_out)
    pe = {k: int(v) for k, v in (kv.split("=") for kv in args.precomputed_epochs.split(",") if kv)}
    res = evaluate(params, configs=tuple(args.configs.split(",")), log=log, precomputed_epochs=pe,
                   fsc_tables=args.fsc_tables)
    txt = json.dumps(res)
    print(txt, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(txt + "\n")

