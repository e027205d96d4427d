"""Benchmark: one step = one iteration of Algorithm 1 (Hutchinson arm) on a
batch of 1024 images of 256 x 256 against a 256^3 complex64 Fourier volume
(the steps take 8 distinct resident batches of the data set in turn) -- the
whole hot path: Rademacher probes and their Hessian-vector
product, the fused minibatch gradient (forward projection, residual, loss,
adjoint), the running-mean / exponential-average / threshold update of the
diagonal, the preconditioned step and the Armijo line-search forward pass.
Each step queues the next batch's gradient and probe product at its line
search's first trial point, as a training loop that knows its next batch
does (used by the next step when that trial is accepted); the last warm-up
step and the last timed step queue nothing, so the timed region holds
exactly its own steps' work.

Prints one JSON line.  `value` = images per second through full iterations;
`fwd_adj_images_per_s` = images per second of one plain forward projection
plus one adjoint of the same batch.  `roofline` is for the dominant kernel
of the timed steps: its algorithmic bytes per launch (per-image footprint:
image read 8P, gather 8U, scatter read-modify-write 16U; P disk pixels, U
distinct voxels an image's stencils touch) over its average launch duration
from HIP events recorded around each launch on its stream; `traffic` is the
measured HBM rate of the same launches from the committed counter summary,
when it was taken on the current kernel sources and mode; `compulsory` gives
the bytes any implementation must move once per launch (for the gradient the
disk pixels of the batch, one volume read and one read-modify-write of the
accumulator) and their rate against the peak.  `fwd_adj_roofline` is the
same figure for the separate forward and adjoint kernels together (16P + 24U
bytes per image over the sum of their average durations).
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "fwd+adj images/s @256³; time-to-1e-2 err: learned vs Hutchinson vs plain"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--M", type=int, default=256)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--batches", type=int, default=8, help="distinct resident minibatches the timed steps cycle through")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-images", type=int, default=192, help="images in the oracle's timed sample")
    ap.add_argument("--deterministic", action="store_true")
    ap.add_argument("--separate", action="store_true",
                    help="Hutchinson arm in two calls (gradient and probe product, each queued for the next "
                         "batch behind the line search) instead of the one-kernel gradient and probe product")
    ap.add_argument("--no-tta", action="store_true", help="skip the time-to-1e-2 comparison of the SGD arms")
    return ap.parse_args()


def disk_pixels(M, rmax):
    ax = np.arange(M) - M // 2
    return int(np.sum((ax[:, None] ** 2 + ax[None, :] ** 2) <= rmax * rmax))


# Distinct voxels touched per image by trilinear stencils, as a multiple of
# the disk pixels (measured on random rotations: 2.51 at M = 256).
U_OVER_P = 2.51


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_2311_16100_amd import binding as B
    from paper_2311_16100_amd.sgd import Alg1Config, Alg1Runner

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    W = synth.WORKLOADS["hires_256"]
    M, Bsz, N = args.M, args.batch, W.N
    grid, optics = B.Grid(M), B.Optics()
    rmax = grid.rmax
    P = disk_pixels(M, rmax)
    U = U_OVER_P * P

    t0 = time.time()
    vol_true = synth.blob_volume(M, W.n_blobs, W.seed)
    rot_all = synth.uniform_rotations(N, W.seed)
    df_all = synth.defocus_values(N, W.defocus_um[0], W.defocus_um[1], W.seed)
    print("[bench] inputs generated in %.1fs" % (time.time() - t0), file=sys.stderr, flush=True)

    v_true = torch.from_numpy(vol_true).to(dev)
    rot_d = torch.from_numpy(rot_all).to(dev)
    df_d = torch.from_numpy(df_all).to(dev)
    # distinct resident minibatches of the data set (images 0 .. nb*B - 1),
    # taken in turn by the timed steps: noise-free projections of the ground
    # truth
    nb = max(1, min(args.batches, N // Bsz))
    batches = []
    for b in range(nb):
        rb = rot_d[b * Bsz:(b + 1) * Bsz].contiguous()
        db = df_d[b * Bsz:(b + 1) * Bsz].contiguous()
        batches.append((rb, db, B.project(grid, optics, rb, db, v_true)))
    rot_b, df_b, x_b = batches[0]
    scale = N / Bsz
    lam = 1e-2
    alpha = B.threshold_alpha(grid, optics, rot_d, df_d, lam).item()
    v0 = torch.zeros_like(v_true)
    cfg = Alg1Config(deterministic=args.deterministic, fused=not args.separate)
    run = Alg1Runner(grid, optics, "hutchinson", scale, lam, alpha, cfg, v0, batch=Bsz)
    run_fused = run.fused  # gradient and probe product in one kernel (fast mode)

    # per-call event timing inside the step
    calls = {}

    def timed(name, fn):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        calls.setdefault(name, []).append((s, e))

    def step(i, last=False):
        # the next batch's work is queued during this step's line search,
        # except on the last warmup and the last timed step: the timed region
        # holds exactly the work of its own steps
        r, d, x = batches[i % nb]
        rn, dn, xn = batches[(i + 1) % nb]
        run.iteration(r, d, x, next_poses=None if last else (rn, dn), next_images=None if last else xn)

    for i in range(args.warmup):
        step(i, last=i == args.warmup - 1)
    torch.cuda.synchronize()
    calls.clear()
    # HIP events around every brick-kernel launch of the timed steps, on the
    # stream the kernels run on
    B.timing_enable(True)
    for k in B.KERNELS:
        B.timing_read(k)
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, last=i == args.steps - 1)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t_start
    B.timing_enable(False)
    kern = {k: B.timing_read(k) for k in ("gradient_probe", "gradient", "hvp", "project")}
    kern = {k: v for k, v in kern.items() if v[1] > 0}
    ms_per_step = 1e3 * t_steps / args.steps
    # halvings of the timed steps' line searches (a rejected first trial also
    # discards the next batch's queued results: that work is redone)
    halvings_timed = int(sum(run.state.halvings[-args.steps:]))
    print("[bench] %d Alg.1 steps: %.3f ms/step" % (args.steps, ms_per_step), file=sys.stderr, flush=True)

    # per-call breakdown of the same step (separate, identical iterations)
    for _ in range(args.steps):
        st = run.state
        g_, o_ = grid, optics
        st.k += 1
        if run.fused:
            timed("gradient_probe", lambda: B.gradient_hutchinson(g_, o_, rot_b, df_b, st.v, x_b, scale, lam,
                                                                  cfg.n_probe, cfg.probe_seed,
                                                                  probe0=(st.k - 1) * cfg.n_probe, grad_out=run.g,
                                                                  loss_out=run.sc[0:1], diag_out=run.zHz,
                                                                  workspace=run.ws_grad))
        else:
            timed("hutchinson_probe", lambda: B.hutchinson_diag(g_, o_, rot_b, df_b, cfg.n_probe, cfg.probe_seed,
                                                                scale, lam, probe0=(st.k - 1) * cfg.n_probe,
                                                                diag_out=run.zHz, workspace=run.ws_hutch))
            timed("gradient", lambda: B.gradient(g_, o_, rot_b, df_b, st.v, x_b, scale, lam, grad_out=run.g,
                                                 loss_out=run.sc[0:1], deterministic=cfg.deterministic,
                                                 workspace=run.ws_grad))
        timed("precond_step", lambda: B.precond_sgd_step(st.v, run.g, st.D, st.D_avg, run.zHz, st.k, cfg.beta,
                                                         alpha, st.eta, v_out=run.v_new, stats_out=run.sc[1:3]))
        timed("armijo_project", lambda: B.project(g_, o_, rot_b, df_b, run.v_new, subtract=x_b, out=None,
                                                  loss=run.sc[3:4], want_out=False, workspace=run.ws_proj))
    # plain forward + adjoint of the batch
    y = torch.empty_like(x_b)
    acc = torch.zeros_like(v_true)
    ws_bp = B.alloc_workspace(grid, Bsz, B.CSG_WS_BACKPROJECT_DETERMINISTIC if args.deterministic
                              else B.CSG_WS_BACKPROJECT, dev)
    B.timing_enable(True)
    for k in B.KERNELS:
        B.timing_read(k)
    for _ in range(args.steps):
        timed("project", lambda: B.project(grid, optics, rot_b, df_b, v_true, out=y, workspace=run.ws_proj))
        timed("backproject", lambda: B.backproject(grid, optics, rot_b, df_b, x_b, ctf_power=1, accum=acc,
                                                   deterministic=args.deterministic, workspace=ws_bp))
    torch.cuda.synchronize()
    B.timing_enable(False)
    kern_fa = {k: B.timing_read(k) for k in ("project", "backproject")}
    ms = {k: float(np.mean([s.elapsed_time(e) for s, e in v])) for k, v in calls.items()}
    fwd_adj = Bsz / ((ms["project"] + ms["backproject"]) * 1e-3)

    # dominant kernel of the timed steps: algorithmic bytes per launch (the
    # per-image footprint times the images of one launch) over its average
    # event-timed launch duration
    # (footprint model: image read 8P, gather 8U, scatter read-modify-write
    # 16U; a probe pair generated from its hash costs no gather bytes)
    per_image = {
        "gradient": 8 * P + 24 * U,  # image read, gather, read-modify-write
        "hvp": 16 * U,  # the packed probe pair's read-modify-write
        # both: the gradient's bytes and the probe pair's read-modify-write
        "gradient_probe": 8 * P + 24 * U + 16 * U,
        "project": 8 * P + 8 * U,  # Armijo forward: image read, gather (loss only)
    }
    dominant = max(kern, key=lambda k: kern[k][0])
    tot_ms, launches = kern[dominant]
    avg_ms = tot_ms / max(launches, 1)
    achieved = per_image[dominant] * Bsz / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "brick_kernel<%s%s>" % (dominant, ", fixed point" if args.deterministic else ""),
                "kernel_avg_ms": round(avg_ms, 4), "launches": launches,
                "bytes_per_image": round(per_image[dominant]), "P": P, "U": round(U),
                "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in kern.items()}}
    # compulsory bytes of one launch: what any implementation must move once
    # (the batch's disk pixels, plus one read of the volume and one
    # read-modify-write of the accumulator for the gradient; one
    # read-modify-write of the packed accumulator for the probe product; one
    # volume read for the loss-only forward)
    nvox = M ** 3
    compulsory = {"gradient": 8 * P * Bsz + 24 * nvox, "hvp": 16 * nvox, "project": 8 * P * Bsz + 8 * nvox,
                  # the gradient's, plus one read-modify-write of the real
                  # diagonal (the probe pair is generated, not read)
                  "gradient_probe": 8 * P * Bsz + 24 * nvox + 8 * nvox}
    cb = compulsory[dominant]
    roofline["compulsory"] = {"bytes_per_launch": cb,
                              "frac": round(cb / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    # the separate forward + adjoint pair: disk-pixel write 8P and gather 8U
    # (project), image read 8P and read-modify-write 16U (backproject), over
    # the two kernels' average durations (the zero fill outside the disk is a
    # separate kernel and not counted)
    fwd_adj_roofline = None
    if all(kern_fa[k][1] > 0 for k in kern_fa):
        pair_ms = sum(kern_fa[k][0] / kern_fa[k][1] for k in kern_fa)
        fa = (16 * P + 24 * U) * Bsz / (pair_ms * 1e-3) / 1e9
        fwd_adj_roofline = {"bound": "hbm", "achieved": round(fa, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(fa / HBM_PEAK_GBS, 4),
                            "kernels_avg_ms": {k: round(kern_fa[k][0] / kern_fa[k][1], 4) for k in kern_fa},
                            "bytes_per_image": round(16 * P + 24 * U)}
    # the same bytes over the whole entry point's event-timed duration (for
    # the gradient: the volume copy lam v, cull, plan and the kernel)
    if dominant in ms:
        # (the fused kernel's call is csg_gradient_hutchinson: the lambda v
        # copy, the lambda fill of the diagonal, cull, plan and the kernel)
        roofline["call_ms"] = round(ms[dominant], 4)
        roofline["call_frac"] = round(per_image[dominant] * Bsz / (ms[dominant] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    tr = traffic_record(dominant, Bsz, M, args.deterministic)
    if tr:
        # measured HBM bytes of one launch over the same average duration (GB/s)
        roofline["traffic"] = round(tr["hbm_bytes_per_launch"] / (avg_ms * 1e-3) / 1e9, 1)
        roofline["traffic_detail"] = tr

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(vol_true, rot_all, df_all, M, args.cpu_images, scale, lam, alpha)

    tta = None
    if not args.no_tta:
        del run, x_b, y, acc, ws_bp, batches
        torch.cuda.empty_cache()
        from paper_2311_16100_amd import tta as TTA
        log = lambda m: print(m, file=sys.stderr, flush=True)
        params, _ = TTA.train_network(log=log)
        # the precomputed arm: the paper's 1000 epochs at 128^3; 100 epochs at
        # 256^3 (20 000 iterations) to keep the run within minutes
        tta = TTA.evaluate(params, configs=("mid_128", "hires_256", "mid_128_snr005"), log=log,
                           precomputed_epochs={"mid_128": 1000, "hires_256": 100, "mid_128_snr005": 1000})

    out = {
        "metric": METRIC,
        "value": round(Bsz / (ms_per_step * 1e-3), 1),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "hires_256: Algorithm 1 iteration (Hutchinson arm, 2 probes%s) per batch of "
                               "%d images of %dx%d (%d distinct resident batches in turn), %d^3 complex64 volume of %d "
                               "Gaussian blobs, N=%d, trilinear, CTF 300kV/Cs2.7/A0.1, defocus 1-3um"
                               % (", gradient and probe product in one kernel" if run_fused else "", Bsz, M, M, nb,
                                  M, W.n_blobs, N),
                   "global_batch": Bsz, "M": M, "deterministic": bool(args.deterministic),
                   "fused_gradient_probe": bool(run_fused), "line_search_halvings": halvings_timed},
        "fwd_adj_images_per_s": round(fwd_adj, 1),
        "fwd_adj_roofline": fwd_adj_roofline,
        "breakdown_ms": {k: round(v, 4) for k, v in ms.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_1e-2": tta,
    }
    print(json.dumps(out), flush=True)


TRAFFIC_SUMMARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "hbm_traffic_hires256.md")
KERNEL_SOURCES = ["brick_kernels.hip", "csg_device.h"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2311_16100_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_record(kernel, images, M, deterministic=False):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy kernel), or None when
    there is none for this kernel, mode (fast or fixed-point deterministic;
    a record without the field was taken on the fast path) and workload, or
    the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_SUMMARY) as fh:
            line = next(l for l in fh if l.startswith("traffic-record:"))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line.split(":", 1)[1])
    if rec.get("kernel") != kernel or rec.get("images") != images or rec.get("M") != M:
        return None
    if bool(rec.get("deterministic", False)) != bool(deterministic):
        return None
    if rec.get("sources_sha256") != kernel_sources_sha256():
        return None
    return {"hbm_bytes_per_launch": rec["fetch_bytes"] + rec["write_bytes"], "fetch_bytes": rec["fetch_bytes"],
            "write_bytes": rec["write_bytes"], "calibration": rec.get("calibration")}


def cpu_baseline(vol, rot_all, df_all, M, n_img, scale_full, lam, alpha):
    """One Algorithm 1 iteration of the FP64 oracle (Hutchinson arm, 2
    probes) on n_img images of the same workload, single-threaded."""
    import oracle
    from threadpoolctl import threadpool_limits
    grid, opt = oracle.Grid(M), oracle.Optics()
    P = oracle.Poses(rot_all[:n_img], df_all[:n_img])
    v_true = vol.astype(np.complex128)
    with threadpool_limits(limits=1):  # numpy's BLAS and OpenMP pools held to one thread
        x = oracle.project(grid, opt, P, v_true)
        st = oracle.Alg1State(v=np.zeros(M ** 3, np.complex128), D=np.ones(M ** 3), D_avg=np.zeros(M ** 3), eta=1.0)
        t1 = time.perf_counter()
        zHz = oracle.hutchinson_diag(grid, opt, P, 2, 4, scale_full, lam).reshape(-1)
        oracle.alg1_iteration(grid, opt, P, x, st, scale_full, lam, alpha, 0.9, 0.1, zHz=zHz)
        t2 = time.perf_counter()
    return {"value": round(n_img / (t2 - t1), 3), "unit": "images/s", "cores": 1, "kind": "oracle",
            "sample": "one Algorithm 1 iteration (2 probes) on %d images of the %d^3 workload, FP64 C + numpy, "
                      "single thread of %s (%d logical CPUs visible); %.1f s"
                      % (n_img, M, cpu_model(), os.cpu_count() or 0, t2 - t1)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


if __name__ == "__main__":
    main()
