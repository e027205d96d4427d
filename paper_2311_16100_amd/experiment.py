"""Synthetic data sets, the ground truth v* and the time-to-accuracy runs of
the preconditioned SGD arms (Sec. 4 of the paper, with synthetic data in
place of its EMPIAR set).

Data: x_i = C_i P_i v_true + eta_i (eq. (fwd model)), v_true the Fourier
transform of a sum of Gaussian blobs, eta complex Gaussian of variance sigma^2
on the disk, sigma^2 = signal power / SNR.  The regularisation follows the
MAP reading lambda = sigma^2 / tau^2 (Sec. 3), tau^2 the mean power of v_true
on the ball; noise-free sets use a small lambda relative to the threshold.

Ground truth: v* solves H v = b (eq. (lin sys)) with all N images; it is
found with conjugate gradients (the paper uses L-BFGS on the same quadratic,
Sec. 4.1).  The CG vector algebra is ordinary torch arithmetic (evaluation,
not the method); every H v product is the library's HVP.

Arms (all share Algorithm 1's loop, the Armijo rule and the step schedule):
  plain        D_hat = 1
  hutchinson   D estimated on the fly (Algorithm 1)
  learned      D_hat = max(D_pred, alpha) from the preconditioner network
  precomputed  D_hat = max(|D|, alpha), D from eq. (diag est rule) run over
               many epochs before SGD starts (Sec. 4.1: 1000 epochs, batch
               1000), then held fixed
  exact        D_hat = max(diag H, alpha), diag H from one squared-weight
               backprojection: the exact diagonal, the limit the precomputed
               estimate approaches
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

import synth

from . import binding as B
from .sgd import Alg1Config, Alg1Runner

CHUNK = 2048  # images per library call when sweeping a whole data set


@dataclass
class Dataset:
    """Poses, defocus and ground truth of a synthetic data set, with its
    images either resident (`x`) or, for sets larger than device memory,
    regenerated batch by batch from v_true, with the noise of each image
    made on the device from (seed, image index) (synth.gpu_noise), so a
    regenerated image is always the same image."""
    grid: B.Grid
    optics: B.Optics
    rot: torch.Tensor
    defocus: torch.Tensor
    x: torch.Tensor | None
    v_true: torch.Tensor
    sigma2: float
    lam: float
    seed: int

    @property
    def N(self) -> int:
        return self.rot.shape[0]

    @property
    def M(self) -> int:
        return self.grid.M

    @property
    def device(self):
        return self.v_true.device

    @property
    def streamed(self) -> bool:
        return self.x is None

    def images(self, idx) -> torch.Tensor:
        """Images of the index tensor or slice `idx` (contiguous)."""
        if self.x is not None:
            return self.x[idx].contiguous()
        y = B.project(self.grid, self.optics, self.rot[idx].contiguous(), self.defocus[idx].contiguous(),
                      self.v_true)
        if self.sigma2 > 0:
            from synth import gpu_noise
            ii = torch.arange(*idx.indices(self.N), device=self.device) if isinstance(idx, slice) else idx
            gpu_noise.add_disk_noise(y, ii.to(torch.int64), int(math.floor(self.grid.rmax ** 2)), self.sigma2,
                                     gpu_noise.noise_seed(self.seed, synth.STREAM_NOISE))
        return y


def disk_mask(M: int, r: float, device) -> torch.Tensor:
    ax = torch.arange(M, device=device) - M // 2
    return (ax[:, None] ** 2 + ax[None, :] ** 2) <= r * r


def ball_mask(M: int, r: float, device) -> torch.Tensor:
    ax = torch.arange(M, device=device) - M // 2
    return (ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2) <= r * r


def make_dataset(M: int, N: int, n_blobs: int, seed: int, snr: float, defocus_um=(1.0, 3.0), poses="uniform",
                 kappa: float = 10.0, device="cuda", lam: float | None = None, stream: bool = False) -> Dataset:
    """stream=True keeps only poses and defocus resident and regenerates the
    images of each batch when they are needed (with their noise, made on the
    device per image).  The noise variance is sigma^2 = (mean signal power
    on the disk of the first 1024 images) / snr either way."""
    grid, optics = B.Grid(M), B.Optics()
    v_true = torch.from_numpy(synth.blob_volume(M, n_blobs, seed)).to(device)
    rot = synth.vmf_rotations(N, kappa, seed) if poses == "vmf" else synth.uniform_rotations(N, seed)
    rot = torch.from_numpy(rot).to(device)
    df = torch.from_numpy(synth.defocus_values(N, defocus_um[0], defocus_um[1], seed)).to(device)
    noisy = math.isfinite(snr) and snr > 0
    if stream:
        if not noisy:
            return Dataset(grid, optics, rot, df, None, v_true, 0.0, float(1e-3 if lam is None else lam), seed)
        n0 = min(N, 1024)
        pilot = B.project(grid, optics, rot[:n0].contiguous(), df[:n0].contiguous(), v_true)
        disk = disk_mask(M, grid.rmax, device)
        power = float((torch.abs(pilot) ** 2)[:, disk].mean().item())
        del pilot
        tau2 = float((torch.abs(v_true) ** 2)[ball_mask(M, grid.rmax, device)].mean().item())
        sigma2 = power / snr
        return Dataset(grid, optics, rot, df, None, v_true, sigma2, float(sigma2 / tau2 if lam is None else lam),
                       seed)
    x = torch.empty((N, M, M), dtype=torch.complex64, device=device)
    for s in range(0, N, CHUNK):
        e = min(N, s + CHUNK)
        B.project(grid, optics, rot[s:e].contiguous(), df[s:e].contiguous(), v_true, out=x[s:e])
    disk = disk_mask(M, grid.rmax, device)
    pilot = x[: min(N, 1024)]
    power = float((torch.abs(pilot) ** 2)[:, disk].mean().item())
    ball = ball_mask(M, grid.rmax, device)
    tau2 = float((torch.abs(v_true) ** 2)[ball].mean().item())
    if math.isfinite(snr) and snr > 0:
        sigma2 = power / snr
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed) * 1000 + synth.STREAM_NOISE)
        for s in range(0, N, CHUNK):
            e = min(N, s + CHUNK)
            noise = torch.randn((e - s, M, M, 2), generator=gen, device=device) * math.sqrt(sigma2 / 2)
            x[s:e] += torch.view_as_complex(noise) * disk
        lam_ = sigma2 / tau2 if lam is None else lam
    else:
        sigma2 = 0.0
        lam_ = 1e-3 if lam is None else lam
    return Dataset(grid, optics, rot, df, x, v_true, sigma2, float(lam_), seed)


def full_hvp(ds: Dataset, z: torch.Tensor, ws=None) -> torch.Tensor:
    """H z over all N images (scale 1)."""
    out = ds.lam * z
    for s in range(0, ds.N, CHUNK):
        e = min(ds.N, s + CHUNK)
        h = B.hvp(ds.grid, ds.optics, ds.rot[s:e].contiguous(), ds.defocus[s:e].contiguous(), z, 1.0, 0.0,
                  workspace=ws)
        out = out + h
    return out


def rhs(ds: Dataset) -> torch.Tensor:
    """b = sum_i P_i^T C_i x_i (eq. (lin sys) with the CTF)."""
    b = torch.zeros_like(ds.v_true)
    for s in range(0, ds.N, CHUNK):
        e = min(ds.N, s + CHUNK)
        B.backproject(ds.grid, ds.optics, ds.rot[s:e].contiguous(), ds.defocus[s:e].contiguous(),
                      ds.images(slice(s, e)), ctf_power=1, accum=b)
    return b


def exact_diagonal(ds: Dataset, scale: float = 1.0) -> torch.Tensor:
    """diag H = lambda + sum_ij C_ij^2 w_ijk^2 over all N images."""
    d = torch.zeros((ds.M,) * 3, dtype=torch.float32, device=ds.device)
    tmp = torch.empty_like(d)
    ws = B.alloc_workspace(ds.grid, min(ds.N, CHUNK), B.CSG_WS_BACKPROJECT, ds.device)
    for s in range(0, ds.N, CHUNK):
        e = min(ds.N, s + CHUNK)
        d += B.exact_diag(ds.grid, ds.optics, ds.rot[s:e].contiguous(), ds.defocus[s:e].contiguous(), scale, 0.0,
                          diag_out=tmp, workspace=ws)
    return d + ds.lam


def precomputed_diagonal(grid: B.Grid, optics: B.Optics, rot: torch.Tensor, defocus: torch.Tensor, lam: float,
                         epochs: int, batch: int, n_probe: int = 2, probe_seed: int = 0, perm_seed: int = 0,
                         beta: float = 0.9, progress=None):
    """The precomputed preconditioner of Sec. 4.1: the diagonal estimate of
    eq. (diag est rule), with Algorithm 1's running mean, run for `epochs`
    epochs of minibatches of `batch` images (a permutation per epoch) before
    SGD starts, from D = 1, D_avg = 0; iteration k's sample is the Hutchinson
    product of its minibatch with the probes (k-1) n_probe .. k n_probe - 1.
    Every step runs in the library (csg_hutchinson_diag, then the diagonal
    update of csg_precond_sgd_step).  Returns (D, D_avg, iterations)."""
    dev = rot.device
    N = rot.shape[0]
    M = grid.M
    scale = N / batch
    D = torch.ones((M, M, M), dtype=torch.float32, device=dev)
    D_avg = torch.zeros_like(D)
    zHz = torch.empty_like(D)
    ws = B.alloc_workspace(grid, batch, B.CSG_WS_HUTCHINSON, dev)
    k = 0
    t_log = time.perf_counter()
    for epoch in range(epochs):
        perm = torch.from_numpy(synth.epoch_permutation(N, perm_seed, epoch)).to(dev)
        for s in range(0, N - batch + 1, batch):
            idx = perm[s:s + batch]
            k += 1
            B.hutchinson_diag(grid, optics, rot[idx].contiguous(), defocus[idx].contiguous(), n_probe, probe_seed,
                              scale, lam, probe0=(k - 1) * n_probe, diag_out=zHz, workspace=ws)
            B.diag_update(D, D_avg, zHz, k, beta)
        if progress and time.perf_counter() - t_log > 30.0:
            t_log = time.perf_counter()
            progress("  precomputed diagonal: epoch %d of %d" % (epoch + 1, epochs))
    return D, D_avg, k


def ground_truth(ds: Dataset, tol: float = 1e-6, max_iter: int = 500, log=None):
    """v* = H^{-1} b by Jacobi-preconditioned CG (double-precision dots).
    Returns (v*, iterations, true relative residual ||b - H v*|| / ||b||).
    The error of v* is bounded by the residual times the condition number,
    so ill-conditioned sets need a small tolerance."""
    b = rhs(ds)
    dinv = 1.0 / exact_diagonal(ds)
    ws = B.alloc_workspace(ds.grid, min(ds.N, CHUNK), B.CSG_WS_GRADIENT, ds.device)
    x = torch.zeros_like(b)
    r = b.clone()
    z = dinv * r
    p = z.clone()
    rz = torch.vdot(r.reshape(-1).to(torch.complex128), z.reshape(-1).to(torch.complex128)).real
    bn = torch.linalg.vector_norm(b.to(torch.complex128))
    it = 0
    for it in range(max_iter):
        if torch.linalg.vector_norm(r.to(torch.complex128)) <= tol * bn:
            break
        if log and it % 20 == 0:
            log("  cg iteration %d residual %.3e" % (
                it, float((torch.linalg.vector_norm(r.to(torch.complex128)) / bn).item())))
        Ap = full_hvp(ds, p, ws)
        alpha = rz / torch.vdot(p.reshape(-1).to(torch.complex128), Ap.reshape(-1).to(torch.complex128)).real
        x = x + (alpha * p.to(torch.complex128)).to(torch.complex64)
        r = r - (alpha * Ap.to(torch.complex128)).to(torch.complex64)
        z = dinv * r
        rz_new = torch.vdot(r.reshape(-1).to(torch.complex128), z.reshape(-1).to(torch.complex128)).real
        p = z + (rz_new / rz).to(torch.float32) * p
        rz = rz_new
    # the true residual b - H x (the recursion accumulates float32 rounding)
    res = float((torch.linalg.vector_norm((b - full_hvp(ds, x, ws)).to(torch.complex128)) / bn).item())
    if log:
        log("  cg stopped after %d iterations, true residual %.3e" % (it, res))
    return x, it, res


def rel_error(v, v_star, ball) -> float:
    d = (v - v_star)[ball]
    return float((torch.linalg.vector_norm(d) / torch.linalg.vector_norm(v_star[ball])).item())


@dataclass
class RunResult:
    arm: str
    reached: bool
    iterations: int
    seconds: float
    setup_seconds: float
    errors: list = field(default_factory=list)  # (iteration, seconds, ball error, high-band error)
    halvings: int = 0
    capped: int = 0
    gen_seconds: float = 0.0  # regeneration of streamed images (not in `seconds`)
    eval_seconds: float = 0.0  # error evaluations (not in `seconds`)
    fsc: list = field(default_factory=list)  # (iteration, FSC per shell vs v*) at epoch ends and at the stop
    note: str = ""

    @property
    def total_seconds(self) -> float:
        return self.setup_seconds + self.seconds


def high_band_mask(M: int, r_max: float, device) -> torch.Tensor:
    """Voxels with M/4 <= |k| <= r_max: the high-resolution half of the ball."""
    ax = torch.arange(M, device=device) - M // 2
    k2 = ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2
    return (k2 >= (M / 4) ** 2) & (k2 <= r_max * r_max)


def save_checkpoint(path: str, arrays: dict, meta: dict):
    """Arrays and a JSON record in one .npz (read back without pickle)."""
    import json
    np.savez(path, __meta__=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8), **arrays)


def load_checkpoint(path: str):
    import json
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(bytes(z["__meta__"]).decode())
        arrays = {k: z[k].copy() for k in z.files if k != "__meta__"}
    return arrays, meta


def run_arm(ds: Dataset, v_star: torch.Tensor, arm: str, batch: int, target: float = 1e-2, max_epochs: int = 20,
            eval_every: int = 1, eta0: float = 1.0, decay_epochs: int = 0, D_fixed=None, setup_seconds: float = 0.0,
            seed: int = 0, time_limit: float = 120.0, n_probe: int = 2, stop_on: str = "ball",
            deterministic: bool = False, progress=None, queue_probes: bool = True, fused: bool = True,
            average_from_epoch: int | None = None, fsc_every: int = 0, checkpoint: str | None = None,
            checkpoint_every: int = 0, resume: str | None = None, stop_at: int | None = None) -> RunResult:
    """Algorithm 1 from v = 0 until the relative error of `stop_on` ("ball":
    the whole ball |k| <= r_max; "high": M/4 <= |k| <= r_max) is <= target,
    evaluated every `eval_every` iterations.
    `decay_epochs` > 0 halves the step-size cap every that many epochs, and
    `average_from_epoch` (not None) keeps from that epoch on the running
    (Polyak-Ruppert) average of the iterates, whose error is then the one
    reported and tested; both identically in every arm (a schedule for noisy
    data; Algorithm 1 itself has neither).  Wall time counts the iterations
    (and the averaging); the error evaluations are timed apart (`eval_seconds`)
    and not counted, and for a streamed data set neither is the regeneration
    of each batch's images (`gen_seconds`).
    `deterministic` selects the bitwise-reproducible adjoint.  `fused` (fast
    adjoint only) has the Hutchinson arm form each iteration's gradient and
    probe product in one call; otherwise, with `queue_probes`, the runner is
    told the next batch's poses and computes that batch's probe product
    during the line search.
    The shell correlation with v* is recorded after every epoch, at the stop,
    and every `fsc_every` iterations if that is > 0 (outside the timing).
    Checkpoints: with `checkpoint` a path, the run's state (iterate, diagonal
    estimate, step size, iteration counter, position in the epoch, averaging
    and the results so far) is written there every `checkpoint_every`
    iterations and when `stop_at` iterations are done (the run then returns,
    note "stopped"); `resume` continues from such a file.  The minibatch order
    (a permutation per epoch) and the probes (numbered by iteration) are
    functions of the seeds and counters, so a resumed run takes the same
    minibatches and probes as an uninterrupted one."""
    dev = ds.device
    scale = ds.N / batch
    alpha = B.threshold_alpha(ds.grid, ds.optics, ds.rot, ds.defocus, ds.lam).item()
    cfg = Alg1Config(eta0=eta0, n_probe=n_probe, probe_seed=seed + 17, deterministic=deterministic, fused=fused)
    kind = {"plain": "plain", "hutchinson": "hutchinson", "learned": "fixed", "exact": "fixed",
            "precomputed": "fixed"}[arm]
    v0 = torch.zeros_like(v_star)
    run = Alg1Runner(ds.grid, ds.optics, kind, scale, ds.lam, alpha, cfg, v0, D_fixed=D_fixed, batch=batch)
    ball = ball_mask(ds.M, ds.grid.rmax, dev)
    high = high_band_mask(ds.M, ds.grid.rmax, dev)
    res = RunResult(arm, False, 0, 0.0, setup_seconds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_log = t0
    it = 0
    eta_cap = eta0
    v_avg = None  # Polyak-Ruppert average of the iterates
    n_avg = 0
    start_epoch, start_s = 0, 0
    if resume:
        arrays, meta = load_checkpoint(resume)
        if meta["arm"] != arm or meta["batch"] != batch or meta["N"] != ds.N or meta["M"] != ds.M:
            raise ValueError("checkpoint %s is for another run" % resume)
        run.load_state_dict({"arrays": {k: arrays[k] for k in ("v", "D", "D_avg") if k in arrays},
                             **{k: meta[k] for k in ("eta", "k", "capped", "halvings")}})
        it, eta_cap, n_avg = meta["it"], meta["eta_cap"], meta["n_avg"]
        start_epoch, start_s = meta["epoch"], meta["s"]
        if "v_avg" in arrays:
            v_avg = torch.from_numpy(arrays["v_avg"]).to(dev)
        res.errors = [tuple(e) for e in meta["errors"]]
        res.fsc = [(i, f) for i, f in meta["fsc"]]
        res.halvings, res.gen_seconds, res.eval_seconds = meta["halvings_sum"], meta["gen_s"], meta["eval_s"]
        t0 -= meta["seconds"]  # continue the wall-time count

    def write_checkpoint(epoch, s_next):
        torch.cuda.synchronize()
        tc = time.perf_counter()
        sd = run.state_dict()
        arrays = dict(sd["arrays"])
        if v_avg is not None:
            arrays["v_avg"] = v_avg.cpu().numpy()
        meta = {"arm": arm, "batch": batch, "N": ds.N, "M": ds.M, "epoch": epoch, "s": s_next, "it": it,
                "eta_cap": eta_cap, "n_avg": n_avg, "eta": sd["eta"], "k": sd["k"], "capped": sd["capped"],
                "halvings": sd["halvings"], "errors": res.errors, "fsc": res.fsc, "halvings_sum": res.halvings,
                "gen_s": res.gen_seconds, "eval_s": res.eval_seconds,
                "seconds": tc - t0 - res.gen_seconds - res.eval_seconds}
        save_checkpoint(checkpoint, arrays, meta)
        return time.perf_counter() - tc

    def evaluate(now):
        """Record the error (of the average, when averaging) at `now`; the
        evaluation's own time is added to res.eval_seconds."""
        torch.cuda.synchronize()
        te = time.perf_counter()
        el = now - t0 - res.gen_seconds - res.eval_seconds
        v_eval = v_avg if v_avg is not None else run.state.v
        eb = rel_error(v_eval, v_star, ball)
        eh = rel_error(v_eval, v_star, high)
        res.errors.append((it, el, eb, eh))
        res.eval_seconds += time.perf_counter() - te
        return el, (eb if stop_on == "ball" else eh), v_eval

    def poses_of(idx):
        return ds.rot[idx].contiguous(), ds.defocus[idx].contiguous()

    # the poses of the current and the next batch: the next ones let the
    # Hutchinson arm compute its next probe product during the line search
    cur = None
    perm_next = None
    for epoch in range(start_epoch, max_epochs):
        if decay_epochs and epoch > 0 and epoch % decay_epochs == 0 and not (resume and epoch == start_epoch
                                                                             and start_s > 0):
            eta_cap *= 0.5
            run.state.eta = min(run.state.eta, eta_cap)
        perm = perm_next if perm_next is not None else torch.from_numpy(
            synth.epoch_permutation(ds.N, seed, epoch)).to(dev)
        perm_next = None
        first_s = start_s if epoch == start_epoch else 0
        for s in range(first_s, ds.N - batch + 1, batch):
            idx = perm[s:s + batch]
            if cur is None:
                cur = poses_of(idx)
            if not queue_probes:
                nxt = None
            elif s + 2 * batch <= ds.N:
                nxt = poses_of(perm[s + batch:s + 2 * batch])
            elif epoch + 1 < max_epochs:
                perm_next = torch.from_numpy(synth.epoch_permutation(ds.N, seed, epoch + 1)).to(dev)
                nxt = poses_of(perm_next[:batch])
            else:
                nxt = None
            if ds.streamed:
                torch.cuda.synchronize()
                tg = time.perf_counter()
                xb = ds.images(idx)
                torch.cuda.synchronize()
                res.gen_seconds += time.perf_counter() - tg
            else:
                xb = ds.images(idx)
            res.halvings += run.iteration(cur[0], cur[1], xb, next_poses=nxt)
            cur = nxt
            del xb
            it += 1
            if average_from_epoch is not None and epoch >= average_from_epoch:
                n_avg += 1
                if v_avg is None:
                    v_avg = run.state.v.clone()
                else:
                    v_avg.lerp_(run.state.v, 1.0 / n_avg)
            if progress and time.perf_counter() - t_log > 30.0:
                t_log = time.perf_counter()
                progress("  %s: iteration %d, %.1f s" % (arm, it, t_log - t0 - res.gen_seconds - res.eval_seconds))
            if checkpoint and ((checkpoint_every and it % checkpoint_every == 0) or it == stop_at):
                nxt_s = s + batch
                ce, cs = (epoch, nxt_s) if nxt_s <= ds.N - batch else (epoch + 1, 0)
                t0 += write_checkpoint(ce, cs)
            if stop_at is not None and it >= stop_at:
                res.iterations, res.note = it, "stopped"
                res.seconds = time.perf_counter() - t0 - res.gen_seconds - res.eval_seconds
                res.capped = run.state.capped
                return res
            if fsc_every and it % fsc_every == 0:
                tf = time.perf_counter()
                res.fsc.append((it, B.fsc(ds.grid, v_avg if v_avg is not None else run.state.v,
                                          v_star).cpu().tolist()))
                t0 += time.perf_counter() - tf
            if it % eval_every == 0:
                el, e_stop, v_eval = evaluate(time.perf_counter())
                if e_stop <= target:
                    res.reached, res.iterations, res.seconds = True, it, el
                    res.capped = run.state.capped
                    res.fsc.append((it, B.fsc(ds.grid, v_eval, v_star).cpu().tolist()))
                    return res
                if el > time_limit:
                    res.iterations, res.seconds, res.note = it, el, "time limit"
                    res.capped = run.state.capped
                    res.fsc.append((it, B.fsc(ds.grid, v_eval, v_star).cpu().tolist()))
                    return res
        # shell correlation with v* after each epoch (Sec. 4.1), outside the timed region
        if not (res.fsc and res.fsc[-1][0] == it):
            tf = time.perf_counter()
            res.fsc.append((it, B.fsc(ds.grid, v_avg if v_avg is not None else run.state.v,
                                      v_star).cpu().tolist()))
            t0 += time.perf_counter() - tf
    res.iterations, res.note = it, "epoch limit"
    res.seconds = time.perf_counter() - t0 - res.gen_seconds - res.eval_seconds
    res.capped = run.state.capped
    if not res.errors or res.errors[-1][0] != it:
        evaluate(time.perf_counter())
    return res


def compare_diagonals(D_est: torch.Tensor, D_ref: torch.Tensor, ds: Dataset) -> dict:
    """How far an estimated diagonal is from a reference one: relative L2
    over the ball, and the relative error of the Fourier-shell means (largest
    over the shells and count-weighted)."""
    from . import learned as L
    a, n = L.shell_stats(D_est, ds.M)
    b, _ = L.shell_stats(D_ref, ds.M)
    shell_rel = torch.abs(a - b) / torch.abs(b)
    return {"ball_rel_l2": round(L.diag_rel_error(D_est, D_ref, ds), 6),
            "shell_mean_rel_max": round(float(shell_rel.max().item()), 6),
            "shell_mean_rel_weighted": round(float((torch.sqrt(torch.sum(n * (a - b) ** 2))
                                                     / torch.sqrt(torch.sum(n * b * b))).item()), 6)}


def compare_arms(ds: Dataset, batch: int, params=None,
                 arms=("plain", "hutchinson", "learned", "precomputed", "exact"),
                 target: float = 1e-2, stop_on: str = "ball", judge_threshold: float = 0.2, log=print,
                 feature_images: int = 8192, judge_images: int = 4096, cg_tol: float = 1e-6, cg_max_iter: int = 500,
                 precomputed_epochs: int = 1000, precomputed_batch: int = 1000, v_star=None, cache=None, **kw):
    """Time to `target` for each arm on the same data set and ground truth.
    Setup time is charged to the arm that needs it: the exact arm one
    squared-weight pass over the data; the precomputed arm its
    `precomputed_epochs` epochs of eq. (diag est rule) at batch
    `precomputed_batch` (reported, as in the paper, as a precomputation); the
    learned arm the feature pass (over `feature_images` random images), the
    network and the judge (one complex probe over `judge_images` images); if
    the judge rejects the prediction the arm continues as the Hutchinson arm.
    The precomputed and learned diagonals are also compared with the exact
    one.  `v_star` = (v*, CG iterations, residual) reuses a ground truth;
    `cache` (a dict) keeps the precomputed diagonal and its setup time for
    later calls on the same data set."""
    from . import learned as L
    if v_star is None:
        v_star = ground_truth(ds, tol=cg_tol, max_iter=cg_max_iter, log=log if ds.N * ds.M ** 2 > 10 ** 10 else None)
    v_star, cg_it, cg_res = v_star
    # one untimed pass through every setup kernel on a few images, so that no
    # arm is charged for first-launch costs
    few = min(ds.N, 64)
    B.exact_diag(ds.grid, ds.optics, ds.rot[:few].contiguous(), ds.defocus[:few].contiguous(), 1.0, 0.0)
    if params is not None:
        c2, cv = L.features(ds, n_images=few)
        L.judge(ds, L.predict(ds, params, c2, cv), n_images=few)
    torch.cuda.synchronize()
    out = {"cg_iterations": cg_it, "cg_residual": cg_res, "arms": {}, "diagonals": {}}
    D_exact = None
    for arm in arms:
        D = None
        setup = 0.0
        note = ""
        run_as = arm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if arm == "exact":
            D = exact_diagonal(ds)
        elif arm == "precomputed":
            if cache is not None and "precomputed" in cache:
                D, setup, note = cache["precomputed"]
            else:
                D, _, n_it = precomputed_diagonal(ds.grid, ds.optics, ds.rot, ds.defocus, ds.lam, precomputed_epochs,
                                                  min(precomputed_batch, ds.N), probe_seed=ds.seed + 29,
                                                  perm_seed=ds.seed + 31, progress=log)
                note = "%d epochs x batch %d (%d iterations)" % (precomputed_epochs, min(precomputed_batch, ds.N),
                                                                 n_it)
        elif arm == "learned":
            if params is None:
                continue
            ctf2, cover = L.features(ds, n_images=feature_images)
            D = L.predict(ds, params, ctf2, cover)
            err = L.judge(ds, D, n_images=judge_images)
            note = "judge %.3f" % err
            if not math.isfinite(err) or err > judge_threshold:
                run_as, D, note = "hutchinson", None, note + " -> fallback to hutchinson"
        torch.cuda.synchronize()
        if not (arm == "precomputed" and cache is not None and "precomputed" in cache):
            setup = time.perf_counter() - t0
        if arm == "precomputed" and cache is not None:
            cache["precomputed"] = (D, setup, note)
        if D is not None and arm in ("precomputed", "learned"):
            if D_exact is None:
                D_exact = exact_diagonal(ds)
            out["diagonals"][arm] = compare_diagonals(D, D_exact, ds)
        r = run_arm(ds, v_star, run_as, batch, target=target, D_fixed=D, setup_seconds=setup, stop_on=stop_on,
                    progress=log, **kw)
        r.arm, r.note = arm, (r.note + " " + note).strip()
        out["arms"][arm] = r
        if log:
            log("  %-10s reached=%s it=%d run=%.3fs setup=%.3fs total=%.3fs %s" % (
                arm, r.reached, r.iterations, r.seconds, r.setup_seconds, r.total_seconds, r.note))
    return out
