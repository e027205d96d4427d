"""Learned preconditioner: a per-voxel regression of the Hessian diagonal
(the quantity Hutchinson's estimator targets, Sec. 3.2) from cheap features,
used in place of the on-the-fly estimate of Algorithm 1, with a short
Hutchinson estimate as judge and the Hutchinson arm as fallback.

Features of voxel k over the N images of a data set (csg_feature_sums):
  |k| / (M/2),  log(F2_k M / N),  log(F3_k M / N)
F2_k = sum_ij C_ij^2 w_ijk (CTF^2 weight), F3_k = sum_ij w_ijk, the
interpolation weight that reaches k (the pose coverage: for nearest-neighbour
stencils it counts the voxel mapping set of Sec. 3.1).
Target: log((D_k - lambda) M / N), D the Hutchinson estimate with many probes.
Prediction: D_k = lambda + (N / M) exp(net(features)) (csg_learned_diag).
The M / N scaling: the chance that an image reaches a voxel at a given
fraction of the maximum radius falls like 1/M, so the scaled quantities are
comparable across grid sizes and a network trained at 64^3 and 128^3 applies
at 256^3.

Training runs on the GPU through csg_mlp_grad / csg_mlp_adam.  Assembling
the training set (selecting voxels, taking logs) is host-side torch
arithmetic on the library's outputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

import synth

from . import binding as B
from .experiment import CHUNK, Dataset, ball_mask


def features(ds: Dataset, n_images: int | None = None, seed: int = 0):
    """(F2, F3) per image of the data set, i.e. the sums over the N images
    divided by N, in one scatter pass (csg_feature_sums): F2 = sum C^2 w,
    F3 = sum w.  With n_images < N the sums run over a uniform random subset
    of that many images (an unbiased estimate of the per-image means).
    Returned already multiplied back by N, so both cases have the same scale."""
    acc = torch.zeros((ds.M,) * 3, dtype=torch.complex64, device=ds.device)
    n = ds.N if n_images is None else min(ds.N, n_images)
    if n < ds.N:
        idx = torch.from_numpy(np.random.default_rng([seed, synth.STREAM_MISC]).choice(ds.N, n, replace=False)).to(
            ds.device)
        rot, df = ds.rot[idx].contiguous(), ds.defocus[idx].contiguous()
    else:
        rot, df = ds.rot, ds.defocus
    ws = B.alloc_workspace(ds.grid, min(n, CHUNK), B.CSG_WS_BACKPROJECT, ds.device)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        B.feature_sums(ds.grid, ds.optics, rot[s:e].contiguous(), df[s:e].contiguous(), acc, workspace=ws)
    f = ds.N / n
    return (acc.real * f).contiguous(), (acc.imag * f).contiguous()


def hutchinson_full(ds: Dataset, n_probe: int, seed: int, n_images: int | None = None, probe0: int = 0):
    """Hutchinson estimate of diag H over the data set (or an unbiased
    estimate from its first n_images images, rescaled by N / n_images)."""
    n = ds.N if n_images is None else min(ds.N, n_images)
    scale = ds.N / n
    d = torch.zeros((ds.M,) * 3, dtype=torch.float32, device=ds.device)
    ws = B.alloc_workspace(ds.grid, min(n, CHUNK), B.CSG_WS_HUTCHINSON, ds.device)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        d += B.hutchinson_diag(ds.grid, ds.optics, ds.rot[s:e].contiguous(), ds.defocus[s:e].contiguous(),
                               n_probe, seed, scale, 0.0, probe0=probe0, workspace=ws)
    return d + ds.lam


def inputs(M: int, N: int, ctf2: torch.Tensor, cover: torch.Tensor) -> torch.Tensor:
    dev = ctf2.device
    ax = (torch.arange(M, device=dev) - M // 2).float()
    k = torch.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2) / (M // 2)
    x1 = torch.log(torch.clamp(ctf2 * (M / N), min=1e-30))
    x2 = torch.log(torch.clamp(cover * (M / N), min=1e-30))
    return torch.stack([k, x1, x2], dim=-1).reshape(-1, 3).contiguous()


@dataclass
class TrainingSet:
    X: torch.Tensor  # float32 [n, 3]
    T: torch.Tensor  # float32 [n]


def training_set(ds: Dataset, n_probe: int = 200, seed: int = 0, max_samples: int = 200_000) -> TrainingSet:
    ctf2, cover = features(ds)
    D = hutchinson_full(ds, n_probe, seed)
    X = inputs(ds.M, ds.N, ctf2, cover)
    data = (D - ds.lam).reshape(-1)
    ok = (cover.reshape(-1) > 0) & (data > 0)
    idx = torch.nonzero(ok).reshape(-1)
    if idx.numel() > max_samples:
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        idx = idx[torch.randperm(idx.numel(), generator=g)[:max_samples].to(idx.device)]
    T = torch.log(data[idx] * (ds.M / ds.N)).float().contiguous()
    return TrainingSet(X[idx].contiguous(), T)


def train(sets, steps: int = 2000, batch: int = 8192, lr: float = 3e-3, seed: int = 0, device="cuda", log=None):
    """Adam on the mean squared error over the union of training sets."""
    X = torch.cat([s.X for s in sets]).contiguous()
    T = torch.cat([s.T for s in sets]).contiguous()
    n = X.shape[0]
    g = np.random.default_rng([seed, synth.STREAM_MLP])
    # He-style initialisation of the float32 master weights
    H = 64
    p = np.zeros(B.mlp_param_count(), np.float32)
    o = 0
    p[o:o + 3 * H] = g.standard_normal(3 * H) * math.sqrt(2.0 / 3); o += 3 * H
    o += H
    p[o:o + H * H] = g.standard_normal(H * H) * math.sqrt(2.0 / H); o += H * H
    o += H
    p[o:o + H] = g.standard_normal(H) * math.sqrt(1.0 / H); o += H
    p[o] = float(T.mean().item())
    params = torch.from_numpy(p).to(device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    hist = []
    nb = min(batch, n)
    ws = B.mlp_grad_workspace(nb, device)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float64, device=device)
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (nb,), generator=gen, device=device)
        B.mlp_grad(params, X[idx].contiguous(), T[idx].contiguous(), grad=grad, loss=loss, workspace=ws)
        lr_t = lr * (0.5 * (1 + math.cos(math.pi * step / steps)))  # cosine schedule
        B.mlp_adam(params, m, v, grad, step, lr_t)
        if step % 200 == 0 or step == steps:
            hist.append((step, loss.item()))
            if log:
                log("  mlp step %d loss %.4e" % (step, hist[-1][1]))
    return params, hist


def predict(ds: Dataset, params: torch.Tensor, ctf2=None, cover=None):
    if ctf2 is None:
        ctf2, cover = features(ds)
    return B.learned_diag(ds.grid, ds.N, ds.lam, params, ctf2, cover)


_SHELLS = {}


def _shell_order(M: int, device):
    """Voxels sorted by integer shell round(|k|) < M/2, with shell bounds."""
    key = (M, str(device))
    if key not in _SHELLS:
        ax = torch.arange(M, device=device) - M // 2
        r = torch.round(torch.sqrt((ax[:, None, None] ** 2 + ax[None, :, None] ** 2
                                    + ax[None, None, :] ** 2).float())).long().reshape(-1)
        order = torch.argsort(r, stable=True)
        rs = r[order]
        nsh = M // 2
        bounds = torch.searchsorted(rs, torch.arange(nsh + 1, device=device))
        _SHELLS[key] = (order, bounds)
    return _SHELLS[key]


def shell_stats(d: torch.Tensor, M: int):
    """(shell means, voxel counts) over integer shells round(|k|) < M/2,
    from prefix sums of the voxels sorted by shell."""
    order, bounds = _shell_order(M, d.device)
    vals = d.reshape(-1)[order].double()
    csum = torch.cat([torch.zeros(1, dtype=torch.float64, device=d.device), torch.cumsum(vals, 0)])
    sums = csum[bounds[1:]] - csum[bounds[:-1]]
    cnt = (bounds[1:] - bounds[:-1]).double()
    return sums / cnt, cnt


_SECTORS = {}


def sector_index(M: int, device):
    """Bin of every voxel: Fourier shell round(|k|) (< M/2, else -1) times 6
    plus the direction sector, the signed axis of the largest |k_d| (ties to
    the lower axis).  Within a shell the sectors separate directions, which
    preferred orientations make differ."""
    key = (M, str(device))
    if key not in _SECTORS:
        ax = torch.arange(M, device=device) - M // 2
        kz, ky, kx = torch.meshgrid(ax, ax, ax, indexing="ij")
        k = torch.stack([kx, ky, kz]).reshape(3, -1)
        shell = torch.round(torch.sqrt((k.double() ** 2).sum(0))).long()
        axis = torch.argmax(torch.abs(k), dim=0)
        sign = (torch.gather(k, 0, axis[None])[0] < 0).long()
        idx = shell * 6 + axis * 2 + sign
        idx[shell >= M // 2] = -1
        _SECTORS[key] = idx
    return _SECTORS[key]


def sector_stats(d: torch.Tensor, M: int):
    """(means, voxel counts) over the shell x direction-sector bins of
    sector_index (empty bins have count 0 and mean 0)."""
    idx = sector_index(M, d.device)
    keep = idx >= 0
    nb = (M // 2) * 6
    sums = torch.bincount(idx[keep], weights=d.reshape(-1)[keep].double(), minlength=nb)
    cnt = torch.bincount(idx[keep], minlength=nb).double()
    return sums / torch.clamp(cnt, min=1.0), cnt


def _binned_rel_error(a, b, n):
    return float((torch.sqrt(torch.sum(n * (a - b) ** 2)) / torch.sqrt(torch.sum(n * b * b))).item())


def judge(ds: Dataset, D_pred: torch.Tensor, n_probe: int = 2, n_images: int = 4096, seed: int = 99,
          detail: bool = False):
    """Relative error between the prediction and a short Hutchinson estimate
    (n_probe probes over n_images images, rescaled to the data set), on bin
    means weighted by their voxel counts, the larger of two binnings: the
    Fourier shells, and the shells split into six direction sectors (a
    prediction can match the shell means and still be wrong by direction,
    as with preferred orientations).  Bin means average out the probe noise
    of a short estimate; the count weights keep the few-voxel central bins
    from dominating.  detail=True also returns the two figures."""
    Dh = hutchinson_full(ds, n_probe, seed, n_images=n_images, probe0=1_000_000)
    a, n = shell_stats(D_pred, ds.M)
    b, _ = shell_stats(Dh, ds.M)
    e_shell = _binned_rel_error(a, b, n)
    a, n = sector_stats(D_pred, ds.M)
    b, _ = sector_stats(Dh, ds.M)
    e_sector = _binned_rel_error(a, b, n)
    e = max(e_shell, e_sector)
    return (e, e_shell, e_sector) if detail else e


def diag_rel_error(D_a: torch.Tensor, D_b: torch.Tensor, ds: Dataset) -> float:
    ball = ball_mask(ds.M, ds.grid.rmax, D_a.device)
    return float((torch.linalg.vector_norm((D_a - D_b)[ball]) / torch.linalg.vector_norm(D_b[ball])).item())
