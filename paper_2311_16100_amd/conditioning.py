"""Conditioning of the reconstruction problem against resolution (Sec. 3.1,
Proposition "Condition number bound" and the figure that follows it).

With nearest-neighbour projections and no CTF the Hessian is diagonal,
H_jj = n_j + lambda, where n_j counts the image pixels assigned to voxel j
(equal to the voxel mapping set size |Omega_j| when no image maps two of its
pixels to one voxel, Assumptions 1).  Restricting the reconstruction to the
ball |k| <= R restricts H to the voxels of that ball, so

    kappa(R) = max_{|k|<=R} H_jj / min_{|k|<=R} H_jj.

The proposition bounds it from below by (N + lambda) / (p(R) N + lambda),
p(R) = (pixels of the disk of radius R) / (voxels of the ball of radius R),
whenever 1 / p(R) <= N, and gives kappa = (N + lambda) / lambda when some
voxel of the ball receives no pixel.

The counts come from the library's squared-weight backprojection
(csg_exact_diag on a nearest-neighbour grid without CTF) and the distinct-image
coverage (csg_features); the reductions over the ball are torch arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

import synth

from . import binding as B

CHUNK = 2048


@dataclass
class KappaRow:
    R: int
    kappa: float      # max / min of H over the ball
    bound: float      # lower bound of the proposition
    h_max: float
    h_min: float
    unseen: int       # voxels of the ball no pixel reaches
    p: float          # pixels of the disk / voxels of the ball


def nn_counts(N: int, M: int, r_max: float, seed: int, distinct: bool = False, device="cuda"):
    """Per-voxel pixel counts (sum over images of (P_i^T P_i)_jj) of N
    Haar-uniform nearest-neighbour slices on an M^3 grid; with `distinct`
    also the number of distinct images per voxel (|Omega_j|)."""
    grid = B.Grid(M, r_max=r_max, interp=0)
    rot = torch.from_numpy(synth.uniform_rotations(N, seed)).to(device)
    df = torch.zeros(N, dtype=torch.float32, device=device)
    n = torch.zeros((M,) * 3, dtype=torch.float32, device=device)
    tmp = torch.empty_like(n)
    ws = B.alloc_workspace(grid, min(N, CHUNK), B.CSG_WS_BACKPROJECT, device)
    for s in range(0, N, CHUNK):
        e = min(N, s + CHUNK)
        n += B.exact_diag(grid, B.NO_CTF, rot[s:e].contiguous(), df[s:e].contiguous(), 1.0, 0.0, diag_out=tmp,
                          workspace=ws)
    if not distinct:
        return n, None
    ctf2 = torch.zeros_like(n)
    cover = torch.zeros_like(n)
    for s in range(0, N, CHUNK):
        e = min(N, s + CHUNK)
        B.features(grid, B.NO_CTF, rot[s:e].contiguous(), df[s:e].contiguous(), ctf2, cover)
    return n, cover


def disk_ball_counts(R: int):
    """Integer points with x^2 + y^2 <= R^2 and with x^2 + y^2 + z^2 <= R^2."""
    a = np.arange(-R, R + 1)
    d2 = a[:, None] ** 2 + a[None, :] ** 2
    disk = int(np.sum(d2 <= R * R))
    ball = int(np.sum(d2[:, :, None] + a[None, None, :] ** 2 <= R * R))
    return disk, ball


def kappa_bound(N: int, lam: float, R: int) -> tuple[float, float]:
    disk, ball = disk_ball_counts(R)
    p = disk / ball
    if 1.0 / p <= N:
        return (N + lam) / (p * N + lam), p
    return (N + lam) / lam, p


def kappa_vs_radius(N: int = 10000, radii=tuple(range(1, 305, 16)), lam: float = 1e-8, seed: int = 0,
                    device="cuda") -> list[KappaRow]:
    """kappa(H) of the ball-restricted problem for each radius, from one
    data set of N full-resolution slices (grid side 2 max(R) + 2)."""
    Rm = max(radii)
    M = 2 * Rm + 2
    counts, _ = nn_counts(N, M, float(Rm), seed, device=device)
    ax = torch.arange(M, device=device, dtype=torch.int32) - M // 2
    rows = []
    for R in radii:
        lo, hi = M // 2 - R, M // 2 + R + 1
        sub = counts[lo:hi, lo:hi, lo:hi]
        a = ax[lo:hi]
        ball = (a[:, None, None] ** 2 + a[None, :, None] ** 2 + a[None, None, :] ** 2) <= R * R
        h = sub[ball].double() + lam
        bound, p = kappa_bound(N, lam, R)
        rows.append(KappaRow(R, float((h.max() / h.min()).item()), bound, float(h.max().item()),
                             float(h.min().item()), int((sub[ball] == 0).sum().item()), p))
    return rows


if __name__ == "__main__":
    import json
    import sys

    rows = kappa_vs_radius()
    for r in rows:
        print("R=%3d kappa=%.4e bound=%.4e h_max=%.0f h_min=%.3g unseen=%d" % (
            r.R, r.kappa, r.bound, r.h_max, r.h_min, r.unseen), file=sys.stderr, flush=True)
    print(json.dumps([r.__dict__ for r in rows]))
