"""Conditioning of the reconstruction problem against resolution (Sec. 3.1,
Proposition "Condition number bound" and the figure that follows it).

With nearest-neighbour projections and no CTF the Hessian is diagonal,
H_jj = n_j + lambda, where n_j counts the image pixels assigned to voxel j
(equal to the voxel mapping set size |Omega_j| when no image maps two of its
pixels to one voxel, Assumptions 1).  Restricting the reconstruction to the
ball |k| <= R restricts H to the voxels of that ball, so

    kappa(R) = max_{|k|<=R} H_jj / min_{|k|<=R} H_jj.

The proposition bounds it from below by (N + lambda) / (p(R) N + lambda)
whenever 1 / p(R) <= N, and gives kappa = (N + lambda) / lambda when some
voxel of the ball receives no pixel.  p(R) is the ratio of image pixels to
volume voxels at radius R; the paper's figure computes it from the circular
and spherical shells of radius R (integer shells round(|k|) = R, about
1 / (2R)); the ratio of the disk to the ball of radius R (about 3 / (4R))
gives the weaker form of the same bound.  Both are reported.  The figure's
curve is the mean of kappa over 10 sets of N uniform orientations, with the
minimum and maximum as error bars.

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
    kappa: float      # max / min of H over the ball (the first pose set)
    bound: float      # lower bound of the proposition, p from the disk and the ball
    h_max: float
    h_min: float
    unseen: int       # voxels of the ball no pixel reaches
    p: float          # pixels of the disk / voxels of the ball
    bound_shell: float = 0.0  # the same with p from the shells of radius R
    p_shell: float = 0.0
    kappa_mean: float = 0.0   # over the pose sets
    kappa_min: float = 0.0
    kappa_max: float = 0.0
    sets: int = 1


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


def shell_point_counts(R: int):
    """Integer points with round(|k|) = R in the plane and in space
    (R - 1/2 <= |k| < R + 1/2, i.e. R^2 - R + 1 <= |k|^2 <= R^2 + R)."""
    a = np.arange(-R - 1, R + 2)
    lo, hi = R * R - R + 1, R * R + R
    d2 = a[:, None] ** 2 + a[None, :] ** 2
    disk = int(np.sum((d2 >= lo) & (d2 <= hi))) if R > 0 else 1
    d3 = d2[:, :, None] + a[None, None, :] ** 2
    ball = int(np.sum((d3 >= lo) & (d3 <= hi))) if R > 0 else 1
    return disk, ball


def _bound(N: int, lam: float, p: float) -> float:
    return (N + lam) / (p * N + lam) if 1.0 / p <= N else (N + lam) / lam


def kappa_bound(N: int, lam: float, R: int) -> tuple[float, float]:
    """The bound with p(R) from the disk and the ball of radius R."""
    disk, ball = disk_ball_counts(R)
    p = disk / ball
    return _bound(N, lam, p), p


def kappa_bound_shell(N: int, lam: float, R: int) -> tuple[float, float]:
    """The bound with p(R) from the shells of radius R (the paper's figure)."""
    px, pv = shell_point_counts(R)
    p = px / pv
    return _bound(N, lam, p), p


PAPER_RADII = (1,) + tuple(range(16, 305, 16))  # {1, 16, 32, ..., 304}


def kappa_vs_radius(N: int = 10000, radii=PAPER_RADII, lam: float = 1e-8, seed: int = 0, sets: int = 1,
                    device="cuda", progress=None) -> list[KappaRow]:
    """kappa(H) of the ball-restricted problem for each radius, from `sets`
    data sets (seeds seed, seed + 1, ...) of N full-resolution slices (grid
    side 2 max(R) + 2); `kappa` is the first set's, kappa_mean/min/max are
    over all sets."""
    Rm = max(radii)
    M = 2 * Rm + 2
    ax = torch.arange(M, device=device, dtype=torch.int32) - M // 2
    per_set = []
    first = []
    for sidx in range(sets):
        counts, _ = nn_counts(N, M, float(Rm), seed + sidx, device=device)
        ks = []
        for R in radii:
            lo, hi = M // 2 - R, M // 2 + R + 1
            sub = counts[lo:hi, lo:hi, lo:hi]
            a = ax[lo:hi]
            ball = (a[:, None, None] ** 2 + a[None, :, None] ** 2 + a[None, None, :] ** 2) <= R * R
            h = sub[ball].double() + lam
            ks.append(float((h.max() / h.min()).item()))
            if sidx == 0:
                first.append((float(h.max().item()), float(h.min().item()), int((sub[ball] == 0).sum().item())))
        per_set.append(ks)
        del counts
        if progress:
            progress("  conditioning: pose set %d of %d" % (sidx + 1, sets))
    rows = []
    for i, R in enumerate(radii):
        bound, p = kappa_bound(N, lam, R)
        bs, ps = kappa_bound_shell(N, lam, R)
        k = [per_set[j][i] for j in range(sets)]
        rows.append(KappaRow(R, k[0], bound, first[i][0], first[i][1], first[i][2], p, bs, ps,
                             float(np.mean(k)), float(np.min(k)), float(np.max(k)), sets))
    return rows


def z0_slice(N: int, M: int = 256, lam: float = 1e-8, seed: int = 0, device="cuda"):
    """The z = 0 plane (kz = 0) of the nearest-neighbour Hessian diagonal
    without CTF, H_jj = n_j + lambda, for N uniform slices on an M^3 grid
    (panels (b, c) of the paper's figure), and its radial profile: per integer
    radius round(|k|) of the plane, the mean of H and the fraction of voxels
    no pixel reaches."""
    counts, _ = nn_counts(N, M, float(M // 2 - 1), seed, device=device)
    plane = counts[M // 2].double() + lam
    ax = torch.arange(M, device=device) - M // 2
    r = torch.round(torch.sqrt((ax[:, None] ** 2 + ax[None, :] ** 2).double())).long()
    prof = []
    for R in range(M // 2):
        m = r == R
        v = plane[m]
        prof.append({"R": R, "mean": round(float(v.mean().item()), 6),
                     "unseen": round(float((v <= lam * 1.5).double().mean().item()), 6)})
    return plane.cpu().numpy(), prof


if __name__ == "__main__":
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="condition number against resolution (Sec. 3.1 figure)")
    ap.add_argument("--sets", type=int, default=10, help="pose sets for the mean and spread of kappa")
    ap.add_argument("--N", type=int, default=10000)
    ap.add_argument("--slices-out", default=None, help="save the z = 0 planes for N = 5 and 100 (.npz)")
    a = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    rows = kappa_vs_radius(N=a.N, sets=a.sets, progress=log)
    for r in rows:
        log("R=%3d kappa mean=%.4e [%.4e, %.4e] bound(shells)=%.4e bound(disk/ball)=%.4e unseen=%d" % (
            r.R, r.kappa_mean, r.kappa_min, r.kappa_max, r.bound_shell, r.bound, r.unseen))
    planes, profiles = {}, {}
    for n in (5, 100):
        planes["N%d" % n], profiles[n] = z0_slice(n)
    if a.slices_out:
        np.savez(a.slices_out, **planes)
    print(json.dumps({"kappa": [r.__dict__ for r in rows], "z0_profiles": profiles}))
