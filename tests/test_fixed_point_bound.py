"""The constant behind the fixed-point accumulators of the adjoint.

A voxel receives a trilinear contribution from a pixel only if the pixel's
sample point lies within distance < 1 of it on every axis, i.e. inside the
open cube of side 2 around it.  The sample points of one image form a unit
square lattice on a plane through the grid centre (the rows e1, e2 of the
rotation).  Pick's theorem bounds the lattice points in a convex plane
section of area A by 2 A + 2, and a plane cuts the side-2 cube in at most
4 sqrt(2) (the diagonal rectangle), so at most 13 pixels of one image reach
one voxel.  The packed probe accumulator assumes 16 and the 64-bit
accumulators assume 32.  This test counts by brute force over random
rotations and voxel positions near the plane (no GPU).
"""
import numpy as np

import synth


def max_pixels_per_voxel(n_rot, n_vox, seed):
    rng = np.random.default_rng(seed)
    R = synth.uniform_rotations(n_rot, seed).reshape(n_rot, 3, 3).astype(np.float64)
    k = np.arange(-6, 7)
    kx, ky = np.meshgrid(k, k, indexing="ij")
    best = 0
    for i in range(n_rot):
        e1, e2, nrm = R[i, 0], R[i, 1], R[i, 2]
        pts = kx[..., None] * e1 + ky[..., None] * e2  # lattice around the origin
        # integer voxel offsets u with the cube u +- 1 meeting the plane
        for _ in range(n_vox):
            a, b = rng.integers(-3, 4, size=2)
            u0 = np.rint(a * e1 + b * e2 + rng.uniform(-1.7, 1.7) * nrm)
            inside = np.all(np.abs(pts - u0) < 1.0, axis=-1)
            best = max(best, int(inside.sum()))
    return best


def test_at_most_thirteen_pixels_of_one_image_reach_a_voxel():
    m = max_pixels_per_voxel(400, 40, 21)
    assert m <= 13
    # the section is large for some planes: the bound is not loose by much
    assert m >= 7


def test_axis_aligned_plane_reaches_four_pixels():
    # e1, e2 along x, y: the cube around a voxel on the plane holds the
    # lattice points with |kx|, |ky| < 1, i.e. only the voxel's own pixel;
    # half a step off the lattice it holds four
    pts = np.stack(np.meshgrid(np.arange(-3, 4), np.arange(-3, 4), indexing="ij"), -1).reshape(-1, 2)
    assert int(np.all(np.abs(pts - np.array([0.0, 0.0])) < 1, axis=1).sum()) == 1
    assert int(np.all(np.abs(pts - np.array([0.5, 0.5])) < 1, axis=1).sum()) == 4
