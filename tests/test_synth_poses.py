"""Pins of the seeded pose generators shared by both sides.

* Haar-uniform rotations (normalised Gaussian quaternions): the mean of a
  Haar-distributed rotation matrix is zero, E[R_ij^2] = 1/3, and every
  sample is orthogonal with determinant +1.
* Preferred orientations: the viewing direction (row 2 of R) is von
  Mises-Fisher on S^2 with mean +z, whose mean cosine is the Langevin
  function coth(kappa) - 1/kappa; the in-plane angle is uniform, so the
  image axes (rows 0 and 1) average to zero.
"""
import math

import numpy as np

import synth


def _orthonormal(R):
    n = R.shape[0]
    RRt = np.einsum("nij,nkj->nik", R.astype(np.float64), R.astype(np.float64))
    assert np.max(np.abs(RRt - np.eye(3)[None])) < 2e-6
    assert np.allclose(np.linalg.det(R.astype(np.float64)), np.ones(n), atol=2e-6)


def test_haar_rotations_moments():
    n = 200_000
    R = synth.uniform_rotations(n, seed=11).astype(np.float64)
    _orthonormal(R[:2000])
    sd = 1.0 / math.sqrt(3.0 * n)  # standard deviation of the mean of one entry
    assert np.max(np.abs(R.mean(axis=0))) < 6 * sd
    assert np.allclose((R ** 2).mean(axis=0), 1.0 / 3.0, atol=6 * math.sqrt(4.0 / 45.0 / n))
    # the trace of a Haar rotation is 1 + 2 cos(angle) with the angle density
    # (1 - cos a) / pi on [0, pi]: E[tr R] = 0 and E[tr R^2] = 1
    tr = np.trace(R, axis1=1, axis2=2)
    assert abs(tr.mean()) < 6 * 1.0 / math.sqrt(n)
    assert abs((tr ** 2).mean() - 1.0) < 6 * math.sqrt(3.0 / n)


def test_vmf_rotations_mean_cosine():
    n = 200_000
    for kappa in (1.0, 10.0):
        R = synth.vmf_rotations(n, kappa, seed=12).astype(np.float64)
        _orthonormal(R[:2000])
        w = R[:, 2, 2]  # cosine between the viewing direction and +z
        langevin = 1.0 / math.tanh(kappa) - 1.0 / kappa
        # Var[w] = 1 - 2 L(kappa)/kappa - L(kappa)^2 for vMF on S^2
        var = 1.0 - 2.0 * langevin / kappa - langevin ** 2
        assert abs(w.mean() - langevin) < 6 * math.sqrt(var / n)
        # the azimuth of the viewing direction and the in-plane angle are uniform
        assert np.max(np.abs(R[:, 2, :2].mean(axis=0))) < 6 / math.sqrt(n)
        assert np.max(np.abs(R[:, :2, :].mean(axis=0))) < 6 / math.sqrt(n)
