"""Conditioning against resolution (Sec. 3.1, Proposition "Condition number
bound"): nearest-neighbour pixel counts from the library equal the oracle's
(integers, exact), the ball-restricted condition number obeys the
proposition's lower bound, and equals (N + lambda) / lambda once some voxel
of the ball is unseen (GPU)."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    from paper_2311_16100_amd import binding, conditioning
    binding.lib()
    return conditioning


def test_nn_counts_match_oracle(C):
    N, M = 40, 18
    counts, cover = C.nn_counts(N, M, float(M // 2 - 1), 3, distinct=True)
    P = oracle.Poses(synth.uniform_rotations(N, 3), np.zeros(N, np.float32))
    g = oracle.Grid(M, interp=0)
    ref = oracle.exact_diag(g, oracle.NO_CTF, P, 1.0, 0.0)
    _, ref_cover = oracle.features(g, oracle.NO_CTF, P)
    assert np.array_equal(counts.cpu().numpy().astype(np.float64), ref)
    assert np.array_equal(cover.cpu().numpy().astype(np.float64), ref_cover)
    # the centre voxel is reached by the zero-frequency pixel of every image
    assert counts[M // 2, M // 2, M // 2].item() == N


def test_kappa_obeys_bound(C):
    N, lam = 400, 1e-8
    rows = C.kappa_vs_radius(N=N, radii=(1, 4, 8, 12, 15), lam=lam, seed=5)
    for r in rows:
        # the centre voxel is seen by every image; without Assumptions 1 a
        # voxel may receive two pixels of one image, so the maximum is >= N
        assert r.h_max >= N - 1e-6
        assert r.kappa >= r.bound * (1 - 1e-9), r
    # growth with the radius
    ks = [r.kappa for r in rows]
    assert all(b >= a for a, b in zip(ks, ks[1:]))


def test_kappa_unseen_voxel(C):
    # five slices cannot cover a ball of radius 15 (more voxels than pixels)
    N, lam = 5, 1e-8
    (r,) = C.kappa_vs_radius(N=N, radii=(15,), lam=lam, seed=7)
    assert r.unseen > 0
    assert r.kappa == pytest.approx((N + lam) / lam, rel=1e-9)
    assert r.bound == pytest.approx((N + lam) / lam, rel=1e-12)


def test_z0_slice_matches_oracle(C):
    """Panels (b, c) of the figure: the kz = 0 plane of the nearest-neighbour
    Hessian diagonal, against the oracle's counts."""
    N, M, lam = 5, 24, 1e-8
    plane, prof = C.z0_slice(N, M=M, lam=lam, seed=11)
    P = oracle.Poses(synth.uniform_rotations(N, 11), np.zeros(N, np.float32))
    ref = oracle.exact_diag(oracle.Grid(M, interp=0), oracle.NO_CTF, P, 1.0, lam)
    assert np.allclose(plane, ref[M // 2], rtol=0, atol=1e-12)
    assert len(prof) == M // 2 and prof[0]["mean"] == pytest.approx(N + lam)


def test_kappa_spread_over_pose_sets(C):
    # kappa(R) is taken on the full-resolution grid of the largest radius, so
    # the single-set run uses the same radii
    rows = C.kappa_vs_radius(N=300, radii=(1, 6, 12), lam=1e-8, seed=21, sets=3)
    one = C.kappa_vs_radius(N=300, radii=(1, 6, 12), lam=1e-8, seed=21)
    for r, r1 in zip(rows, one):
        assert r.sets == 3 and r.kappa_min <= r.kappa_mean <= r.kappa_max
        assert r.kappa == pytest.approx(r1.kappa) and r1.kappa_mean == pytest.approx(r1.kappa)
