"""Pins of the oracle's forward operator and its adjoint (Definition
"Projection operator" and eq. (fwd model), Sec. 2.1) against closed forms,
invariants and brute force.

* Fourier slice theorem, exact: for the 24 rotations of the cube every sample
  point R^T r is a grid point, so both interpolations must return the analytic
  2D transform of the projected Gaussian blobs (rotation convention, use of
  the rows of R, sign of the phase, centring).
* Fourier slice theorem, random rotations: the trilinear error stays under
  the tensor-product interpolation bound and is second order.
* Trilinear interpolation reproduces affine functions exactly (weights,
  corner indices, transposition).
* Nearest neighbour equals the brute-force argmin of the definition.
* Adjoint identity <A x, y> = <x, A^H y>, CTF powers.
* Hermitian symmetry of the slices of a real density.
* Discrete slice identity of the synthetic volume pipeline.
"""
import math

import numpy as np
import pytest

import synth


def analytic_blob_ft(blobs, kvec, M):
    """Continuous Fourier transform of the blob sum at frequencies kvec [...,3]
    (cycles per M voxels): a (2 pi s^2)^{3/2} exp(-2 pi^2 s^2 |k|^2 / M^2)
    exp(-2 pi i k.c / M)."""
    out = np.zeros(kvec.shape[:-1], dtype=np.complex128)
    k2 = np.sum(kvec ** 2, axis=-1)
    for c, s, a in zip(blobs.centres, blobs.sigmas, blobs.amps):
        out += a * (2 * np.pi * s * s) ** 1.5 * np.exp(-2 * np.pi ** 2 * s * s * k2 / M ** 2) \
            * np.exp(-2j * np.pi * (kvec @ c) / M)
    return out


def grid_k(M):
    ax = np.arange(M) - M // 2
    kz, ky, kx = np.meshgrid(ax, ax, ax, indexing="ij")
    return np.stack([kx, ky, kz], axis=-1).astype(np.float64)


def disk(M, r):
    ax = np.arange(M) - M // 2
    ky, kx = np.meshgrid(ax, ax, indexing="ij")
    return (kx ** 2 + ky ** 2) <= r * r, kx, ky


@pytest.mark.parametrize("interp", [0, 1])
def test_fourier_slice_exact_cube_group(orc, interp):
    M = 16
    blobs = synth.blob_params(M, 4, seed=11, sigma_range=(1.0, 2.0), centre_halfwidth=M / 8)
    vol = analytic_blob_ft(blobs, grid_k(M), M)
    rots = synth.cube_group()
    poses = orc.Poses(rots, np.zeros(len(rots), np.float32))
    grid = orc.Grid(M, interp=interp)
    out = orc.project(grid, orc.NO_CTF, poses, vol)
    mask, kx, ky = disk(M, grid.rmax)
    for i, R in enumerate(rots.astype(np.float64)):
        # projection of the density rotated by R: blob centres move to R c;
        # its 2D transform on the pixel grid
        exp2d = np.zeros((M, M), dtype=np.complex128)
        k2 = kx ** 2 + ky ** 2
        for c, s, a in zip(blobs.centres, blobs.sigmas, blobs.amps):
            rc = R @ c
            exp2d += a * (2 * np.pi * s * s) ** 1.5 * np.exp(-2 * np.pi ** 2 * s * s * k2 / M ** 2) \
                * np.exp(-2j * np.pi * (kx * rc[0] + ky * rc[1]) / M)
        got = out[i]
        assert np.all(got[~mask] == 0)
        err = np.linalg.norm(got[mask] - exp2d[mask]) / np.linalg.norm(exp2d[mask])
        assert err < 1e-12, (i, err)


def _smooth_fn(kvec, alphas, betas, amps):
    out = np.zeros(kvec.shape[:-1], dtype=np.complex128)
    for a, b, A in zip(alphas, betas, amps):
        out += A * np.exp(-a * np.sum(kvec ** 2, axis=-1)) * np.exp(-1j * (kvec @ b))
    return out


def _second_derivative_bound(p, alphas, betas, amps):
    """sqrt(2)/8 * sum_d sup over the cell of |d^2 phi / dk_d^2| for
    phi = sum A exp(-a|k|^2 - i b.k); sup bounded with |k_d| <= |p_d| + 1 and
    |k| >= |p| - sqrt(3)."""
    pa = np.abs(p)
    kmin = np.clip(np.linalg.norm(p, axis=-1) - math.sqrt(3), 0, None)
    tot = np.zeros(p.shape[:-1])
    for a, b, A in zip(alphas, betas, amps):
        env = abs(A) * np.exp(-a * kmin ** 2)
        for d in range(3):
            tot += env * (4 * a * a * (pa[..., d] + 1) ** 2 + b[d] ** 2 + 2 * a)
    return math.sqrt(2) / 8 * tot


def test_fourier_slice_random_rotations_bound_and_order(orc):
    M = 32
    g = np.random.default_rng(5)
    nb = 3
    alphas = g.uniform(0.004, 0.01, nb)
    betas = g.uniform(-0.3, 0.3, (nb, 3))
    amps = g.uniform(0.5, 1.0, nb) * np.exp(2j * np.pi * g.uniform(size=nb))
    rots = synth.uniform_rotations(6, seed=3)
    poses = orc.Poses(rots, np.zeros(6, np.float32))
    grid = orc.Grid(M)
    mask, kx, ky = disk(M, grid.rmax)
    # coarse: v[k] = phi(k); fine: v2[k] = phi(k/2) on a 2M grid, sampled at 2r
    v1 = _smooth_fn(grid_k(M), alphas, betas, amps)
    v2 = _smooth_fn(grid_k(2 * M) / 2.0, alphas, betas, amps)
    out1 = orc.project(grid, orc.NO_CTF, poses, v1)
    out2 = orc.project(orc.Grid(2 * M, r_max=2 * grid.rmax), orc.NO_CTF, poses, v2)
    e1_all, e2_all = [], []
    for i in range(6):
        R = rots[i].astype(np.float64)
        p = kx[..., None] * R[0] + ky[..., None] * R[1]
        exact = _smooth_fn(p, alphas, betas, amps)
        e1 = np.abs(out1[i] - exact)[mask]
        bound = _second_derivative_bound(p, alphas, betas, amps)[mask]
        assert np.all(e1 <= bound + 1e-14)
        # fine-grid pixel (2kx, 2ky) sits at index 2k + M on the 2M grid
        idx_y = 2 * ky + M
        idx_x = 2 * kx + M
        e2 = np.abs(out2[i][idx_y, idx_x] - exact)[mask]
        e1_all.append(e1)
        e2_all.append(e2)
    e1 = np.sqrt(np.mean(np.concatenate(e1_all) ** 2))
    e2 = np.sqrt(np.mean(np.concatenate(e2_all) ** 2))
    assert 3.0 < e1 / e2 < 5.0, e1 / e2


def test_trilinear_reproduces_affine(orc):
    M = 24
    a = np.array([0.3 - 0.2j, -1.1 + 0.5j, 0.7 + 0.9j])
    b = 2.0 - 1.0j
    kv = grid_k(M)
    vol = kv @ a + b
    rots = synth.uniform_rotations(8, seed=21)
    poses = orc.Poses(rots, np.zeros(8, np.float32))
    grid = orc.Grid(M)
    out = orc.project(grid, orc.NO_CTF, poses, vol)
    mask, kx, ky = disk(M, M // 2 - 2)  # all 8 corners inside the grid
    for i in range(8):
        R = rots[i].astype(np.float64)
        p = kx[..., None] * R[0] + ky[..., None] * R[1]
        want = p @ a + b
        assert np.max(np.abs(out[i][mask] - want[mask])) < 1e-12
    # partition of unity: a constant volume gives C_i at every interior pixel
    opt = orc.Optics()
    df = synth.defocus_values(8, 1.0, 3.0, seed=2)
    outc = orc.project(grid, opt, orc.Poses(rots, df), np.ones((M, M, M)))
    for i in range(8):
        for (yy, xx) in [(M // 2, M // 2), (M // 2 + 3, M // 2 - 5), (M // 2 - 7, M // 2 + 2)]:
            k2 = float((yy - M // 2) ** 2 + (xx - M // 2) ** 2)
            assert outc[i, yy, xx] == pytest.approx(orc.ctf(opt, M, float(df[i]), k2), abs=1e-13)


def test_nearest_neighbour_is_argmin(orc):
    M = 8
    vol = synth.random_complex((M, M, M), seed=4).astype(np.complex128)
    rots = synth.uniform_rotations(5, seed=8)
    poses = orc.Poses(rots, np.zeros(5, np.float32))
    grid = orc.Grid(M, interp=0)
    out = orc.project(grid, orc.NO_CTF, poses, vol)
    pts = grid_k(M).reshape(-1, 3)
    flat = vol.reshape(-1)
    mask, kx, ky = disk(M, grid.rmax)
    for i in range(5):
        R = rots[i].astype(np.float64)
        for yy, xx in zip(*np.nonzero(mask)):
            p = kx[yy, xx] * R[0] + ky[yy, xx] * R[1]
            k = np.argmin(np.sum((pts - p) ** 2, axis=1))
            assert out[i, yy, xx] == flat[k]


@pytest.mark.parametrize("interp", [0, 1])
def test_adjoint_identity(orc, interp):
    M, n = 16, 5
    grid = orc.Grid(M, interp=interp)
    opt = orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(n, seed=1), synth.defocus_values(n, 1.0, 3.0, seed=1))
    x = synth.random_complex((M, M, M), seed=2).astype(np.complex128)
    y = synth.random_complex((n, M, M), seed=3).astype(np.complex128)
    Ax = orc.project(grid, opt, poses, x)
    Ahy = orc.backproject(grid, opt, poses, y, ctf_power=1)
    lhs = np.vdot(Ax, y)
    rhs = np.vdot(x, Ahy)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)
    # the CTF powers of the adjoint: P^T C^2 P = (C P)^T (C P), and C^0 = no CTF
    z = synth.random_complex((M, M, M), seed=5).astype(np.complex128)
    lhs2 = orc.backproject(grid, opt, poses, orc.project(grid, orc.NO_CTF, poses, z), ctf_power=2)
    rhs2 = orc.backproject(grid, opt, poses, orc.project(grid, opt, poses, z), ctf_power=1)
    assert np.linalg.norm(lhs2 - rhs2) <= 1e-12 * np.linalg.norm(rhs2)
    b0 = orc.backproject(grid, opt, poses, y, ctf_power=0)
    b1 = orc.backproject(grid, orc.NO_CTF, poses, y, ctf_power=1)
    assert np.array_equal(b0, b1)
    # scale and accumulation
    b3 = orc.backproject(grid, opt, poses, y, ctf_power=1, scale=2.5, accum=x)
    assert np.linalg.norm(b3 - (x + 2.5 * Ahy)) <= 1e-13 * np.linalg.norm(b3)


def test_hermitian_symmetry_of_real_density(orc):
    M, n = 16, 4
    rho = np.random.default_rng(9).standard_normal((M, M, M))
    vol = synth.centred_fftn(rho)
    grid = orc.Grid(M)
    poses = orc.Poses(synth.uniform_rotations(n, seed=6), synth.defocus_values(n, 1.0, 3.0, seed=6))
    out = orc.project(grid, orc.Optics(), poses, vol)
    mask, kx, ky = disk(M, grid.rmax)
    for i in range(n):
        for yy, xx in zip(*np.nonzero(mask)):
            my, mx = M - yy, M - xx  # index of -k
            assert abs(out[i, my, mx] - np.conj(out[i, yy, xx])) < 1e-11 * max(1.0, abs(out[i, yy, xx]))


def test_discrete_slice_identity_of_volume_pipeline():
    M = 16
    rho = synth.blob_density(M, synth.blob_params(M, 5, seed=3))
    vol = synth.centred_fftn(rho)
    # projection along z <-> kz = 0 plane; along x <-> kx = 0 plane
    proj_z = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(rho.sum(axis=0))))
    assert np.max(np.abs(proj_z - vol[M // 2])) < 1e-10 * np.max(np.abs(proj_z))
    proj_x = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(rho.sum(axis=2))))
    assert np.max(np.abs(proj_x - vol[:, :, M // 2])) < 1e-10 * np.max(np.abs(proj_x))
    # and the analytic blob transform is its continuum limit for blobs that
    # are well sampled on both sides (no wrap-around, negligible aliasing)
    M2 = 32
    blobs = synth.blob_params(M2, 5, seed=3, sigma_range=(1.5, 2.5), centre_halfwidth=M2 / 8)
    an = analytic_blob_ft(blobs, grid_k(M2), M2)
    vol2 = synth.centred_fftn(synth.blob_density(M2, blobs))
    assert np.linalg.norm(an - vol2) / np.linalg.norm(an) < 1e-3


# ---------------------------------------------------------------------------
# In-plane shifts T_i (Definition "Projection operator", Sec. 2.1)
# ---------------------------------------------------------------------------
def test_shift_is_the_discrete_shift_theorem(orc):
    """An integer shift (sx, sy) multiplies the centred 2D transform so that
    the real-space image is translated by (sx, sy) pixels (np.roll), i.e.
    T_jj = exp(-2 pi i (kx sx + ky sy) / M)."""
    M, n = 16, 3
    grid = orc.Grid(M)
    rot = synth.uniform_rotations(n, seed=21)
    df = synth.defocus_values(n, 1.0, 3.0, seed=21)
    shifts = np.array([[2, -3], [-5, 1], [0, 4]], np.float32)
    vol = synth.random_complex((M, M, M), seed=22).astype(np.complex128)
    y0 = orc.project(grid, orc.Optics(), orc.Poses(rot, df), vol)
    y1 = orc.project(grid, orc.Optics(), orc.Poses(rot, df, shifts), vol)
    for i in range(n):
        real0 = np.fft.ifft2(np.fft.ifftshift(y0[i]))
        real1 = np.fft.ifft2(np.fft.ifftshift(y1[i]))
        sx, sy = int(shifts[i, 0]), int(shifts[i, 1])
        assert np.allclose(real1, np.roll(real0, (sy, sx), axis=(0, 1)), atol=1e-12 * np.abs(real0).max())


def test_fourier_slice_exact_with_shift(orc):
    """Cube-group rotations and fractional shifts: the slice of the analytic
    blob transform with the projected centres moved by the shift."""
    M = 16
    blobs = synth.blob_params(M, 4, seed=12, sigma_range=(1.0, 2.0), centre_halfwidth=M / 8)
    vol = analytic_blob_ft(blobs, grid_k(M), M)
    rots = synth.cube_group()
    shifts = np.random.default_rng(4).uniform(-3, 3, (len(rots), 2)).astype(np.float32)
    grid = orc.Grid(M)
    out = orc.project(grid, orc.NO_CTF, orc.Poses(rots, np.zeros(len(rots), np.float32), shifts), vol)
    mask, kx, ky = disk(M, grid.rmax)
    k2 = kx ** 2 + ky ** 2
    for i, R in enumerate(rots.astype(np.float64)):
        t = shifts[i].astype(np.float64)
        exp2d = np.zeros((M, M), dtype=np.complex128)
        for c, s, a in zip(blobs.centres, blobs.sigmas, blobs.amps):
            rc = R @ c
            exp2d += a * (2 * np.pi * s * s) ** 1.5 * np.exp(-2 * np.pi ** 2 * s * s * k2 / M ** 2) \
                * np.exp(-2j * np.pi * (kx * (rc[0] + t[0]) + ky * (rc[1] + t[1])) / M)
        err = np.linalg.norm(out[i][mask] - exp2d[mask]) / np.linalg.norm(exp2d[mask])
        assert err < 1e-12, (i, err)


@pytest.mark.parametrize("interp", [0, 1])
def test_adjoint_identity_with_shift_and_hessian_unchanged(orc, interp):
    M, n = 16, 5
    grid = orc.Grid(M, interp=interp)
    opt = orc.Optics()
    rot, df = synth.uniform_rotations(n, seed=31), synth.defocus_values(n, 1.0, 3.0, seed=31)
    shifts = np.random.default_rng(6).uniform(-6, 6, (n, 2)).astype(np.float32)
    P = orc.Poses(rot, df, shifts)
    x = synth.random_complex((M, M, M), seed=32).astype(np.complex128)
    y = synth.random_complex((n, M, M), seed=33).astype(np.complex128)
    lhs = np.vdot(orc.project(grid, opt, P, x), y)
    rhs = np.vdot(x, orc.backproject(grid, opt, P, y, ctf_power=1))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y) * n
    # T is unitary and diagonal: P^T T^* C^2 T P = P^T C^2 P (eq. (hessian))
    h_shift = orc.hvp(grid, opt, P, x, 1.0, 0.0)
    h_none = orc.hvp(grid, opt, orc.Poses(rot, df), x, 1.0, 0.0)
    assert np.linalg.norm(h_shift - h_none) <= 1e-12 * np.linalg.norm(h_none)
