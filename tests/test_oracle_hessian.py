"""Pins of the oracle's Hessian, Hutchinson estimator, features, threshold,
Algorithm 1 and ground-truth solver (Sec. 3).

* 8^3 dense Hessian: the forward operator is assembled column by column and
  H = s A^T A + lambda I is formed with a plain matrix product; the HVP and
  the squared-weight diagonal must equal it (eq. (hessian)).
* Nearest neighbour: H is diagonal and H_kk = s sum_{(i,j) -> k} C_ij^2 +
  lambda with the brute-force argmin map (eqs. (pp), (H diag)); one Rademacher
  probe returns it exactly (Remark after Fig. 2).
* Trilinear: the Hutchinson mean lies within the closed-form Rademacher
  deviation of the exact diagonal.
* Proposition "Condition number bound" for nearest neighbour without CTF.
* Algorithm 1 reaches v* in one step when the preconditioner is the exact
  diagonal of a diagonal H and eta = 1; its invariants hold in general.
* Central finite differences of the loss give the gradient.
* CG against a dense solve; FSC identities; shell counts of eq. (thresh value).
"""
import math

import numpy as np
import pytest

import synth


def dense_A(orc, grid, optics, poses):
    """Columns of the (real) forward operator, shape [n*M*M, M^3]."""
    M = grid.M
    nv = M ** 3
    A = np.zeros((poses.n * M * M, nv))
    e = np.zeros(nv)
    for k in range(nv):
        e[:] = 0
        e[k] = 1.0
        col = orc.project(grid, optics, poses, e)
        assert np.all(col.imag == 0)
        A[:, k] = col.real.reshape(-1)
    return A


def nn_argmin_map(M, R, rmax):
    ax = np.arange(M) - M // 2
    kz, ky, kx = np.meshgrid(ax, ax, ax, indexing="ij")
    pts = np.stack([kx, ky, kz], -1).reshape(-1, 3).astype(float)
    out = []
    for y in ax:
        for x in ax:
            if x * x + y * y > rmax * rmax:
                continue
            p = x * R[0] + y * R[1]
            out.append(((y, x), int(np.argmin(np.sum((pts - p) ** 2, axis=1)))))
    return out


@pytest.fixture(scope="module")
def small_problem(orc):
    M, n = 8, 6
    grid = orc.Grid(M, interp=1)
    opt = orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(n, seed=31), synth.defocus_values(n, 1.0, 3.0, seed=31))
    A = dense_A(orc, grid, opt, poses)
    return grid, opt, poses, A


def test_dense_hessian_hvp_and_diag(orc, small_problem):
    grid, opt, poses, A = small_problem
    scale, lam = 3.0, 0.25
    H = scale * A.T @ A + lam * np.eye(A.shape[1])
    z = synth.random_complex(grid.M ** 3, seed=12).astype(np.complex128)
    hz = orc.hvp(grid, opt, poses, z, scale, lam).reshape(-1)
    assert np.linalg.norm(hz - H @ z) <= 1e-12 * np.linalg.norm(H @ z)
    d = orc.exact_diag(grid, opt, poses, scale, lam).reshape(-1)
    assert np.max(np.abs(d - np.diag(H))) <= 1e-12 * np.max(np.diag(H))
    # features: CTF^2 weight = row sums of the data Hessian; coverage = number
    # of images whose operator has a nonzero entry in the voxel's column
    f2, f3 = orc.features(grid, opt, poses)
    data_H = A.T @ A
    assert np.max(np.abs(f2.reshape(-1) - data_H.sum(axis=1))) <= 1e-12 * data_H.sum(axis=1).max()
    Mx = grid.M ** 2
    cover = np.zeros(grid.M ** 3)
    A_noctf = dense_A(orc, grid, orc.NO_CTF, poses)
    for i in range(poses.n):
        cover += np.any(A_noctf[i * Mx:(i + 1) * Mx] != 0, axis=0)
    assert np.array_equal(f3.reshape(-1), cover)


def test_nearest_neighbour_hessian_is_diagonal_and_counts(orc):
    M, n = 8, 7
    grid = orc.Grid(M, interp=0)
    opt = orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(n, seed=41), synth.defocus_values(n, 1.0, 3.0, seed=41))
    A = dense_A(orc, grid, opt, poses)
    scale, lam = 2.0, 0.5
    H = scale * A.T @ A + lam * np.eye(M ** 3)
    assert np.count_nonzero(H - np.diag(np.diag(H))) == 0
    want = np.full(M ** 3, lam)
    for i in range(n):
        R = poses.rot[i].astype(np.float64)
        for (y, x), k in nn_argmin_map(M, R, grid.rmax):
            want[k] += scale * orc.ctf(opt, M, float(poses.defocus[i]), float(x * x + y * y)) ** 2
    assert np.max(np.abs(np.diag(H) - want)) <= 1e-12 * want.max()
    # one Rademacher probe is exact for a diagonal H
    d1 = orc.hutchinson_diag(grid, opt, poses, n_probe=1, seed=5, scale=scale, lam=lam).reshape(-1)
    assert np.max(np.abs(d1 - want)) <= 1e-12 * want.max()


def test_hutchinson_within_rademacher_deviation(orc, small_problem):
    grid, opt, poses, A = small_problem
    scale, lam = 1.0, 0.1
    H = scale * A.T @ A + lam * np.eye(A.shape[1])
    P = 200
    est = orc.hutchinson_diag(grid, opt, poses, n_probe=P, seed=77, scale=scale, lam=lam).reshape(-1)
    off = H - np.diag(np.diag(H))
    # z_k (H z)_k - H_kk = sum_{l != k} H_kl z_k z_l has variance sum_{l!=k} H_kl^2
    sd = np.sqrt(np.sum(off ** 2, axis=1) / P)
    assert np.all(np.abs(est - np.diag(H)) <= 5 * sd + 1e-12)
    # the estimate is unbiased: the error shrinks like 1/sqrt(P)
    est_small = orc.hutchinson_diag(grid, opt, poses, n_probe=8, seed=78, scale=scale, lam=lam).reshape(-1)
    assert np.linalg.norm(est - np.diag(H)) < np.linalg.norm(est_small - np.diag(H))


def test_condition_number_bound_nearest_neighbour(orc):
    # Proposition "Condition number bound" in its eq. (cond number p) form, on
    # the ball of radius R = r_max: kappa >= (N + lambda) / (p(R) N + lambda).
    M, N, lam = 16, 40, 1e-8
    grid = orc.Grid(M, interp=0)
    poses = orc.Poses(synth.uniform_rotations(N, seed=51), np.zeros(N, np.float32))
    d = orc.exact_diag(grid, orc.NO_CTF, poses, 1.0, lam)
    c = M // 2
    # the centre voxel is hit by exactly one pixel of every image
    assert d[c, c, c] == pytest.approx(N + lam, rel=1e-15)
    ball = synth.ball_mask(M, grid.rmax)
    n_pix = sum(1 for y in range(-c, c) for x in range(-c, c) if x * x + y * y <= grid.rmax ** 2)
    p = n_pix / ball.sum()
    kappa = d[ball].max() / d[ball].min()
    assert d[ball].max() == pytest.approx(N + lam)
    assert kappa >= (N + lam) / (p * N + lam)
    # with more voxels than pixels in all images, some voxel is never seen
    few = orc.Poses(poses.rot[:1], np.zeros(1, np.float32))
    d1 = orc.exact_diag(grid, orc.NO_CTF, few, 1.0, lam)
    assert d1[ball].min() == pytest.approx(lam)


def test_alg1_one_step_with_exact_diagonal(orc):
    # Nearest neighbour, full batch: H is diagonal, the preconditioned step with
    # D_hat = diag(H) and eta = 1 is the Newton step and lands on v* = H^{-1} b.
    M, N = 8, 10
    grid = orc.Grid(M, interp=0)
    opt = orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(N, seed=61), synth.defocus_values(N, 1.0, 3.0, seed=61))
    lam = 0.3
    x = synth.random_complex((N, M, M), seed=62).astype(np.complex128)
    dH = orc.exact_diag(grid, opt, poses, 1.0, lam).reshape(-1)
    b = orc.backproject(grid, opt, poses, x, ctf_power=1).reshape(-1)
    v_star = b / dH
    st = orc.Alg1State(v=synth.random_complex(M ** 3, seed=63).astype(np.complex128), D=None, D_avg=None, eta=1.0)
    halvings = orc.alg1_iteration(grid, opt, poses, x, st, scale=1.0, lam=lam, alpha=0.0, beta=0.9, c=0.1,
                                  D_hat_fixed=dH)
    assert halvings == 0
    assert np.linalg.norm(st.v - v_star) <= 1e-12 * np.linalg.norm(v_star)
    # and v* zeroes the gradient
    g = orc.gradient(grid, opt, poses, v_star, x, 1.0, lam)
    assert np.linalg.norm(g) <= 1e-12 * np.linalg.norm(b)


def test_alg1_invariants(orc):
    M, N, B = 16, 64, 16
    grid = orc.Grid(M)
    opt = orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(N, seed=71), synth.defocus_values(N, 1.0, 3.0, seed=71))
    v_true = synth.blob_volume(M, 5, seed=71).astype(np.complex128)
    x = orc.project(grid, opt, poses, v_true)
    lam = 1e-3
    alpha = orc.alpha_threshold(grid, opt, poses.defocus, lam)
    st = orc.Alg1State(v=np.zeros(M ** 3, np.complex128), D=np.ones(M ** 3), D_avg=np.zeros(M ** 3), eta=1.0)
    scale = N / B
    perm = synth.epoch_permutation(N, 71, 0)
    eta_prev = st.eta
    f_first = None
    for it in range(4):
        I = perm[it * B:(it + 1) * B]
        pI = poses.subset(I)
        z = orc.rademacher(71, it, M ** 3)
        zHz = z * orc.hvp(grid, opt, pI, z, scale, lam).reshape(-1).real
        v_old = st.v.copy()
        D_before = st.D.copy()
        f0 = orc.loss(grid, opt, pI, v_old, x[I], scale, lam)
        g = orc.gradient(grid, opt, pI, v_old, x[I], scale, lam).reshape(-1)
        orc.alg1_iteration(grid, opt, pI, x[I], st, scale, lam, alpha, 0.9, 0.1, zHz=zHz)
        D_hat = np.maximum(np.abs(st.D), alpha)
        assert np.all(D_hat >= alpha)
        # the EMA moved from D_before towards D_avg
        assert np.allclose(st.D, 0.9 * D_before + 0.1 * st.D_avg)
        f1 = orc.loss(grid, opt, pI, st.v, x[I], scale, lam)
        assert f1 <= f0 - 0.1 * st.eta * np.sum(np.abs(g) ** 2 / D_hat) + 1e-9 * abs(f0)
        assert st.eta <= eta_prev
        eta_prev = st.eta
        f_first = f0 if f_first is None else f_first
    assert orc.loss(grid, opt, poses, st.v, x, 1.0, lam) < orc.loss(grid, opt, poses, np.zeros(M ** 3), x, 1.0, lam)


def test_gradient_central_differences(orc):
    M, n = 8, 4
    grid = orc.Grid(M)
    opt = orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(n, seed=81), synth.defocus_values(n, 1.0, 3.0, seed=81))
    v = synth.random_complex(M ** 3, seed=82).astype(np.complex128)
    x = synth.random_complex((n, M, M), seed=83).astype(np.complex128)
    scale, lam, h = 2.0, 0.05, 1e-6
    g = orc.gradient(grid, opt, poses, v, x, scale, lam).reshape(-1)
    rng = np.random.default_rng(84)
    ball = np.flatnonzero(synth.ball_mask(M, 3.0).reshape(-1))
    for k in rng.choice(ball, 16, replace=False):
        for unit, part in ((1.0, "re"), (1j, "im")):
            vp = v.copy(); vp[k] += unit * h
            vm = v.copy(); vm[k] -= unit * h
            fd = (orc.loss(grid, opt, poses, vp, x, scale, lam) - orc.loss(grid, opt, poses, vm, x, scale, lam)) / (2 * h)
            want = g[k].real if part == "re" else g[k].imag
            assert fd == pytest.approx(want, abs=1e-6 * np.max(np.abs(g)))


def test_cg_matches_dense_solve(orc, small_problem):
    grid, opt, poses, A = small_problem
    lam = 0.2
    H = A.T @ A + lam * np.eye(A.shape[1])
    b = synth.random_complex(grid.M ** 3, seed=91).astype(np.complex128)
    x_cg, it = orc.cg_solve(lambda u: orc.hvp(grid, opt, poses, u, 1.0, lam).reshape(-1), b,
                            precond=orc.exact_diag(grid, opt, poses, 1.0, lam), tol=1e-12)
    x_ref = np.linalg.solve(H, b)
    assert np.linalg.norm(x_cg - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


def test_fsc_identities(orc):
    M = 16
    u = synth.random_complex((M, M, M), seed=3)
    assert np.allclose(orc.fsc(u, u, M), 1.0)
    assert np.allclose(orc.fsc(u, -u, M), -1.0)
    assert np.allclose(orc.fsc(u, 3.0 * u, M), 1.0)
    w = synth.random_complex((M, M, M), seed=4)
    f = orc.fsc(u, w, M)
    assert np.all(np.abs(f[3:]) < 0.5)


def test_threshold_shell_counts(orc):
    # P_x(R), P_v(R) of eq. (thresh value): unit-thick shells round(|k|) = R.
    # Summed over R <= Rm they count the lattice points of the disk / ball of
    # radius Rm + 1/2 (Gauss circle problem: area pi r^2 and volume 4/3 pi r^3
    # up to a boundary term); a single shell fluctuates by several percent, so
    # its ratio is only required to be near 2 pi R / (4 pi R^2) = 1/(2R).
    for M in (32, 64, 128, 256):
        Rm = M // 2 - 2
        cx = sum(orc.shell_counts(M, R)[0] for R in range(Rm + 1)) if M <= 64 else None
        if cx is not None:
            r = Rm + 0.5
            cv = sum(orc.shell_counts(M, R)[1] for R in range(Rm + 1))
            assert cx == pytest.approx(math.pi * r * r, rel=0.02)
            assert cv == pytest.approx(4.0 / 3.0 * math.pi * r ** 3, rel=0.02)
        R = M // 2 - 1
        px, pv = orc.shell_counts(M, R)
        assert px / pv == pytest.approx(1.0 / (2 * R), rel=0.15)
    # alpha: with no CTF it is P_x/P_v * N + lambda
    grid = orc.Grid(32)
    px, pv = orc.shell_counts(32, 15)
    assert orc.alpha_threshold(grid, orc.NO_CTF, np.zeros(50), 0.5) == pytest.approx(px / pv * 50 + 0.5)
