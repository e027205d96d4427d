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


def _shell_counts_integer(M, R):
    """(P_x(R), P_v(R)) by integer arithmetic alone: round(|k|) = R exactly
    when (2R - 1)^2 <= 4|k|^2 < (2R + 1)^2 (|k|^2 is an integer, so |k| is
    never a half-integer and the rounding has no ties)."""
    ax = np.arange(M, dtype=np.int64) - M // 2
    k2_2 = ax[:, None] ** 2 + ax[None, :] ** 2
    k2_3 = k2_2[None, :, :] + (ax ** 2)[:, None, None]
    lo, hi = (2 * R - 1) ** 2 if R > 0 else -1, (2 * R + 1) ** 2
    px = int(np.count_nonzero(4 * k2_2 < hi) - np.count_nonzero(4 * k2_2 < lo))
    pv = int(np.count_nonzero(4 * k2_3 < hi) - np.count_nonzero(4 * k2_3 < lo))
    return px, pv


# P_x(R) / P_v(R) at R = M/2 - 1, the shell of eq. (thresh value) for the
# workloads' grids, as exact integer ratios (enumerated independently of the
# oracle when the workloads were specified).
SHELL_RATIOS = {32: 0.03204, 64: 0.01581, 128: 0.00745, 256: 0.00412}


def test_threshold_shell_counts(orc):
    # P_x(R), P_v(R) of eq. (thresh value): unit-thick shells round(|k|) = R.
    # Exact against an integer count, for every shell of small grids and the
    # threshold shell of the workload grids; the ratios reproduce the
    # enumerated values to their printed digits.  A floor(|k|) shell
    # definition is 6% off at M = 32, so it fails here.
    for M in (8, 16, 32):
        for R in range(M // 2):
            assert orc.shell_counts(M, R) == _shell_counts_integer(M, R)
    for M, ratio in SHELL_RATIOS.items():
        R = M // 2 - 1
        px, pv = orc.shell_counts(M, R)
        assert (px, pv) == _shell_counts_integer(M, R)
        assert px / pv == pytest.approx(ratio, abs=5e-6)
    # Summed over R <= Rm the shells count the lattice points of the disk /
    # ball of radius Rm + 1/2 (Gauss circle problem: area pi r^2 and volume
    # 4/3 pi r^3 up to a boundary term).
    for M in (32, 64):
        Rm = M // 2 - 2
        cx = sum(orc.shell_counts(M, R)[0] for R in range(Rm + 1))
        cv = sum(orc.shell_counts(M, R)[1] for R in range(Rm + 1))
        r = Rm + 0.5
        assert cx == pytest.approx(math.pi * r * r, rel=0.02)
        assert cv == pytest.approx(4.0 / 3.0 * math.pi * r ** 3, rel=0.02)
    # alpha: with no CTF it is P_x/P_v * N + lambda
    grid = orc.Grid(32)
    px, pv = orc.shell_counts(32, 15)
    assert orc.alpha_threshold(grid, orc.NO_CTF, np.zeros(50), 0.5) == pytest.approx(px / pv * 50 + 0.5)


def test_shell_pin_rejects_floor_shells():
    # the pin above is sensitive to the shell definition: floor(|k|) = R
    # shells give ratios 1-6% away from the enumerated ones
    for M, ratio in SHELL_RATIOS.items():
        R = M // 2 - 1
        ax = np.arange(M) - M // 2
        r2 = np.floor(np.sqrt(ax[:, None] ** 2 + ax[None, :] ** 2))
        r3 = np.floor(np.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2))
        wrong = np.sum(r2 == R) / np.sum(r3 == R)
        assert abs(wrong - ratio) > 5e-6


def _ema_closed_form(samples, beta):
    """D^(k) of Algorithm 1 written out: with D^(0) = 1 and m_j the mean of
    the first j probe samples, D^(k) = beta^k + (1 - beta) sum_j beta^(k-j) m_j."""
    k = len(samples)
    means = [np.mean(samples[:j], axis=0) for j in range(1, k + 1)]
    D = beta ** k * np.ones_like(samples[0])
    for j, m in enumerate(means, start=1):
        D = D + (1.0 - beta) * beta ** (k - j) * m
    return D


def _running_mean_ok(update, beta=0.9, k_max=7, n=257, seed=5):
    rng = np.random.default_rng(seed)
    samples = [rng.uniform(0.1, 50.0, n) for _ in range(k_max)]
    D, D_avg = np.ones(n), np.zeros(n)
    for k in range(1, k_max + 1):
        D, D_avg, _ = update(D, D_avg, samples[k - 1], k, beta, 0.0)
        if not np.allclose(D_avg, np.mean(samples[:k], axis=0), rtol=1e-13, atol=0):
            return False
        if not np.allclose(D, _ema_closed_form(samples[:k], beta), rtol=1e-13, atol=0):
            return False
    return True


def test_running_mean_and_ema_closed_form(orc):
    # Algorithm 1's running-mean line: after k probe samples D_avg is their
    # plain mean, and D follows the exponential average from D^(0) = 1 in the
    # closed form above.  Checked on precond_update and through
    # alg1_iteration (which must call it with the iteration counter k).
    assert _running_mean_ok(orc.precond_update)
    M, N = 8, 6
    grid, opt = orc.Grid(M), orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(N, seed=72), synth.defocus_values(N, 1.0, 3.0, seed=72))
    x = synth.random_complex((N, M, M), seed=73).astype(np.complex128)
    st = orc.Alg1State(v=np.zeros(M ** 3, np.complex128), D=np.ones(M ** 3), D_avg=np.zeros(M ** 3), eta=1.0)
    rng = np.random.default_rng(74)
    samples = []
    for _ in range(5):
        s = rng.uniform(1.0, 20.0, M ** 3)
        samples.append(s)
        orc.alg1_iteration(grid, opt, poses, x, st, 1.0, 0.1, 0.5, 0.9, 0.1, zHz=s)
        assert np.allclose(st.D_avg, np.mean(samples, axis=0), rtol=1e-13, atol=0)
        assert np.allclose(st.D, _ema_closed_form(samples, 0.9), rtol=1e-13, atol=0)


def test_running_mean_pin_rejects_garbled_update(orc):
    # the printed eq. (hutch update), D_avg = (1/k) z (.) Hz (no running sum),
    # and an update that forgets the (k-1)/k factor both fail the pin
    def garbled(D, D_avg, zHz, k, beta, alpha):
        D_avg = zHz / k
        D = beta * D + (1.0 - beta) * D_avg
        return D, D_avg, np.maximum(np.abs(D), alpha)

    def no_decay(D, D_avg, zHz, k, beta, alpha):
        D_avg = D_avg + zHz / k
        D = beta * D + (1.0 - beta) * D_avg
        return D, D_avg, np.maximum(np.abs(D), alpha)

    def ema_of_sample(D, D_avg, zHz, k, beta, alpha):
        D_avg = (k - 1) / k * D_avg + zHz / k
        D = beta * D + (1.0 - beta) * zHz
        return D, D_avg, np.maximum(np.abs(D), alpha)

    for wrong in (garbled, no_decay, ema_of_sample):
        assert not _running_mean_ok(wrong)


def test_alg1_line_search_cap_keeps_last_step(orc):
    # With c = 2 the sufficient-decrease test of eq. (stochastic armijo) fails
    # for every eta > 0 on a convex quadratic (the decrease is at most eta
    # |g|^2_D^-1 to first order), so the line search runs into its bound:
    # after 30 halvings the last trial step, eta = 2^-30 eta0, is kept and the
    # iteration is counted as capped.
    M, N = 8, 6
    grid, opt = orc.Grid(M), orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(N, seed=75), synth.defocus_values(N, 1.0, 3.0, seed=75))
    x = synth.random_complex((N, M, M), seed=76).astype(np.complex128)
    v0 = synth.random_complex(M ** 3, seed=77).astype(np.complex128)
    st = orc.Alg1State(v=v0.copy(), D=None, D_avg=None, eta=1.0)
    g = orc.gradient(grid, opt, poses, v0, x, 1.0, 0.1).reshape(-1)
    h = orc.alg1_iteration(grid, opt, poses, x, st, 1.0, 0.1, 0.0, 0.9, 2.0)
    assert h == 30 and st.capped == 1
    assert st.eta == 2.0 ** -30
    assert np.array_equal(st.v, v0 - 2.0 ** -30 * g)
    # the next iteration starts from the reduced step (eta is never raised)
    h = orc.alg1_iteration(grid, opt, poses, x, st, 1.0, 0.1, 0.0, 0.9, 0.1)
    assert h == 0 and st.eta == 2.0 ** -30 and st.capped == 1


def test_alg1_non_finite_raises(orc):
    M, N = 8, 6
    grid, opt = orc.Grid(M), orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(N, seed=78), synth.defocus_values(N, 1.0, 3.0, seed=78))
    x = synth.random_complex((N, M, M), seed=79).astype(np.complex128)
    x[2, M // 2, M // 2 + 1] = np.nan
    v0 = np.zeros(M ** 3, np.complex128)
    st = orc.Alg1State(v=v0.copy(), D=None, D_avg=None, eta=1.0)
    with pytest.raises(FloatingPointError):
        orc.alg1_iteration(grid, opt, poses, x, st, 1.0, 0.1, 0.0, 0.9, 0.1)
    assert np.array_equal(st.v, v0)


def test_precomputed_diagonal_nearest_neighbour_closed_form(orc):
    # Sec. 4.1's precomputed preconditioner with nearest-neighbour
    # interpolation: H_I is diagonal, so every iteration's Hutchinson sample
    # is exactly diag(H_I) (the Remark after the diagonal estimate), whatever
    # the probes.  The result must then equal the exponential average (from
    # D^(0) = 1) of the running means of the batch diagonals, each computed
    # here from the squared-weight backprojection (a code path that shares
    # nothing with the HVP): after the first epoch the running mean is diag H
    # itself, and D approaches it like beta^k.
    M, N, B = 8, 12, 4
    grid, opt = orc.Grid(M, interp=0), orc.Optics()
    poses = orc.Poses(synth.uniform_rotations(N, seed=81), synth.defocus_values(N, 1.0, 3.0, seed=81))
    scale, lam, beta = N / B, 0.2, 0.9
    batches = [synth.epoch_permutation(N, 82, e)[s:s + B] for e in range(4) for s in range(0, N, B)]
    D, D_avg = orc.precomputed_diagonal(grid, opt, poses, batches, scale, lam, beta, 2, 83)
    samples = [orc.exact_diag(grid, opt, poses.subset(list(b)), scale, lam).reshape(-1) for b in batches]
    running = [np.mean(samples[:k], axis=0) for k in range(1, len(samples) + 1)]
    want = np.ones(M ** 3)
    for r in running:
        want = beta * want + (1 - beta) * r
    assert np.allclose(D_avg, running[-1], rtol=1e-12, atol=1e-12)
    assert np.allclose(D, want, rtol=1e-12, atol=1e-12)
    # a whole number of epochs: the running mean is the full diagonal
    full = orc.exact_diag(grid, opt, poses, 1.0, lam).reshape(-1)
    assert np.allclose(D_avg, full, rtol=1e-12, atol=1e-12)
    assert np.max(np.abs(D - full)) <= beta ** len(batches) * np.max(np.abs(1 - full)) + \
        np.max(np.abs(np.array(running[: N // B]) - full)) + 1e-12


def test_conditioning_shell_counts_match_oracle(orc):
    # p(R) of the paper's condition-number figure comes from the same integer
    # shells as the threshold of eq. (thresh value)
    from paper_2311_16100_amd import conditioning as C
    for R in (1, 2, 5, 16, 31):
        assert C.shell_point_counts(R) == tuple(orc.shell_counts(2 * R + 4, R))
