"""FP64 CPU oracle for the known-pose Fourier-slice refinement of Toader,
Brubaker & Lederman (arXiv:2311.16100).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product package.  It shares no
code with the HIP library.  The operators live in plain C (oracle.c, built
with gcc -O2 into liboracle.so); the algorithms on top of them (HVP,
Hutchinson's estimator, the preconditioned SGD of Algorithm 1, the
Armijo line search, conjugate gradients for the ground truth, the MLP of the
learned preconditioner) are written here in numpy, step by step in the
paper's order.

Every function is double precision.  Inputs the GPU receives in float32
(rotations, defocus, volumes, images) are accepted in float32 / complex64 and
promoted.

Parity status: every function here is pinned by a CPU test in tests/ against
a closed form, an invariant or brute force; see the test module named in each
docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("r_max", ctypes.c_double), ("interp", ctypes.c_int32)]


class _Optics(ctypes.Structure):
    _fields_ = [("kv", ctypes.c_double), ("cs_mm", ctypes.c_double), ("amp_contrast", ctypes.c_double),
                ("pixel_A", ctypes.c_double), ("ctf_on", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        d, i64, u64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        vp = ctypes.c_void_p
        L.or_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.or_rademacher.argtypes = [u64, u64, i64, vp]
        L.or_wavelength_A.argtypes = [d]
        L.or_wavelength_A.restype = d
        L.or_ctf.argtypes = [P(_Optics), i32, d, d]
        L.or_ctf.restype = d
        L.or_project.argtypes = [P(_Grid), P(_Optics), i64, vp, vp, vp, vp, vp]
        L.or_backproject.argtypes = [P(_Grid), P(_Optics), i64, vp, vp, vp, vp, i32, d, vp]
        L.or_sq_backproject.argtypes = [P(_Grid), P(_Optics), i64, vp, vp, d, vp]
        L.or_features.argtypes = [P(_Grid), P(_Optics), i64, vp, vp, vp, vp]
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# Problem description
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Grid:
    """M: grid side (even); r_max: disk radius of the pixels used (default
    M/2 - 1); interp: 0 nearest neighbour, 1 trilinear (Definition
    "Projection operator", Sec. 2.1)."""
    M: int
    r_max: float | None = None
    interp: int = 1

    @property
    def rmax(self) -> float:
        return float(self.M // 2 - 1) if self.r_max is None else float(self.r_max)

    def c(self):
        return _Grid(self.M, self.rmax, self.interp)


@dataclass(frozen=True)
class Optics:
    kv: float = 300.0
    cs_mm: float = 2.7
    amp_contrast: float = 0.1
    pixel_A: float = 1.0
    ctf_on: bool = True

    def c(self):
        return _Optics(self.kv, self.cs_mm, self.amp_contrast, self.pixel_A, int(self.ctf_on))


NO_CTF = Optics(ctf_on=False)


@dataclass
class Poses:
    rot: np.ndarray      # float32 [n,3,3]
    defocus: np.ndarray  # float32 [n], Angstrom
    shift: np.ndarray | None = None  # float32 [n,2] in-plane shift (sx, sy) in pixels, or None (T = I)

    def __post_init__(self):
        self.rot = np.ascontiguousarray(self.rot, dtype=np.float32).reshape(-1, 3, 3)
        self.defocus = np.ascontiguousarray(self.defocus, dtype=np.float32).reshape(-1)
        assert self.rot.shape[0] == self.defocus.shape[0]
        if self.shift is not None:
            self.shift = np.ascontiguousarray(self.shift, dtype=np.float32).reshape(-1, 2)
            assert self.shift.shape[0] == self.rot.shape[0]

    @property
    def n(self) -> int:
        return self.rot.shape[0]

    def subset(self, idx) -> "Poses":
        return Poses(self.rot[idx], self.defocus[idx], None if self.shift is None else self.shift[idx])


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


# ---------------------------------------------------------------------------
# Primitives (C)
# ---------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block (Salmon et al., SC'11). Pinned by the published
    known-answer vectors (tests/test_oracle_rng_ctf.py)."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def rademacher(seed: int, probe: int, nvox: int) -> np.ndarray:
    """Rademacher(0.5) probe z in {+1,-1}^nvox of eq. (hutch), Sec. 3.2."""
    z = np.empty(nvox, dtype=np.float64)
    lib().or_rademacher(int(seed), int(probe), int(nvox), _ptr(z))
    return z


def wavelength_A(kv: float) -> float:
    """Relativistic electron wavelength in Angstrom."""
    return lib().or_wavelength_A(float(kv))


def ctf(optics: Optics, M: int, defocus_A: float, k2: float) -> float:
    """Weak-phase CTF at squared integer radius k2 (the paper's C_i, Sec. 2.1,
    with the textbook formula; see oracle.c)."""
    o = optics.c()
    return lib().or_ctf(ctypes.byref(o), int(M), float(defocus_A), float(k2))


def project(grid: Grid, optics: Optics, poses: Poses, vol) -> np.ndarray:
    """C_i P_i v for every image, eq. (fwd model) without noise.  [n][M][M]."""
    M = grid.M
    v = _c128(vol).reshape(M, M, M)
    out = np.zeros((poses.n, M, M), dtype=np.complex128)
    g, o = grid.c(), optics.c()
    lib().or_project(ctypes.byref(g), ctypes.byref(o), poses.n, _ptr(poses.rot), _ptr(poses.defocus),
                     _ptr(poses.shift), _ptr(v), _ptr(out))
    return out


def backproject(grid: Grid, optics: Optics, poses: Poses, img, ctf_power: int = 1,
                scale: float = 1.0, accum=None) -> np.ndarray:
    """accum + scale * sum_i P_i^T C_i^p img_i (the adjoint, eq. (em v))."""
    M = grid.M
    im = _c128(img).reshape(poses.n, M, M)
    out = np.zeros((M, M, M), dtype=np.complex128) if accum is None else _c128(accum).copy()
    g, o = grid.c(), optics.c()
    lib().or_backproject(ctypes.byref(g), ctypes.byref(o), poses.n, _ptr(poses.rot), _ptr(poses.defocus),
                         _ptr(poses.shift), _ptr(im), int(ctf_power), float(scale), _ptr(out))
    return out


def sq_backproject(grid: Grid, optics: Optics, poses: Poses, scale: float = 1.0) -> np.ndarray:
    """scale * diag(sum_i P_i^T C_i^2 P_i), the squared-weight backprojection."""
    M = grid.M
    out = np.zeros((M, M, M), dtype=np.float64)
    g, o = grid.c(), optics.c()
    lib().or_sq_backproject(ctypes.byref(g), ctypes.byref(o), poses.n, _ptr(poses.rot), _ptr(poses.defocus),
                            float(scale), _ptr(out))
    return out


def features(grid: Grid, optics: Optics, poses: Poses):
    """(sum_ij C_ij^2 w_ijk, |Omega_k|) per voxel, both float64 [M][M][M]."""
    M = grid.M
    f2 = np.zeros((M, M, M), dtype=np.float64)
    f3 = np.zeros((M, M, M), dtype=np.float64)
    g, o = grid.c(), optics.c()
    lib().or_features(ctypes.byref(g), ctypes.byref(o), poses.n, _ptr(poses.rot), _ptr(poses.defocus),
                      _ptr(f2), _ptr(f3))
    return f2, f3


# ---------------------------------------------------------------------------
# Objective, gradient and Hessian (Sec. 3.1, eqs. (optim cp), (hessian))
# with the CTF re-inserted as in eq. (em v) and the minibatch scaled to an
# unbiased estimate of the full sum: f_I(v) = (N/B) sum_{i in I} 1/2 ||x_i -
# C_i P_i v||^2 + lambda/2 ||v||^2.
# ---------------------------------------------------------------------------
def loss(grid, optics, poses, v, x, scale: float, lam: float) -> float:
    r = project(grid, optics, poses, v) - _c128(x)
    v = _c128(v)
    return float(scale * 0.5 * np.vdot(r, r).real + 0.5 * lam * np.vdot(v, v).real)


def gradient(grid, optics, poses, v, x, scale: float, lam: float) -> np.ndarray:
    """scale * sum_i P_i^T C_i (C_i P_i v - x_i) + lambda v.  The complex
    gradient convention is d/dRe + i d/dIm of the real loss."""
    r = project(grid, optics, poses, v) - _c128(x)
    return backproject(grid, optics, poses, r, ctf_power=1, scale=scale) + lam * _c128(v).reshape(grid.M, grid.M, grid.M)


def hvp(grid, optics, poses, z, scale: float, lam: float) -> np.ndarray:
    """H_I z = scale * sum_i P_i^T C_i^2 P_i z + lambda z (complex z allowed;
    H is real, so real and imaginary parts are independent products)."""
    M = grid.M
    z = _c128(z).reshape(M, M, M)
    return backproject(grid, optics, poses, project(grid, optics, poses, z), ctf_power=1, scale=scale) + lam * z


def hutchinson_diag(grid, optics, poses, n_probe: int, seed: int, scale: float, lam: float,
                    probe0: int = 0) -> np.ndarray:
    """Hutchinson's estimate mean_p z_p (.) H z_p with Rademacher z_p, eq. (hutch),
    probes probe0 .. probe0+n_probe-1."""
    M = grid.M
    acc = np.zeros(M ** 3)
    for p in range(n_probe):
        z = rademacher(seed, probe0 + p, M ** 3)
        hz = hvp(grid, optics, poses, z, scale, lam).reshape(-1)
        acc += z * hz.real
    return (acc / n_probe).reshape(M, M, M)


def exact_diag(grid, optics, poses, scale: float, lam: float) -> np.ndarray:
    """diag(H_I) = scale * sum_ij C_ij^2 w_ijk^2 + lambda, from eq. (hessian)
    with the trilinear weights of eq. (def tri interp)."""
    return sq_backproject(grid, optics, poses, scale) + lam


def shell_counts(M: int, R: int):
    """(P_x(R), P_v(R)): pixels of the M x M grid and voxels of the M^3 grid
    whose radius rounds to R (the Fourier shells of eq. (thresh value))."""
    ax = np.arange(M) - M // 2
    r2 = np.sqrt(ax[:, None] ** 2 + ax[None, :] ** 2)
    r3 = np.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2)
    return int(np.sum(np.rint(r2) == R)), int(np.sum(np.rint(r3) == R))


def alpha_threshold(grid: Grid, optics: Optics, defocus_all, lam: float, R: int | None = None) -> float:
    """alpha = (P_x(R)/P_v(R)) sum_{i=1}^N |C_i(R)|^2 + lambda, eq. (thresh value),
    at the maximum radius R = r_max, summed over all N images of the data set."""
    R = int(round(grid.rmax)) if R is None else int(R)
    px, pv = shell_counts(grid.M, R)
    s = sum(ctf(optics, grid.M, float(df), float(R * R)) ** 2 for df in np.asarray(defocus_all, dtype=np.float32))
    return px / pv * s + lam


# ---------------------------------------------------------------------------
# Algorithm 1 (Sec. 3.4): preconditioned SGD with the estimated, thresholded
# diagonal and the stochastic Armijo line search of eq. (stochastic armijo).
# ---------------------------------------------------------------------------
@dataclass
class Alg1State:
    v: np.ndarray            # complex128 [M^3]
    D: np.ndarray | None     # float64 [M^3]; None = plain SGD (D-hat == 1)
    D_avg: np.ndarray | None
    eta: float
    k: int = 0
    capped: int = 0  # iterations whose line search stopped at max_halvings


def precond_update(D, D_avg, zHz, k: int, beta: float, alpha: float):
    """Running mean of the probe samples, exponential average and
    thresholding (Alg. 1, the three lines after drawing I_k and z):
      D_avg <- (k-1)/k D_avg + (1/k) zHz
      D     <- beta D + (1 - beta) D_avg
      D_hat <- max(|D|, alpha).
    Returns (D, D_avg, D_hat) as new arrays."""
    D_avg = (k - 1) / k * D_avg + zHz / k
    D = beta * D + (1.0 - beta) * D_avg
    D_hat = np.maximum(np.abs(D), alpha)
    return D, D_avg, D_hat


def precomputed_diagonal(grid, optics, poses, batches, scale: float, lam: float, beta: float, n_probe: int,
                         probe_seed: int):
    """The precomputed preconditioner of Sec. 4.1 (SGD's second arm): the
    diagonal estimate of eq. (diag est rule), read with Algorithm 1's running
    mean, run over the given minibatches (index arrays, in order: many epochs
    of batches) before SGD starts, from D = 1, D_avg = 0.  Iteration k's
    sample is Hutchinson's estimate on its minibatch with the probes
    (k-1) n_probe .. k n_probe - 1.  Returns (D, D_avg), unthresholded."""
    M = grid.M
    D = np.ones(M ** 3)
    D_avg = np.zeros(M ** 3)
    for k, idx in enumerate(batches, start=1):
        zHz = hutchinson_diag(grid, optics, poses.subset(list(idx)), n_probe, probe_seed, scale, lam,
                              probe0=(k - 1) * n_probe).reshape(-1)
        D, D_avg, _ = precond_update(D, D_avg, zHz, k, beta, 0.0)
    return D, D_avg


def precond_step(v, g, D_hat, eta: float):
    """v - eta D_hat^{-1} g (eq. (sgd step)) and ||g||^2_{D_hat^{-1}}."""
    v = _c128(v).reshape(-1)
    g = _c128(g).reshape(-1)
    Dh = np.ones(v.shape) if D_hat is None else np.asarray(D_hat, dtype=np.float64).reshape(-1)
    return v - eta * g / Dh, float(np.sum(np.abs(g) ** 2 / Dh))


def alg1_iteration(grid, optics, poses_I, x_I, state: Alg1State, scale: float, lam: float,
                   alpha: float, beta: float, c: float, zHz=None, D_hat_fixed=None,
                   max_halvings: int = 30):
    """One iteration k of Algorithm 1 on the minibatch (poses_I, x_I).
    zHz: the probe sample z (.) H_I z for this iteration (None: no update of D,
    e.g. plain SGD or a fixed preconditioner).  D_hat_fixed overrides D-hat
    (learned or precomputed preconditioner).  Returns the number of halvings.

    The line search of eq. (stochastic armijo) halves eta until the
    sufficient-decrease test holds.  The paper's loop has no bound; here it
    stops after max_halvings halvings and keeps the last (tiny) trial step,
    counting the iteration in state.capped: in floating point the test can
    fail on rounding alone once the decrease is below the resolution of the
    minibatch loss.  A loss or gradient norm that is not finite raises
    FloatingPointError (no step is taken)."""
    state.k += 1
    k = state.k
    if D_hat_fixed is not None:
        D_hat = np.asarray(D_hat_fixed, dtype=np.float64).reshape(-1)
    elif state.D is not None:
        if zHz is not None:
            state.D, state.D_avg, D_hat = precond_update(state.D, state.D_avg,
                                                         np.asarray(zHz).reshape(-1), k, beta, alpha)
        else:
            D_hat = np.maximum(np.abs(state.D), alpha)
    else:
        D_hat = None
    g = gradient(grid, optics, poses_I, state.v, x_I, scale, lam).reshape(-1)
    f0 = loss(grid, optics, poses_I, state.v, x_I, scale, lam)
    eta = state.eta
    halvings = 0
    while True:
        v_new, gn = precond_step(state.v, g, D_hat, eta)
        f1 = loss(grid, optics, poses_I, v_new, x_I, scale, lam)
        if not (np.isfinite(f0) and np.isfinite(f1) and np.isfinite(gn)):
            raise FloatingPointError("Armijo line search: f(v) = %r, f(v') = %r, |g|^2_D^-1 = %r" % (f0, f1, gn))
        if f1 <= f0 - c * eta * gn:
            break
        if halvings >= max_halvings:
            state.capped += 1
            break
        eta /= 2.0
        halvings += 1
    state.v = v_new
    state.eta = eta
    return halvings


def cg_solve(apply_H, b, precond=None, tol: float = 1e-10, max_iter: int = 1000, x0=None):
    """Conjugate gradients for H v = b (eq. (lin sys)); H is Hermitian positive
    definite.  precond: diagonal (array) of a Jacobi preconditioner or None."""
    b = _c128(b).reshape(-1)
    x = np.zeros_like(b) if x0 is None else _c128(x0).reshape(-1).copy()
    r = b - apply_H(x)
    Minv = None if precond is None else 1.0 / np.asarray(precond, dtype=np.float64).reshape(-1)
    zr = r if Minv is None else Minv * r
    p = zr.copy()
    rz = np.vdot(r, zr).real
    bn = np.linalg.norm(b)
    for it in range(max_iter):
        if np.linalg.norm(r) <= tol * bn:
            return x, it
        Ap = apply_H(p)
        a = rz / np.vdot(p, Ap).real
        x = x + a * p
        r = r - a * Ap
        zr = r if Minv is None else Minv * r
        rz_new = np.vdot(r, zr).real
        p = zr + (rz_new / rz) * p
        rz = rz_new
    return x, max_iter


def relative_error(v, v_star, mask=None) -> float:
    """||m (.) (v - v*)|| / ||m (.) v*||."""
    v = _c128(v).reshape(-1)
    vs = _c128(v_star).reshape(-1)
    if mask is not None:
        m = np.asarray(mask).reshape(-1)
        v, vs = v[m], vs[m]
    return float(np.linalg.norm(v - vs) / np.linalg.norm(vs))


def fsc(u, v, M: int):
    """Fourier shell correlation per integer shell, eq. (fsc)."""
    ax = np.arange(M) - M // 2
    r = np.rint(np.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2)).astype(int)
    u = _c128(u).reshape(M, M, M)
    v = _c128(v).reshape(M, M, M)
    out = []
    for s in range(M // 2):
        m = r == s
        num = np.sum(u[m] * np.conj(v[m]))
        den = np.sqrt(np.sum(np.abs(u[m]) ** 2) * np.sum(np.abs(v[m]) ** 2))
        out.append((num / den).real if den > 0 else 0.0)
    return np.array(out)


# ---------------------------------------------------------------------------
# Learned preconditioner network (not part of the paper's method: a
# per-voxel regression of the Hessian diagonal from cheap features, trained on
# Hutchinson estimates).  MLP 3 -> 64 -> 64 -> 1 with GELU; weights and the
# inputs of each weight product are rounded to bfloat16 (round to nearest
# even), products are accumulated in double here.
# Parameter vector (float32): W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3.
# ---------------------------------------------------------------------------
MLP_H = 64
MLP_NPARAM = MLP_H * 3 + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1


def bf16_round(a) -> np.ndarray:
    """Round to float32 and then to the nearest bfloat16 (ties to even) -- the
    path of a float32 activation or weight on the GPU -- returned as
    float64."""
    x = np.ascontiguousarray(a, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    # NaN/Inf pass through unchanged
    out = np.where(np.isfinite(x), out, x)
    return out.astype(np.float64)


def mlp_unpack(params):
    p = np.asarray(params, dtype=np.float32)
    H = MLP_H
    o = 0
    W1 = p[o:o + 3 * H].reshape(H, 3); o += 3 * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def gelu(x):
    """GELU(x) = x Phi(x) = x/2 (1 + erf(x / sqrt 2))."""
    from scipy.special import erf
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def mlp_forward(params, X, keep=False):
    """y = W3 . g(W2 g(W1 x + b1) + b2) + b3 per row of X [n,3]; weights and
    layer inputs rounded to bfloat16."""
    W1, b1, W2, b2, W3, b3 = (bf16_round(w) if i % 2 == 0 else np.asarray(w, np.float64)
                              for i, w in enumerate(mlp_unpack(params)))
    x0 = bf16_round(np.asarray(X, dtype=np.float64))
    z1 = x0 @ W1.T + b1
    h1 = gelu(z1)
    h1r = bf16_round(h1)
    z2 = h1r @ W2.T + b2
    h2 = gelu(z2)
    h2r = bf16_round(h2)
    y = h2r @ W3 + b3[0]
    if keep:
        return y, dict(x0=x0, z1=z1, h1r=h1r, z2=z2, h2r=h2r, W2=W2, W3=W3)
    return y


def mlp_loss_grad(params, X, t):
    """Mean squared error L = 1/n sum (y - t)^2 and its gradient with respect
    to the parameter vector (straight-through: the bfloat16 roundings are
    treated as identity in the backward pass)."""
    y, c = mlp_forward(params, X, keep=True)
    n = len(t)
    r = y - np.asarray(t, dtype=np.float64)
    L = float(np.mean(r * r))
    dy = 2.0 * r / n
    dW3 = dy @ c["h2r"]
    db3 = np.array([dy.sum()])
    dh2 = np.outer(dy, c["W3"])
    dz2 = dh2 * gelu_grad(c["z2"])
    dW2 = dz2.T @ c["h1r"]
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ c["W2"]
    dz1 = dh1 * gelu_grad(c["z1"])
    dW1 = dz1.T @ c["x0"]
    db1 = dz1.sum(axis=0)
    g = np.concatenate([dW1.reshape(-1), db1, dW2.reshape(-1), db2, dW3, db3])
    return L, g
