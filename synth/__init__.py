"""Seeded synthetic inputs shared by the oracle tests, the GPU tests, the
benchmark and the SGD runs.

This module holds none of the method's arithmetic: no projection, no CTF, no
adjoint, no Hessian.  It only draws the inputs the method is applied to
(volumes, poses, defocus values, images, minibatch orders) from fixed seeds,
with the shapes and value distributions of the paper's setting (Sec. 4.1) as
restated by the synthetic workloads below.  The random numbers the method
itself draws (Hutchinson's Rademacher probes) are NOT made here: each side
generates them from the published Philox4x32-10 definition.

Grid convention: frequencies k in {-M/2, ..., M/2-1} per axis, arrays indexed
[kz][ky][kx] (volumes) and [i][ky][kx] (images), DC at index M/2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Sub-stream ids of each seed: one independent generator per kind of input.
STREAM_BLOBS, STREAM_POSES, STREAM_DEFOCUS, STREAM_NOISE = 0, 1, 2, 3
STREAM_PERM, STREAM_INIT, STREAM_MLP, STREAM_MISC = 5, 6, 7, 8

# Microscope optics of every workload: 300 kV, Cs 2.7 mm, amplitude
# contrast 0.1, pixel 1 Angstrom.
OPTICS_300KV = dict(kv=300.0, cs_mm=2.7, amp_contrast=0.1, pixel_A=1.0)


def generator(seed: int, stream: int) -> np.random.Generator:
    """Independent numpy generator for (seed, stream)."""
    return np.random.default_rng([int(seed), int(stream)])


# --------------------------------------------------------------------------
# Volumes
# --------------------------------------------------------------------------
@dataclass
class Blobs:
    """Isotropic Gaussian blobs rho(x) = sum_b a_b exp(-|x - c_b|^2 / (2 s_b^2)),
    positions in voxels relative to the grid centre."""
    centres: np.ndarray  # [nb, 3] as (x, y, z)
    sigmas: np.ndarray   # [nb]
    amps: np.ndarray     # [nb]


def blob_params(M: int, n_blobs: int, seed: int, sigma_range=(1.0, 3.0),
                amp_range=(0.5, 1.0), centre_halfwidth=None) -> Blobs:
    """Blob centres uniform in the inner half-box [-M/4, M/4)^3, sigma and
    amplitude uniform in the given ranges."""
    g = generator(seed, STREAM_BLOBS)
    hw = M / 4.0 if centre_halfwidth is None else centre_halfwidth
    centres = g.uniform(-hw, hw, size=(n_blobs, 3))
    sigmas = g.uniform(sigma_range[0], sigma_range[1], size=n_blobs)
    amps = g.uniform(amp_range[0], amp_range[1], size=n_blobs)
    return Blobs(centres, sigmas, amps)


def blob_density(M: int, blobs: Blobs) -> np.ndarray:
    """Real-space density on the grid x in {-M/2..M/2-1}^3, indexed [z][y][x].
    Each blob is evaluated only within 6 sigma of its centre (the tail
    beyond that is below 1.6e-8 of the peak)."""
    rho = np.zeros((M, M, M), dtype=np.float64)
    ax = np.arange(M) - M // 2
    for c, s, a in zip(blobs.centres, blobs.sigmas, blobs.amps):
        r = int(math.ceil(6.0 * s))
        lo = [max(0, int(math.floor(c[d])) - r + M // 2) for d in range(3)]
        hi = [min(M, int(math.floor(c[d])) + r + 1 + M // 2) for d in range(3)]
        gx = np.exp(-((ax[lo[0]:hi[0]] - c[0]) ** 2) / (2 * s * s))
        gy = np.exp(-((ax[lo[1]:hi[1]] - c[1]) ** 2) / (2 * s * s))
        gz = np.exp(-((ax[lo[2]:hi[2]] - c[2]) ** 2) / (2 * s * s))
        rho[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += a * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return rho


def centred_fftn(rho: np.ndarray) -> np.ndarray:
    """Centred DFT: fftshift(fftn(ifftshift(rho))).  With the grid centred at
    index M/2 this is sum_x rho(x) exp(-2 pi i k.x / M)."""
    return np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(rho)))


def blob_volume(M: int, n_blobs: int, seed: int, dtype=np.complex64, **kw) -> np.ndarray:
    """Fourier volume of a sum of Gaussian blobs, [M][M][M] complex."""
    rho = blob_density(M, blob_params(M, n_blobs, seed, **kw))
    return centred_fftn(rho).astype(dtype)


def random_complex(shape, seed: int, stream: int = STREAM_MISC, dtype=np.complex64) -> np.ndarray:
    """Entries with independent standard-normal real and imaginary parts."""
    g = generator(seed, stream)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im).astype(dtype)


def ball_mask(M: int, radius: float) -> np.ndarray:
    """Boolean [M][M][M] mask of |k| <= radius."""
    ax = np.arange(M) - M // 2
    k2 = ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2
    return k2 <= radius * radius


# --------------------------------------------------------------------------
# Poses
# --------------------------------------------------------------------------
def quaternion_to_matrix(q: np.ndarray) -> np.ndarray:
    """Unit quaternions (w, x, y, z) [n,4] to rotation matrices [n,3,3] (float64)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def uniform_rotations(n: int, seed: int) -> np.ndarray:
    """Haar-uniform rotations from normalised Gaussian quaternions, computed in
    float64 and rounded once to float32, shape [n,3,3] row-major."""
    g = generator(seed, STREAM_POSES)
    q = g.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return quaternion_to_matrix(q).astype(np.float32)


def vmf_directions(n: int, kappa: float, g: np.random.Generator) -> np.ndarray:
    """Unit vectors from the von Mises-Fisher distribution on S^2 with mean +z
    and concentration kappa (Wood 1994; on S^2 the cosine has the closed-form
    inverse CDF w = 1 + log(u + (1-u) e^{-2 kappa}) / kappa)."""
    u = g.uniform(size=n)
    w = 1.0 + np.log(u + (1.0 - u) * np.exp(-2.0 * kappa)) / kappa
    phi = g.uniform(0.0, 2.0 * np.pi, size=n)
    r = np.sqrt(np.clip(1.0 - w * w, 0.0, None))
    return np.stack([r * np.cos(phi), r * np.sin(phi), w], axis=1)


def vmf_rotations(n: int, kappa: float, seed: int) -> np.ndarray:
    """Preferred-orientation poses: the viewing direction (the image-plane
    normal, row 2 of R) is vMF(kappa) around +z, the in-plane angle uniform.
    float32 [n,3,3]."""
    g = generator(seed, STREAM_POSES)
    d = vmf_directions(n, kappa, g)
    psi = g.uniform(0.0, 2.0 * np.pi, size=n)
    # any orthonormal pair spanning the plane normal to d
    helper = np.where(np.abs(d[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    a = np.cross(d, helper)
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.cross(d, a)
    c, s = np.cos(psi)[:, None], np.sin(psi)[:, None]
    e1 = c * a + s * b
    e2 = np.cross(d, e1)
    R = np.stack([e1, e2, d], axis=1)
    return R.astype(np.float32)


def cube_group() -> np.ndarray:
    """The 24 rotations of the cube (signed permutation matrices with det +1),
    float32 [24,3,3]."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3))
            for r, c in enumerate(perm):
                R[r, c] = signs[r]
            if round(np.linalg.det(R)) == 1:
                out.append(R)
    return np.array(out, dtype=np.float32)


def defocus_values(n: int, lo_um: float, hi_um: float, seed: int) -> np.ndarray:
    """Per-image defocus uniform in [lo, hi] micrometres, returned in Angstrom
    (float32)."""
    g = generator(seed, STREAM_DEFOCUS)
    return (g.uniform(lo_um, hi_um, size=n) * 1.0e4).astype(np.float32)


def complex_noise(shape, sigma2: float, seed: int, first_image: int = 0) -> np.ndarray:
    """Complex Gaussian noise of variance sigma2 (real and imaginary parts
    N(0, sigma2/2)), drawn per image from (seed, image index) so the same
    image always receives the same noise.  shape = (n, M, M)."""
    n = shape[0]
    out = np.empty(shape, dtype=np.complex128)
    for i in range(n):
        g = np.random.default_rng([int(seed), STREAM_NOISE, first_image + i])
        out[i] = (g.standard_normal(shape[1:]) + 1j * g.standard_normal(shape[1:])) * math.sqrt(sigma2 / 2)
    return out


def epoch_permutation(N: int, seed: int, epoch: int) -> np.ndarray:
    """Minibatch order of one epoch: a uniform permutation of the N image
    indices, reshuffled per epoch (sampling without replacement)."""
    return np.random.default_rng([int(seed), STREAM_PERM, int(epoch)]).permutation(N).astype(np.int64)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    M: int
    n_blobs: int
    N: int
    batch: int
    defocus_um: tuple
    snr: float
    n_probe: int
    seed: int
    poses: str = "uniform"   # or "vmf"
    kappa: float = 0.0
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "small_32": Workload("small_32", 32, 20, 1000, 32, (1.0, 3.0), 0.1, 50, 1000),
    "mid_128": Workload("mid_128", 128, 200, 50_000, 256, (0.8, 3.0), 0.05, 100, 2000),
    "hires_256": Workload("hires_256", 256, 1000, 200_000, 1024, (1.0, 3.0), float("inf"), 0, 3000),
    "stress_320": Workload("stress_320", 320, 1000, 500_000, 2048, (0.5, 4.0), 0.02, 0, 5000,
                           poses="vmf", kappa=10.0),
}


def workload_poses(w: Workload, n: int | None = None) -> np.ndarray:
    n = w.N if n is None else n
    if w.poses == "vmf":
        return vmf_rotations(n, w.kappa, w.seed)
    return uniform_rotations(n, w.seed)
