"""The projector as a torch.autograd.Function: its gradient against the FP64
oracle gradient and against FP64 central finite differences of the oracle
loss (step 1e-6), at 256^3 on a 32-image subset and at 32^3 on 64 voxels;
and autograd HVPs against csg_hvp."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    from paper_2311_16100_amd import autograd as AG
    from paper_2311_16100_amd import binding as B
    B.lib()
    return AG, B


def _setup(M, n, seed, blobs):
    rot = synth.uniform_rotations(n, seed)
    df = synth.defocus_values(n, 1.0, 3.0, seed)
    vol = synth.blob_volume(M, blobs, seed)
    v0 = synth.random_complex((M, M, M), seed, stream=21) * np.float32(0.1) + vol
    x = synth.random_complex((n, M, M), seed, stream=22)
    ax = np.arange(M) - M // 2
    disk = (ax[:, None] ** 2 + ax[None, :] ** 2) <= (M // 2 - 1) ** 2
    x = (x * disk[None]).astype(np.complex64)
    return rot, df, v0.astype(np.complex64), x


@pytest.mark.parametrize("M,n,n_vox", [(32, 24, 64), (256, 32, 6)])
def test_autograd_gradient_vs_oracle_and_fd(mods, M, n, n_vox):
    AG, B = mods
    rot, df, v0, x = _setup(M, n, 3000 + M, 1000 if M == 256 else 20)
    dev = torch.device("cuda:0")
    g_, o_ = B.Grid(M), B.Optics()
    rd, dd, xd = (torch.from_numpy(a).to(dev) for a in (rot, df, x))
    v = torch.from_numpy(v0).to(dev).requires_grad_(True)
    y = AG.project(v, g_, o_, rd, dd)
    L = 0.5 * torch.sum(torch.abs(y - xd) ** 2)
    L.backward()
    got = v.grad.detach().cpu().numpy().astype(np.complex128)
    go, oo, P = oracle.Grid(M), oracle.Optics(), oracle.Poses(rot, df)
    want = oracle.gradient(go, oo, P, v0, x, 1.0, 0.0)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-4
    # FP64 central differences of the oracle loss, real and imaginary parts
    rng = np.random.default_rng(M)
    ball = np.flatnonzero(synth.ball_mask(M, M // 4).reshape(-1))
    h = 1e-6
    v64 = v0.astype(np.complex128).reshape(-1)
    gflat = got.reshape(-1)
    scale_g = np.max(np.abs(want))
    for k in rng.choice(ball, n_vox, replace=False):
        for unit in (1.0, 1j):
            vp = v64.copy(); vp[k] += unit * h
            vm = v64.copy(); vm[k] -= unit * h
            fd = (oracle.loss(go, oo, P, vp, x, 1.0, 0.0) - oracle.loss(go, oo, P, vm, x, 1.0, 0.0)) / (2 * h)
            comp = gflat[k].real if unit == 1.0 else gflat[k].imag
            assert abs(fd - comp) <= 2e-4 * scale_g + 1e-3 * abs(fd), (k, unit, fd, comp)


def test_autograd_hvp_matches_hvp_kernel(mods):
    AG, B = mods
    M, n = 48, 40
    rot, df, v0, x = _setup(M, n, 7, 20)
    dev = torch.device("cuda:0")
    g_, o_ = B.Grid(M), B.Optics()
    rd, dd, z = (torch.from_numpy(a).to(dev) for a in (rot, df, v0))
    h1 = AG.hvp_autograd(z, g_, o_, rd, dd, scale=2.0, lam=0.3)
    h2 = B.hvp(g_, o_, rd, dd, z, 2.0, 0.3)
    assert (torch.linalg.vector_norm(h1 - h2) / torch.linalg.vector_norm(h2)).item() <= 1e-5
    want = oracle.hvp(oracle.Grid(M), oracle.Optics(), oracle.Poses(rot, df), v0, 2.0, 0.3)
    got = h1.cpu().numpy()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-4


def test_autograd_with_in_plane_shifts(mods):
    """The autograd projector with shifts T_i: gradient of a data term against
    the oracle gradient, and the HVP obtained by differentiation equals the
    shift-free Hessian product (T^* T = I)."""
    AG, B = mods
    M, n = 32, 20
    rot, df, v0, x = _setup(M, n, 11, 20)
    shifts = np.random.default_rng(3).uniform(-5, 5, (n, 2)).astype(np.float32)
    dev = torch.device("cuda:0")
    g_, o_ = B.Grid(M), B.Optics()
    rd, dd, xd, sd = (torch.from_numpy(a).to(dev) for a in (rot, df, x, shifts))
    v = torch.from_numpy(v0).to(dev).requires_grad_(True)
    L = 0.5 * torch.sum(torch.abs(AG.project(v, g_, o_, rd, dd, sd) - xd) ** 2)
    L.backward()
    P = oracle.Poses(rot, df, shifts)
    want = oracle.gradient(oracle.Grid(M), oracle.Optics(), P, v0, x, 1.0, 0.0)
    got = v.grad.detach().cpu().numpy()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-4
    z = torch.from_numpy(v0).to(dev)
    h_shift = AG.hvp_autograd(z, g_, o_, rd, dd, scale=1.0, lam=0.0, shift=sd)
    h_plain = B.hvp(g_, o_, rd, dd, z, 1.0, 0.0)
    assert (torch.linalg.vector_norm(h_shift - h_plain) / torch.linalg.vector_norm(h_plain)).item() <= 1e-5
