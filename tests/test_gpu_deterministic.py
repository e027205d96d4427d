"""The deterministic adjoint on trilinear grids (GPU): every contribution is
rounded to a 64-bit fixed-point integer whose scale depends only on the
number of images and the largest input magnitude, and the integers are summed
exactly.  The outputs are therefore bitwise reproducible, independent of the
order of the images and of how the batch is split into work items and
sub-batches, and the accumulated value is the exact sum of the float
contributions up to one final rounding.

Checked here: agreement with the FP64 oracle (tighter than the fast path's
1e-4, since no partial sum is rounded to float), bitwise repetition, bitwise
invariance under a permutation of the images, batches beyond one sub-batch,
exact scaling by powers of two, zero and non-finite inputs.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def bits(t):
    return t.detach().cpu().numpy().view(np.uint64)


@pytest.fixture(scope="module")
def b():
    from paper_2311_16100_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    binding.lib()
    return binding


def make(M, n, seed, ctf=True, poses="uniform"):
    grid_o = oracle.Grid(M)
    opt_o = oracle.Optics() if ctf else oracle.NO_CTF
    rot = synth.uniform_rotations(n, seed) if poses == "uniform" else synth.vmf_rotations(n, 10.0, seed)
    df = synth.defocus_values(n, 0.5, 4.0, seed)
    vol = synth.random_complex((M, M, M), seed, stream=11)
    img = synth.random_complex((n, M, M), seed, stream=12)
    return grid_o, opt_o, oracle.Poses(rot, df), vol, img


def dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def desc(b, grid_o, opt_o):
    return b.Grid(grid_o.M, r_max=grid_o.rmax, interp=1), (b.Optics() if opt_o.ctf_on else b.NO_CTF)


def disk(M, rmax):
    ax = np.arange(M) - M // 2
    return (ax[:, None] ** 2 + ax[None, :] ** 2) <= rmax ** 2


@pytest.mark.parametrize("power", [0, 1, 2])
def test_backproject_against_oracle(b, power):
    grid_o, opt_o, P, vol, img = make(36, 300, 9)
    g, o = desc(b, grid_o, opt_o)
    rot, df, x, acc0 = dev(P.rot, P.defocus, img, vol)
    want = oracle.backproject(grid_o, opt_o, P, img, ctf_power=power, scale=1.7, accum=vol)
    acc = b.backproject(g, o, rot, df, x, ctf_power=power, scale=1.7, accum=acc0.clone(), deterministic=True)
    assert rel(acc.cpu().numpy(), want) <= 2e-6


def test_gradient_and_hvp_against_oracle(b):
    grid_o, opt_o, P, vol, img = make(36, 300, 10, poses="vmf")
    g, o = desc(b, grid_o, opt_o)
    rot, df, v, x = dev(P.rot, P.defocus, vol, img)
    img_d = img * disk(36, grid_o.rmax)[None]
    gr = b.gradient(g, o, rot, df, v, x, 3.5, 0.2, deterministic=True)
    assert rel(gr.cpu().numpy(), oracle.gradient(grid_o, opt_o, P, vol, img_d, 3.5, 0.2)) <= 2e-6
    hz = b.hvp(g, o, rot, df, v, 2.0, 0.3, deterministic=True)
    assert rel(hz.cpu().numpy(), oracle.hvp(grid_o, opt_o, P, vol, 2.0, 0.3)) <= 2e-6


def test_bitwise_repeatable_and_order_free(b):
    """Three calls agree bit for bit, and so does a call on the images in
    reversed and in shuffled order (the fast path's float sums do not)."""
    grid_o, opt_o, P, vol, img = make(40, 400, 12)
    g, o = desc(b, grid_o, opt_o)
    rot, df, v, x = dev(P.rot, P.defocus, vol, img)
    perms = [np.arange(400), np.arange(400)[::-1].copy(), np.random.default_rng(3).permutation(400)]

    def run(perm, kind):
        p = torch.from_numpy(perm).cuda()
        r, d = rot[p].contiguous(), df[p].contiguous()
        if kind == "backproject":
            return b.backproject(g, o, r, d, x[p].contiguous(), ctf_power=1, scale=0.9, deterministic=True)
        if kind == "gradient":
            return b.gradient(g, o, r, d, v, x[p].contiguous(), 2.0, 0.1, deterministic=True)
        return b.hvp(g, o, r, d, v, 1.5, 0.2, deterministic=True)

    for kind in ("backproject", "gradient", "hvp"):
        ref = bits(run(perms[0], kind))
        assert np.array_equal(ref, bits(run(perms[0], kind))), kind
        for perm in perms[1:]:
            assert np.array_equal(ref, bits(run(perm, kind))), kind


def test_beyond_one_sub_batch(b):
    """2100 images: two sub-batches (2048 + 52) accumulate into one
    fixed-point volume with one scale."""
    grid_o, opt_o, P, vol, img = make(20, 2100, 13)
    g, o = desc(b, grid_o, opt_o)
    rot, df, x = dev(P.rot, P.defocus, img)
    want = oracle.backproject(grid_o, opt_o, P, img, ctf_power=1, scale=0.5)
    got = b.backproject(g, o, rot, df, x, ctf_power=1, scale=0.5, deterministic=True)
    assert rel(got.cpu().numpy(), want) <= 2e-6
    p = torch.arange(2099, -1, -1, device="cuda")
    got_r = b.backproject(g, o, rot[p].contiguous(), df[p].contiguous(), x[p].contiguous(), ctf_power=1,
                          scale=0.5, deterministic=True)
    assert np.array_equal(bits(got), bits(got_r))


@pytest.mark.parametrize("k", [-40, 40])
def test_power_of_two_scaling_is_exact(b, k):
    """Scaling the input by 2^k scales the fixed-point scale by 2^-k and
    leaves every rounded integer unchanged: the output scales exactly."""
    grid_o, opt_o, P, vol, img = make(32, 100, 14)
    g, o = desc(b, grid_o, opt_o)
    rot, df, v, x = dev(P.rot, P.defocus, vol, img)
    f = float(2.0 ** k)
    base = b.backproject(g, o, rot, df, x, ctf_power=2, scale=1.25, deterministic=True)
    scaled = b.backproject(g, o, rot, df, x * f, ctf_power=2, scale=1.25, deterministic=True)
    assert np.array_equal(bits(base * f), bits(scaled))
    base = b.hvp(g, o, rot, df, v, 0.75, 0.0, deterministic=True)
    scaled = b.hvp(g, o, rot, df, v * f, 0.75, 0.0, deterministic=True)
    assert np.array_equal(bits(base * f), bits(scaled))


def test_zero_and_non_finite_inputs(b):
    grid_o, opt_o, P, vol, img = make(24, 30, 15)
    g, o = desc(b, grid_o, opt_o)
    rot, df, v, x = dev(P.rot, P.defocus, vol, img)
    # zero images add exactly nothing
    acc = b.backproject(g, o, rot, df, torch.zeros_like(x), accum=v.clone(), deterministic=True)
    assert np.array_equal(bits(acc), bits(v))
    # a non-finite input makes every voxel NaN (documented)
    bad = x.clone()
    bad[3, 12, 12] = float("inf")
    acc = b.backproject(g, o, rot, df, bad, deterministic=True)
    assert torch.isnan(torch.view_as_real(acc)).all()


def test_agrees_with_fast_path(b):
    grid_o, opt_o, P, vol, img = make(48, 256, 16)
    g, o = desc(b, grid_o, opt_o)
    rot, df, v, x = dev(P.rot, P.defocus, vol, img)
    for det_out, fast_out in (
            (b.gradient(g, o, rot, df, v, x, 1.0, 0.05, deterministic=True),
             b.gradient(g, o, rot, df, v, x, 1.0, 0.05)),
            (b.hvp(g, o, rot, df, v, 1.0, 0.05, deterministic=True), b.hvp(g, o, rot, df, v, 1.0, 0.05)),
            (b.backproject(g, o, rot, df, x, deterministic=True), b.backproject(g, o, rot, df, x))):
        assert rel(det_out.cpu().numpy(), fast_out.cpu().numpy()) <= 1e-5
