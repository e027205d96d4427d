"""GPU parity: every entry point of the C ABI against the FP64 oracle on the
same seeded float32 inputs.

Tolerances (relative L2 over the whole output, and the largest element error
against the largest element): project 1e-5; backproject, gradient, HVP,
Hutchinson and the exact diagonal 1e-4; integer outputs
(Rademacher probes, coverage counts) bit-exact; the deterministic adjoint
bitwise reproducible.  Sizes span several pixel chunks and voxel bricks with
ragged tails (M = 36: 1296 pixels per image = 5 chunks of 256 + 16; 4.5
bricks of 8 per axis), two image-cull rounds of 256 in the voxel kernels
(n = 300), and the benchmark's full 256^3 / 1024-image configuration.  At
full size this module checks sampled images (forward) and 32-image subsets
(adjoint, gradient), the adjoint identity and the fused gradient and HVP
against the composition of the forward and adjoint kernels; the whole batch
is compared with the oracle element by element in
test_gpu_full_size_oracle.py.
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


def close(got, want, tol, what=""):
    """Relative L2 <= tol and, element by element, max|got - want| <= tol *
    max|want| (a wrong brick face or tail cannot hide under the norm)."""
    got = np.asarray(got, dtype=np.complex128).reshape(-1)
    want = np.asarray(want, dtype=np.complex128).reshape(-1)
    e_l2 = rel(got, want)
    e_max = float(np.abs(got - want).max() / np.abs(want).max())
    assert e_l2 <= tol and e_max <= tol, (what, e_l2, e_max)


@pytest.fixture(scope="module")
def b():
    from paper_2311_16100_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    binding.lib()
    return binding


def make_case(M, n, seed, interp=1, ctf=True, blob=False, rmax=None, poses="uniform"):
    grid_o = oracle.Grid(M, r_max=rmax, interp=interp)
    opt_o = oracle.Optics() if ctf else oracle.NO_CTF
    rot = synth.uniform_rotations(n, seed) if poses == "uniform" else synth.vmf_rotations(n, 10.0, seed)
    df = synth.defocus_values(n, 0.5, 4.0, seed)
    if blob:
        vol = synth.blob_volume(M, 12, seed)
    else:
        vol = synth.random_complex((M, M, M), seed, stream=11)
    img = synth.random_complex((n, M, M), seed, stream=12)
    return grid_o, opt_o, oracle.Poses(rot, df), vol, img


def to_dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def gpu_desc(b, grid_o, opt_o):
    g = b.Grid(grid_o.M, r_max=grid_o.rmax, interp=grid_o.interp)
    o = b.Optics() if opt_o.ctf_on else b.NO_CTF
    return g, o


CASES = [
    dict(M=36, n=37, seed=1, interp=1, ctf=True),
    dict(M=36, n=37, seed=2, interp=0, ctf=True),
    dict(M=32, n=20, seed=3, interp=1, ctf=False, blob=True),
    dict(M=16, n=300, seed=4, interp=1, ctf=True),
    dict(M=8, n=5, seed=5, interp=1, ctf=True),
    dict(M=4, n=3, seed=6, interp=1, ctf=True),
    dict(M=32, n=24, seed=7, interp=1, ctf=True, poses="vmf"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "M%d-n%d-i%d" % (c["M"], c["n"], c["interp"]))
def test_project_parity(b, case):
    grid_o, opt_o, P, vol, img = make_case(**case)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    out = b.project(g, o, rot, df, v).cpu().numpy()
    want = oracle.project(grid_o, opt_o, P, vol)
    close(out, want, 1e-5, "project")
    # residual form with the loss accumulated in double
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    res = b.project(g, o, rot, df, v, subtract=x, loss=loss).cpu().numpy()
    mask = np.abs(want) > 0
    want_r = np.where(mask | (np.abs(res) > 0), want - img, 0)
    # pixels outside the disk are zero in both
    disk = _disk(grid_o)
    want_r = (want - img) * disk[None]
    close(res, want_r, 1e-5, "residual")
    want_loss = 0.5 * np.sum(np.abs(want_r) ** 2)
    assert loss.item() == pytest.approx(want_loss, rel=1e-5)


def _disk(grid_o):
    M = grid_o.M
    ax = np.arange(M) - M // 2
    return (ax[:, None] ** 2 + ax[None, :] ** 2) <= grid_o.rmax ** 2


@pytest.mark.parametrize("case", CASES, ids=lambda c: "M%d-n%d-i%d" % (c["M"], c["n"], c["interp"]))
@pytest.mark.parametrize("power", [0, 1, 2])
def test_backproject_parity(b, case, power):
    grid_o, opt_o, P, vol, img = make_case(**case)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, x, acc0 = to_dev(P.rot, P.defocus, img, vol)
    want = oracle.backproject(grid_o, opt_o, P, img, ctf_power=power, scale=1.7, accum=vol)
    for det in (False, True):
        acc = acc0.clone()
        b.backproject(g, o, rot, df, x, ctf_power=power, scale=1.7, accum=acc, deterministic=det)
        close(acc.cpu().numpy(), want, 1e-4, det)


def test_deterministic_backproject_is_bitwise_reproducible(b):
    grid_o, opt_o, P, vol, img = make_case(M=36, n=300, seed=9)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, x = to_dev(P.rot, P.defocus, img)
    outs = []
    for _ in range(3):
        acc = torch.zeros((36, 36, 36), dtype=torch.complex64, device="cuda")
        b.backproject(g, o, rot, df, x, ctf_power=1, accum=acc, deterministic=True)
        outs.append(acc.cpu().numpy())
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    assert np.array_equal(outs[0].view(np.uint64), outs[2].view(np.uint64))
    acc = torch.zeros((36, 36, 36), dtype=torch.complex64, device="cuda")
    b.backproject(g, o, rot, df, x, ctf_power=1, accum=acc, deterministic=False)
    assert rel(acc.cpu().numpy(), outs[0]) <= 1e-5


@pytest.mark.parametrize("case", CASES[:4], ids=lambda c: "M%d-n%d-i%d" % (c["M"], c["n"], c["interp"]))
def test_gradient_and_loss_parity(b, case):
    grid_o, opt_o, P, vol, img = make_case(**case)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    scale, lam = 3.5, 0.2
    disk = _disk(grid_o)
    img_d = img * disk[None]
    want_g = oracle.gradient(grid_o, opt_o, P, vol, img_d, scale, lam)
    want_f = oracle.loss(grid_o, opt_o, P, vol, img_d, scale, lam)
    for det in (False, True):
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        gr = b.gradient(g, o, rot, df, v, x, scale, lam, loss_out=loss, deterministic=det)
        close(gr.cpu().numpy(), want_g, 1e-4, det)
        assert loss.item() == pytest.approx(want_f, rel=1e-5), det


@pytest.mark.parametrize("blob", [False, True])
def test_gradient_parity_mid_size(b, blob):
    """M = 72 with 200 images (several work items per central brick), random
    and blob volumes: against the oracle, and against the deterministic
    (owner-computes) adjoint."""
    grid_o, opt_o, P, vol, img = make_case(M=72, n=200, seed=31, blob=blob)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    scale, lam = 12.5, 0.07
    want = oracle.gradient(grid_o, opt_o, P, vol, img * _disk(grid_o)[None], scale, lam)
    got = b.gradient(g, o, rot, df, v, x, scale, lam)
    det = b.gradient(g, o, rot, df, v, x, scale, lam, deterministic=True)
    close(got.cpu().numpy(), want, 1e-4)
    close(got.cpu().numpy(), det.cpu().numpy(), 1e-5)


@pytest.mark.parametrize("case", CASES[:4], ids=lambda c: "M%d-n%d-i%d" % (c["M"], c["n"], c["interp"]))
def test_hvp_parity(b, case):
    grid_o, opt_o, P, vol, img = make_case(**case)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, z = to_dev(P.rot, P.defocus, vol)
    want = oracle.hvp(grid_o, opt_o, P, vol, 2.0, 0.3)
    for det in (False, True):
        hz = b.hvp(g, o, rot, df, z, 2.0, 0.3, deterministic=det)
        close(hz.cpu().numpy(), want, 1e-4, det)


@pytest.mark.parametrize("same_pose", [False, True], ids=["4poses", "1pose"])
def test_adjoint_sums_that_wrap_32_bits(b, same_pose):
    """The gradient and HVP accumulate both components of a contribution in
    one 64-bit LDS word whose 32-bit halves wrap, with the wraps counted
    apart.  2048 images on four poses (or one pose and one repeated image,
    so that every contribution to a voxel has the same sign) put hundreds of
    contributions of the largest size into each reached voxel: the halves
    wrap many times per voxel and work item.  Against the oracle and the
    deterministic adjoint."""
    M, n = 24, 2048
    rot = synth.uniform_rotations(4, 41)
    rot = np.repeat(rot[:1], n, axis=0) if same_pose else np.tile(rot, (n // 4, 1, 1))
    df = synth.defocus_values(n, 1.0, 3.0, 41)
    if same_pose:
        df[:] = df[0]
    vol = synth.random_complex((M, M, M), 41, stream=11)
    img = synth.random_complex((n, M, M), 41, stream=12)
    if same_pose:
        img[:] = img[0]
    grid_o, opt_o, P = oracle.Grid(M), oracle.Optics(), oracle.Poses(rot, df)
    g, o = gpu_desc(b, grid_o, opt_o)
    rd, dd, v, x = to_dev(P.rot, P.defocus, vol, img)
    scale, lam = 1.5, 0.25
    want = oracle.gradient(grid_o, opt_o, P, vol, img * _disk(grid_o)[None], scale, lam)
    got = b.gradient(g, o, rd, dd, v, x, scale, lam).cpu().numpy()
    det = b.gradient(g, o, rd, dd, v, x, scale, lam, deterministic=True).cpu().numpy()
    close(got, want, 1e-4, "gradient")
    close(got, det, 1e-5, "gradient vs deterministic")
    want = oracle.hvp(grid_o, opt_o, P, vol, scale, lam)
    close(b.hvp(g, o, rd, dd, v, scale, lam).cpu().numpy(), want, 1e-4, "hvp")


def test_rademacher_bit_exact(b):
    for nvox, seed, probe in ((36 ** 3, 5, 0), (1000, 2 ** 40 + 7, 3), (130, 1, 2 ** 33 + 1), (5, 9, 9)):
        z = b.rademacher(nvox, seed, probe).cpu().numpy()
        assert np.array_equal(z, oracle.rademacher(seed, probe, nvox).astype(np.float32))


@pytest.mark.parametrize("n_probe", [1, 4, 5])
def test_hutchinson_parity(b, n_probe):
    grid_o, opt_o, P, vol, img = make_case(M=16, n=40, seed=21)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df = to_dev(P.rot, P.defocus)
    got = b.hutchinson_diag(g, o, rot, df, n_probe, seed=77, scale=2.5, lam=0.1, probe0=3).cpu().numpy()
    want = oracle.hutchinson_diag(grid_o, opt_o, P, n_probe, 77, 2.5, 0.1, probe0=3)
    close(got, want, 1e-4)


def test_hutchinson_parity_many_images(b):
    """More than 128 images per brick: several work items per brick, several
    image windows per item, and their fixed-point accumulators flushed into one
    voxel by global atomics."""
    grid_o, opt_o, P, vol, img = make_case(M=36, n=300, seed=22)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df = to_dev(P.rot, P.defocus)
    got = b.hutchinson_diag(g, o, rot, df, 2, seed=5, scale=0.7, lam=0.02, probe0=11).cpu().numpy()
    want = oracle.hutchinson_diag(grid_o, opt_o, P, 2, 5, 0.7, 0.02, probe0=11)
    close(got, want, 1e-4)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "M%d-n%d-i%d" % (c["M"], c["n"], c["interp"]))
@pytest.mark.parametrize("n_probe", [1, 2, 3])
def test_gradient_hutchinson_parity(b, case, n_probe):
    """csg_gradient_hutchinson against the oracle's gradient, loss and
    Hutchinson diagonal of the same batch (trilinear grids: one kernel forms
    the gradient and the first probe pair's product, a third probe takes the
    probe kernel; nearest-neighbour grids: the two separate paths)."""
    grid_o, opt_o, P, vol, img = make_case(**case)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    scale, lam = 3.5, 0.2
    img_d = img * _disk(grid_o)[None]
    want_g = oracle.gradient(grid_o, opt_o, P, vol, img_d, scale, lam)
    want_f = oracle.loss(grid_o, opt_o, P, vol, img_d, scale, lam)
    want_d = oracle.hutchinson_diag(grid_o, opt_o, P, n_probe, 77, scale, lam, probe0=3)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gr, dg = b.gradient_hutchinson(g, o, rot, df, v, x, scale, lam, n_probe, 77, probe0=3, loss_out=loss)
    close(gr.cpu().numpy(), want_g, 1e-4, "gradient")
    assert loss.item() == pytest.approx(want_f, rel=1e-5)
    close(dg.cpu().numpy(), want_d, 1e-4, "hutchinson")


@pytest.mark.parametrize("M,n,blob", [(36, 300, False), (72, 200, True)])
def test_gradient_hutchinson_many_images(b, M, n, blob):
    """More than 128 images per brick (several chunks per work item, whose
    probe sums are flushed one chunk at a time, several 32-image windows per
    chunk, several work items per brick): the one-kernel gradient and probe
    product against the oracle."""
    grid_o, opt_o, P, vol, img = make_case(M=M, n=n, seed=23, blob=blob)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    scale, lam = 0.7, 0.02
    want_g = oracle.gradient(grid_o, opt_o, P, vol, img * _disk(grid_o)[None], scale, lam)
    want_d = oracle.hutchinson_diag(grid_o, opt_o, P, 2, 5, scale, lam, probe0=11)
    gr, dg = b.gradient_hutchinson(g, o, rot, df, v, x, scale, lam, 2, 5, probe0=11)
    close(gr.cpu().numpy(), want_g, 1e-4, "gradient")
    close(dg.cpu().numpy(), want_d, 1e-4, "hutchinson")


def test_gradient_hutchinson_two_sub_batches(b):
    """2100 images: two launches of the one-pass kernel (2048 + 52 images per
    launch), each adding its gradient and probe sums."""
    grid_o, opt_o, P, vol, img = make_case(M=24, n=2100, seed=26)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gr, dg = b.gradient_hutchinson(g, o, rot, df, v, x, 0.3, 0.05, 2, 9, probe0=4, loss_out=loss)
    img_d = img * _disk(grid_o)[None]
    close(gr.cpu().numpy(), oracle.gradient(grid_o, opt_o, P, vol, img_d, 0.3, 0.05), 1e-4, "gradient")
    assert loss.item() == pytest.approx(oracle.loss(grid_o, opt_o, P, vol, img_d, 0.3, 0.05), rel=1e-5)
    close(dg.cpu().numpy(), oracle.hutchinson_diag(grid_o, opt_o, P, 2, 9, 0.3, 0.05, probe0=4), 1e-4, "hutchinson")


def test_gradient_hutchinson_nearest_neighbour_many_images(b):
    """Nearest-neighbour grids take the two separate calls in the one
    workspace; at 16^3 with 2048 images the gradient's brick tables are the
    larger part of it."""
    grid_o, opt_o, P, vol, img = make_case(M=16, n=2048, seed=25, interp=0)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    ws = b.alloc_workspace(g, 2048, b.CSG_WS_GRADIENT_HUTCHINSON, v.device)
    gr, dg = b.gradient_hutchinson(g, o, rot, df, v, x, 0.5, 0.1, 2, 6, probe0=1, workspace=ws)
    close(gr.cpu().numpy(), oracle.gradient(grid_o, opt_o, P, vol, img * _disk(grid_o)[None], 0.5, 0.1), 1e-4,
          "gradient")
    close(dg.cpu().numpy(), oracle.hutchinson_diag(grid_o, opt_o, P, 2, 6, 0.5, 0.1, probe0=1), 1e-4, "hutchinson")


def test_gradient_hutchinson_with_shifts_and_empty_batch(b):
    """In-plane shifts take the separate gradient and probe kernels (the
    Hessian ignores the shifts); an empty batch leaves the gradient lambda v,
    the loss lambda/2 |v|^2 and the diagonal lambda."""
    grid_o, opt_o, P, vol, img = make_case(M=32, n=24, seed=24)
    shifts = np.random.default_rng(24).uniform(-8.0, 8.0, (P.n, 2)).astype(np.float32)
    Ps = oracle.Poses(P.rot, P.defocus, shifts)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x, sh = to_dev(P.rot, P.defocus, vol, img, shifts)
    img_d = img * _disk(grid_o)[None]
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gr, dg = b.gradient_hutchinson(g, o, rot, df, v, x, 2.0, 0.1, 2, 8, probe0=2, loss_out=loss, shift=sh)
    close(gr.cpu().numpy(), oracle.gradient(grid_o, opt_o, Ps, vol, img_d, 2.0, 0.1), 1e-4, "gradient")
    assert loss.item() == pytest.approx(oracle.loss(grid_o, opt_o, Ps, vol, img_d, 2.0, 0.1), rel=1e-5)
    close(dg.cpu().numpy(), oracle.hutchinson_diag(grid_o, opt_o, P, 2, 8, 2.0, 0.1, probe0=2), 1e-4, "hutchinson")
    loss.zero_()
    gr, dg = b.gradient_hutchinson(g, o, rot[:0], df[:0], v, x[:0], 2.0, 0.1, 2, 8, loss_out=loss)
    vv = vol.astype(np.complex128)
    close(gr.cpu().numpy(), 0.1 * vv, 1e-6, "empty batch: gradient")
    assert loss.item() == pytest.approx(0.05 * np.vdot(vv, vv).real, rel=1e-6)
    assert np.all(dg.cpu().numpy() == np.float32(0.1))


@pytest.mark.parametrize("interp", [0, 1])
def test_exact_diag_and_features_parity(b, interp):
    grid_o, opt_o, P, vol, img = make_case(M=36, n=37, seed=31, interp=interp)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df = to_dev(P.rot, P.defocus)
    d = b.exact_diag(g, o, rot, df, 1.5, 0.25).cpu().numpy()
    close(d, oracle.exact_diag(grid_o, opt_o, P, 1.5, 0.25), 1e-4)
    f2, f3 = b.features(g, o, rot, df)
    w2, w3 = oracle.features(grid_o, opt_o, P)
    assert rel(f2.cpu().numpy(), w2) <= 1e-4
    assert np.array_equal(f3.cpu().numpy(), w3.astype(np.float32))


def test_feature_sums_parity(b):
    # sum C^2 w and sum w are backprojections of an all-ones image stack with
    # the CTF squared and with no CTF
    grid_o, opt_o, P, vol, img = make_case(M=36, n=300, seed=33)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df = to_dev(P.rot, P.defocus)
    acc = b.feature_sums(g, o, rot, df).cpu().numpy()
    ones = np.ones((P.n, 36, 36), np.complex128)
    assert rel(acc.real, oracle.backproject(grid_o, opt_o, P, ones, ctf_power=2).real) <= 1e-5
    assert rel(acc.imag, oracle.backproject(grid_o, opt_o, P, ones, ctf_power=0).real) <= 1e-5
    f2, _ = oracle.features(grid_o, opt_o, P)
    assert rel(acc.real, f2) <= 1e-5


@pytest.mark.parametrize("n", [36 ** 3, 36 ** 3 + 5], ids=["pairs", "odd"])
def test_precond_step_parity(b, n):
    # an even count takes the two-voxel kernel, an odd one the one-voxel kernel
    g0 = np.random.default_rng(3)
    v = synth.random_complex(n, 1).astype(np.complex64)
    gr = synth.random_complex(n, 2).astype(np.complex64)
    D = (g0.uniform(-1, 3, n)).astype(np.float32)
    Da = (g0.uniform(0, 2, n)).astype(np.float32)
    zHz = (g0.uniform(-1, 4, n)).astype(np.float32)
    k, beta, alpha, eta = 7, 0.9, 0.3, 0.7
    vd, gd, Dd, Dad, zd = to_dev(v, gr, D, Da, zHz)
    Dh = torch.empty(n, dtype=torch.float32, device="cuda")
    vo, st = b.precond_sgd_step(vd, gd, Dd, Dad, zd, k, beta, alpha, eta, Dhat_out=Dh)
    wD, wDa, wDh = oracle.precond_update(D.astype(np.float64), Da.astype(np.float64), zHz.astype(np.float64),
                                         k, beta, alpha)
    wv, wgn = oracle.precond_step(v, gr, wDh, eta)
    assert np.allclose(Dd.cpu().numpy(), wD, rtol=1e-6, atol=1e-6)
    assert np.allclose(Dad.cpu().numpy(), wDa, rtol=1e-6, atol=1e-6)
    assert np.allclose(Dh.cpu().numpy(), wDh, rtol=1e-6, atol=1e-6)
    assert rel(vo.cpu().numpy(), wv) <= 1e-6
    s = st.cpu().numpy()
    assert s[0] == pytest.approx(wgn, rel=1e-6)
    assert s[1] == pytest.approx(np.sum(np.abs(wv) ** 2), rel=1e-6)
    # plain SGD (D = NULL) and a fixed preconditioner (no probe sample)
    vo2, st2 = b.precond_sgd_step(vd, gd, None, None, None, 0, beta, alpha, eta)
    wv2, wgn2 = oracle.precond_step(v, gr, None, eta)
    assert rel(vo2.cpu().numpy(), wv2) <= 1e-6 and st2[0].item() == pytest.approx(wgn2, rel=1e-6)


def test_unaligned_buffers_take_the_one_voxel_kernels(b):
    """Buffers that are 8- but not 16-byte aligned: the step and the
    Hutchinson product give the same results as with aligned buffers."""
    nv = 36 ** 3
    v = torch.from_numpy(synth.random_complex(nv, 4).astype(np.complex64)).cuda()
    g = torch.from_numpy(synth.random_complex(nv, 5).astype(np.complex64)).cuda()
    D = torch.rand(nv, device="cuda") + 0.5
    Da = torch.rand(nv, device="cuda")
    z = torch.rand(nv, device="cuda")
    # offset copies: element 1 of a buffer one element longer
    def off(t):
        big = torch.empty(t.numel() + 1, dtype=t.dtype, device="cuda")
        big[1:] = t
        return big[1:]
    vu, gu, Du, Dau, zu = off(v), off(g), off(D), off(Da), off(z)
    assert vu.data_ptr() % 16 == 8
    vo, st = b.precond_sgd_step(v, g, D, Da, z, 3, 0.9, 0.2, 0.5)
    vou = off(torch.empty_like(v))
    _, stu = b.precond_sgd_step(vu, gu, Du, Dau, zu, 3, 0.9, 0.2, 0.5, v_out=vou)
    assert torch.equal(vo, vou) and torch.equal(D, Du) and torch.equal(Da, Dau)
    assert stu.cpu().numpy() == pytest.approx(st.cpu().numpy(), rel=1e-12)
    # the Hutchinson diagonal into a 4-byte-offset output, the gradient into an
    # 8-byte-offset one
    grid_o, opt_o, P, vol, img = make_case(M=36, n=40, seed=24)
    gg, o = gpu_desc(b, grid_o, opt_o)
    rot, df, vd, xd = to_dev(P.rot, P.defocus, vol, img)
    d1 = b.hutchinson_diag(gg, o, rot, df, 3, seed=9, scale=1.5, lam=0.1)
    d2 = off(torch.empty(nv, device="cuda"))
    assert d2.data_ptr() % 8 == 4
    b.hutchinson_diag(gg, o, rot, df, 3, seed=9, scale=1.5, lam=0.1, diag_out=d2)
    assert rel(d2.cpu().numpy(), d1.reshape(-1).cpu().numpy()) <= 1e-6
    g1 = b.gradient(gg, o, rot, df, vd, xd, 2.0, 0.1)
    g2 = off(torch.empty(nv, dtype=torch.complex64, device="cuda")).reshape(36, 36, 36)
    b.gradient(gg, o, rot, df, vd, xd, 2.0, 0.1, grad_out=g2)
    assert rel(g2.cpu().numpy(), g1.cpu().numpy()) <= 1e-6


def test_sub_batches_beyond_2048_images(b):
    # the brick kernels process at most 2048 images per launch; larger
    # batches run in sub-batches that accumulate into the same outputs
    grid_o, opt_o, P, vol, img = make_case(M=16, n=2100, seed=41)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    assert rel(b.project(g, o, rot, df, v).cpu().numpy(), oracle.project(grid_o, opt_o, P, vol)) <= 1e-5
    acc = b.backproject(g, o, rot, df, x, ctf_power=1, scale=0.5)
    assert rel(acc.cpu().numpy(), oracle.backproject(grid_o, opt_o, P, img, 1, 0.5)) <= 1e-4
    hz = b.hvp(g, o, rot, df, v, 1.0, 0.1)
    assert rel(hz.cpu().numpy(), oracle.hvp(grid_o, opt_o, P, vol, 1.0, 0.1)) <= 1e-4


def test_empty_and_degenerate_inputs(b):
    M = 16
    g, o = b.Grid(M), b.Optics()
    rot = torch.zeros((0, 3, 3), device="cuda")
    df = torch.zeros(0, device="cuda")
    v = torch.ones((M, M, M), dtype=torch.complex64, device="cuda")
    out = b.project(g, o, rot, df, v)
    assert out.shape == (0, M, M)
    acc = torch.zeros_like(v)
    b.backproject(g, o, rot, df, torch.zeros((0, M, M), dtype=torch.complex64, device="cuda"), accum=acc)
    assert torch.count_nonzero(acc).item() == 0
    # lambda z alone when the batch is empty
    hz = b.hvp(g, o, rot, df, v, 1.0, 0.5)
    assert torch.allclose(hz, 0.5 * v)
    # r_max = 0: only the DC pixel is used, C(0) = -A
    P = oracle.Poses(synth.uniform_rotations(3, 1), synth.defocus_values(3, 1, 2, 1))
    rd, dd = to_dev(P.rot, P.defocus)
    g0 = b.Grid(M, r_max=0.0)
    out = b.project(g0, o, rd, dd, v).cpu().numpy()
    assert np.count_nonzero(out) == 3
    assert np.allclose(out[:, M // 2, M // 2], -0.1, atol=1e-7)
    # invalid input is rejected, not run
    with pytest.raises(b.CsgError):
        b.project(b.Grid(M, r_max=float(M)), o, rd, dd, v)
    with pytest.raises(b.CsgError):
        b.project(g, o, rd, dd, torch.ones((M, M, M + 2), dtype=torch.complex64, device="cuda"))


@pytest.mark.parametrize("scale", [1e-12, 1e12])
def test_hutchinson_extreme_scales(b, scale):
    """The fixed-point scale of the probe product follows the bound over 24
    orders of magnitude of the data scale."""
    grid_o, opt_o, P, vol, img = make_case(M=36, n=50, seed=23)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df = to_dev(P.rot, P.defocus)
    nv = 36 ** 3
    za = b.rademacher(nv, 3, 0)
    zb = b.rademacher(nv, 3, 1)
    hz = b.hvp(g, o, rot, df, torch.complex(za, zb).reshape(36, 36, 36), scale, 0.0)
    want = (za * hz.real.reshape(-1) + zb * hz.imag.reshape(-1)) / 2
    got = b.hutchinson_diag(g, o, rot, df, 2, seed=3, scale=scale, lam=0.0, probe0=0).reshape(-1)
    assert rel(got.cpu().numpy(), want.cpu().numpy()) <= 1e-4


def _vdot_chunked(a, c):
    """<a, c> in complex128 over z-planes (a 1024^3 volume is too large to
    promote at once)."""
    t = torch.zeros((), dtype=torch.complex128, device=a.device)
    for z0 in range(0, a.shape[0], 64):
        t += torch.vdot(a[z0:z0 + 64].reshape(-1).to(torch.complex128), c[z0:z0 + 64].reshape(-1).to(torch.complex128))
    return t


def test_max_grid_side(b):
    """M = 1024, the largest grid the library accepts; comparisons on the
    device (one volume is 8.6 GB).  Axis-aligned rotations put every sample
    point on a voxel, so their projections are exact copies of the central
    plane; for random rotations the adjoint identity holds, and the fused
    gradient equals the forward/adjoint composition."""
    M, h = 1024, 512
    gen = torch.Generator(device="cuda").manual_seed(1024)
    v = torch.complex(torch.randn((M, M, M), generator=gen, device="cuda"),
                      torch.randn((M, M, M), generator=gen, device="cuda"))
    g = b.Grid(M)
    # identity and a quarter turn about z, no CTF
    rot = torch.tensor([[[1, 0, 0], [0, 1, 0], [0, 0, 1]], [[0, -1, 0], [1, 0, 0], [0, 0, 1]]],
                       dtype=torch.float32, device="cuda")
    df = torch.full((2,), 1.5e4, dtype=torch.float32, device="cuda")
    y = b.project(g, b.NO_CTF, rot, df, v)
    ax = torch.arange(M, device="cuda") - h
    KY, KX = torch.meshgrid(ax, ax, indexing="ij")
    disk = KX ** 2 + KY ** 2 <= (h - 1) ** 2
    zero = torch.zeros((), dtype=torch.complex64, device="cuda")
    plane = v[h]
    assert torch.equal(y[0], torch.where(disk, plane, zero))
    # pixel (kx, ky) of the quarter turn samples voxel (x, y, z) = (ky, -kx, 0) + h
    assert torch.equal(y[1], torch.where(disk, plane[(-KX + h).clamp(0, M - 1), (KY + h).clamp(0, M - 1)], zero))
    del y
    # random rotations, CTF on
    n = 3
    rr = torch.from_numpy(synth.uniform_rotations(n, 77)).cuda()
    dd = torch.from_numpy(synth.defocus_values(n, 1.0, 3.0, 77)).cuda()
    x = torch.complex(torch.randn((n, M, M), generator=gen, device="cuda"),
                      torch.randn((n, M, M), generator=gen, device="cuda"))
    o = b.Optics()
    Av = b.project(g, o, rr, dd, v)
    At = b.backproject(g, o, rr, dd, x, ctf_power=1)
    lhs = torch.vdot(Av.reshape(-1).to(torch.complex128), x.reshape(-1).to(torch.complex128))
    rhs = _vdot_chunked(v, At)
    assert abs((lhs - rhs).item()) <= 1e-5 * abs(lhs.item())
    del At, Av
    scale, lam = 3.0, 0.05
    gr = b.gradient(g, o, rr, dd, v, x, scale, lam)
    comp = b.backproject(g, o, rr, dd, b.project(g, o, rr, dd, v, subtract=x), ctf_power=1, scale=scale)
    comp += lam * v
    diff = gr - comp
    del gr
    err = _vdot_chunked(diff, diff).real.sqrt()
    ref = _vdot_chunked(comp, comp).real.sqrt()
    assert (err / ref).item() <= 1e-5


# ---------------------------------------------------------------------------
# Full size: 256^3 volume, a batch of 1024 images of 256 x 256 -- the
# configuration the benchmark times, in the same launch configuration.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def full(b):
    M, n = 256, 1024
    grid_o = oracle.Grid(M)
    P = oracle.Poses(synth.uniform_rotations(n, 3000), synth.defocus_values(n, 1.0, 3.0, 3000))
    vol = synth.blob_volume(M, 1000, 3000)
    rot, df, v = to_dev(P.rot, P.defocus, vol)
    return grid_o, P, vol, rot, df, v


def test_full_size_project_sampled(b, full):
    grid_o, P, vol, rot, df, v = full
    g, o = b.Grid(256), b.Optics()
    out = b.project(g, o, rot, df, v)
    torch.cuda.synchronize()
    idx = [0, 1, 511, 1023]
    want = oracle.project(grid_o, oracle.Optics(), P.subset(idx), vol)
    got = out[idx].cpu().numpy()
    assert rel(got, want) <= 1e-5


def test_full_size_backproject_and_adjoint(b, full):
    grid_o, P, vol, rot, df, v = full
    g, o = b.Grid(256), b.Optics()
    n = P.n
    x = torch.from_numpy(synth.random_complex((n, 256, 256), 5, stream=13)).cuda()
    acc = b.backproject(g, o, rot, df, x, ctf_power=1)
    # sampled against the oracle: the subset {0..31} backprojected alone
    sub = list(range(32))
    acc_sub = b.backproject(g, o, rot[sub].contiguous(), df[sub].contiguous(), x[sub].contiguous(), ctf_power=1)
    want_sub = oracle.backproject(grid_o, oracle.Optics(), P.subset(sub), x[sub].cpu().numpy(), ctf_power=1)
    assert rel(acc_sub.cpu().numpy(), want_sub) <= 1e-4
    # adjoint identity of the full batch, inner products in double
    Av = b.project(g, o, rot, df, v)
    lhs = torch.vdot(Av.reshape(-1).to(torch.complex128), x.reshape(-1).to(torch.complex128))
    rhs = torch.vdot(v.reshape(-1).to(torch.complex128), acc.reshape(-1).to(torch.complex128))
    assert abs((lhs - rhs).item()) <= 1e-5 * abs(lhs.item())


def test_full_size_gradient_matches_composition(b, full):
    """The fused gradient of the full 1024-image batch (the launch the
    benchmark times) equals the composition of the separately checked
    forward and adjoint kernels, lam v + scale P^T C (C P v - x), and its loss
    the forward pass's residual norm."""
    grid_o, P, vol, rot, df, v = full
    g, o = b.Grid(256), b.Optics()
    x = torch.from_numpy(synth.random_complex((P.n, 256, 256), 7, stream=14)).cuda()
    scale, lam = 195.3, 0.05
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gr = b.gradient(g, o, rot, df, v, x, scale, lam, loss_out=loss)
    l_res = torch.zeros(1, dtype=torch.float64, device="cuda")
    r = b.project(g, o, rot, df, v, subtract=x, loss=l_res)
    want = b.backproject(g, o, rot, df, r, ctf_power=1, scale=scale) + lam * v
    assert rel(gr.cpu().numpy(), want.cpu().numpy()) <= 1e-5
    vn2 = torch.vdot(v.reshape(-1).to(torch.complex128), v.reshape(-1).to(torch.complex128)).real
    assert loss.item() == pytest.approx(scale * l_res.item() + 0.5 * lam * vn2.item(), rel=1e-6)


def test_full_size_gradient_subset_vs_oracle(b, full):
    grid_o, P, vol, rot, df, v = full
    g, o = b.Grid(256), b.Optics()
    sub = list(range(32))
    x = synth.random_complex((32, 256, 256), 8, stream=15)
    x_d = torch.from_numpy(x).cuda()
    scale, lam = 6250.0, 0.05
    gr = b.gradient(g, o, rot[sub].contiguous(), df[sub].contiguous(), v, x_d, scale, lam)
    want = oracle.gradient(grid_o, oracle.Optics(), P.subset(sub), vol, x * _disk(grid_o)[None], scale, lam)
    assert rel(gr.cpu().numpy(), want) <= 1e-4


def test_full_size_hvp_matches_composition(b, full):
    grid_o, P, vol, rot, df, v = full
    g, o = b.Grid(256), b.Optics()
    z = torch.from_numpy(synth.random_complex((256, 256, 256), 9, stream=16)).cuda()
    scale, lam = 195.3, 0.05
    hz = b.hvp(g, o, rot, df, z, scale, lam)
    want = b.backproject(g, o, rot, df, b.project(g, o, rot, df, z), ctf_power=1, scale=scale) + lam * z
    assert rel(hz.cpu().numpy(), want.cpu().numpy()) <= 1e-5


def test_full_size_hutchinson_matches_general_hvp(b, full):
    """The Hutchinson probe product of the full batch (fixed-point packed
    accumulator) against the general HVP (double accumulator) of the same
    Rademacher pair: z_a (H z_a) / 2 + z_b (H z_b) / 2."""
    grid_o, P, vol, rot, df, v = full
    g, o = b.Grid(256), b.Optics()
    nv = 256 ** 3
    scale, lam = 195.3, 0.05
    za = b.rademacher(nv, 99, 6)
    zb = b.rademacher(nv, 99, 7)
    z = torch.complex(za, zb).reshape(256, 256, 256)
    hz = b.hvp(g, o, rot, df, z, scale, lam)
    want = (za * hz.real.reshape(-1) + zb * hz.imag.reshape(-1)) / 2
    got = b.hutchinson_diag(g, o, rot, df, 2, seed=99, scale=scale, lam=lam, probe0=6).reshape(-1)
    assert rel(got.cpu().numpy(), want.cpu().numpy()) <= 1e-5


@pytest.mark.parametrize("M", [16, 34])
def test_fsc_parity(b, M):
    """Fourier shell correlation (eq. (fsc)) of two related random volumes:
    library shell sums against the oracle, per shell."""
    u = synth.random_complex((M, M, M), 100 + M)
    v = (0.6 * u + 0.8 * synth.random_complex((M, M, M), 200 + M)).astype(np.complex64)
    ref = oracle.fsc(u, v, M)
    got = b.fsc(b.Grid(M), *to_dev(u, v)).cpu().numpy()
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) < 1e-6
    sums = b.shell_sums(b.Grid(M), *to_dev(u, u)).cpu().numpy()
    assert np.allclose(sums[0], sums[1]) and np.allclose(sums[1], sums[2])


SHIFT_CASES = [
    dict(M=36, n=37, seed=41, interp=1, ctf=True),
    dict(M=32, n=300, seed=42, interp=1, ctf=True, poses="vmf"),
    dict(M=16, n=9, seed=43, interp=0, ctf=True),
]


@pytest.mark.parametrize("case", SHIFT_CASES, ids=lambda c: "M%d-n%d-i%d" % (c["M"], c["n"], c["interp"]))
def test_in_plane_shift_parity(b, case):
    """Forward, adjoint (fast and deterministic) and gradient with in-plane
    shifts T_i against the oracle; the Hessian ignores them."""
    grid_o, opt_o, P, vol, img = make_case(**case)
    shifts = np.random.default_rng(case["seed"]).uniform(-0.3 * case["M"], 0.3 * case["M"], (P.n, 2))
    Ps = oracle.Poses(P.rot, P.defocus, shifts.astype(np.float32))
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x, sh = to_dev(P.rot, P.defocus, vol, img, Ps.shift)
    want = oracle.project(grid_o, opt_o, Ps, vol)
    assert rel(b.project(g, o, rot, df, v, shift=sh).cpu().numpy(), want) <= 1e-5
    want_b = oracle.backproject(grid_o, opt_o, Ps, img, ctf_power=1, scale=1.3)
    for det in (False, True):
        acc = b.backproject(g, o, rot, df, x, ctf_power=1, scale=1.3, deterministic=det, shift=sh)
        assert rel(acc.cpu().numpy(), want_b) <= 1e-4, det
    img_d = img * _disk(grid_o)[None]
    want_g = oracle.gradient(grid_o, opt_o, Ps, vol, img_d, 2.0, 0.1)
    want_f = oracle.loss(grid_o, opt_o, Ps, vol, img_d, 2.0, 0.1)
    for det in (False, True):
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        gr = b.gradient(g, o, rot, df, v, x, 2.0, 0.1, loss_out=loss, deterministic=det, shift=sh)
        assert rel(gr.cpu().numpy(), want_g) <= 1e-4, det
        assert loss.item() == pytest.approx(want_f, rel=1e-5), det
    # without shifts the results differ (the shift is applied at all)
    assert rel(b.project(g, o, rot, df, v).cpu().numpy(), want) > 1e-2


def test_non_finite_inputs_give_nan(b):
    """The fast adjoint bounds its fixed-point LDS sums by the largest input
    magnitude; a non-finite image value or volume value must surface as NaN,
    not as a wrapped integer."""
    grid_o, opt_o, P, vol, img = make_case(M=24, n=30, seed=17)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    bad = x.clone()
    bad[3, 12, 12] = float("inf")
    acc = b.backproject(g, o, rot, df, bad)
    assert torch.isnan(torch.view_as_real(acc)).any()
    vbad = v.clone()
    vbad[12, 12, 12] = float("nan")
    for out in (b.gradient(g, o, rot, df, vbad, x, 1.0, 0.0), b.hvp(g, o, rot, df, vbad, 1.0, 0.0)):
        assert torch.isnan(torch.view_as_real(out)).any()
    # finite inputs stay finite
    assert torch.isfinite(torch.view_as_real(b.gradient(g, o, rot, df, v, x, 1.0, 0.0))).all()


@pytest.mark.parametrize("k", [-100, 100])
def test_fast_adjoint_far_from_unit_scale(b, k):
    """The per-item fixed-point scale follows the data: inputs scaled by 2^k
    give outputs scaled by 2^k (to float rounding), for the adjoint, the
    gradient and the HVP."""
    grid_o, opt_o, P, vol, img = make_case(M=32, n=60, seed=18)
    g, o = gpu_desc(b, grid_o, opt_o)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol, img)
    f = float(2.0 ** k)
    pairs = (
        (b.backproject(g, o, rot, df, x, ctf_power=1), b.backproject(g, o, rot, df, x * f, ctf_power=1)),
        (b.gradient(g, o, rot, df, v, x, 1.5, 0.0), b.gradient(g, o, rot, df, v * f, x * f, 1.5, 0.0)),
        (b.hvp(g, o, rot, df, v, 1.5, 0.0), b.hvp(g, o, rot, df, v * f, 1.5, 0.0)),
    )
    for base, scaled in pairs:
        want = base.cpu().numpy().astype(np.complex128) * f
        assert rel(scaled.cpu().numpy().astype(np.complex128), want) <= 1e-6


def test_fast_adjoint_redoes_items_above_the_guess(b):
    """The fast adjoint starts each block from a guess of the largest image
    value (a sample of the disk's inner square and lowest frequencies) and
    redoes an item that meets a larger one.  Here the images are small inside
    and large only on the disk's outer ring, which the sample never sees, so
    every item that reaches the ring is redone: the results must still match
    the oracle and the exact (fixed-point deterministic) path."""
    grid_o, opt_o, P, vol, img = make_case(M=40, n=300, seed=19)
    g, o = gpu_desc(b, grid_o, opt_o)
    M = 40
    ax = np.arange(M) - M // 2
    r2 = ax[:, None] ** 2 + ax[None, :] ** 2
    ring = (r2 > 0.8 * grid_o.rmax ** 2) & (r2 <= grid_o.rmax ** 2)
    x_np = (img * np.where(ring, 1.0, 1e-3)[None]).astype(np.complex64)
    rot, df, v, x = to_dev(P.rot, P.defocus, vol * 1e-3, x_np)
    want = oracle.backproject(grid_o, opt_o, P, x_np, ctf_power=1, scale=1.0)
    got = b.backproject(g, o, rot, df, x, ctf_power=1).cpu().numpy()
    det = b.backproject(g, o, rot, df, x, ctf_power=1, deterministic=True).cpu().numpy()
    assert rel(got, want) <= 1e-4
    assert rel(got, det) <= 1e-5
    disk = _disk(grid_o)
    want_g = oracle.gradient(grid_o, opt_o, P, vol * 1e-3, x_np * disk[None], 2.0, 0.1)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gr = b.gradient(g, o, rot, df, v, x, 2.0, 0.1, loss_out=loss).cpu().numpy()
    gd = b.gradient(g, o, rot, df, v, x, 2.0, 0.1, deterministic=True).cpu().numpy()
    assert rel(gr, want_g) <= 1e-4
    assert rel(gr, gd) <= 1e-5
    assert loss.item() == pytest.approx(oracle.loss(grid_o, opt_o, P, vol * 1e-3, x_np * disk[None], 2.0, 0.1),
                                        rel=1e-5)


def test_diagonal_update_alone(b):
    """csg_precond_sgd_step with no step (v, g, v_out, stats NULL): the
    running mean, the exponential average and D_hat only."""
    n = 4097
    g0 = np.random.default_rng(31)
    D = g0.uniform(-1, 3, n).astype(np.float32)
    Da = g0.uniform(0, 2, n).astype(np.float32)
    zHz = g0.uniform(-1, 4, n).astype(np.float32)
    Dd, Dad, zd = to_dev(D, Da, zHz)
    Dh = torch.empty(n, dtype=torch.float32, device="cuda")
    b.diag_update(Dd, Dad, zd, 5, 0.9, 0.4, Dhat_out=Dh)
    wD, wDa, wDh = oracle.precond_update(D.astype(np.float64), Da.astype(np.float64), zHz.astype(np.float64),
                                         5, 0.9, 0.4)
    assert np.allclose(Dd.cpu().numpy(), wD, rtol=1e-6, atol=1e-6)
    assert np.allclose(Dad.cpu().numpy(), wDa, rtol=1e-6, atol=1e-6)
    assert np.allclose(Dh.cpu().numpy(), wDh, rtol=1e-6, atol=1e-6)


def test_precomputed_diagonal_parity(b):
    """Sec. 4.1's precomputed preconditioner (three epochs of minibatches,
    Hutchinson samples, running mean and exponential average) against the
    oracle's run over the same minibatches and probes."""
    from paper_2311_16100_amd import experiment as E
    M, N, Bt, epochs = 20, 48, 16, 3
    grid_o, opt_o = oracle.Grid(M), oracle.Optics()
    rot = synth.uniform_rotations(N, 32)
    df = synth.defocus_values(N, 1.0, 3.0, 32)
    lam = 0.05
    D, Da, k = E.precomputed_diagonal(b.Grid(M), b.Optics(), torch.from_numpy(rot).cuda(),
                                      torch.from_numpy(df).cuda(), lam, epochs, Bt, n_probe=2, probe_seed=33,
                                      perm_seed=34)
    batches = [synth.epoch_permutation(N, 34, e)[s:s + Bt] for e in range(epochs) for s in range(0, N - Bt + 1, Bt)]
    assert k == len(batches)
    wD, wDa = oracle.precomputed_diagonal(grid_o, opt_o, oracle.Poses(rot, df), batches, N / Bt, lam, 0.9, 2, 33)
    close(D.cpu().numpy(), wD, 1e-4, "D")
    close(Da.cpu().numpy(), wDa, 1e-4, "D_avg")
