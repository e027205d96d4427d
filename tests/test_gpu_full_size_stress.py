"""The stress workload's launch against the FP64 oracle, element by element:
a 320^3 volume of 1000 blobs and one batch of 2048 images of 320 x 320 with
preferred orientations (von Mises-Fisher viewing directions, kappa 10) and
defocus 0.5-4 um, as the time-to-accuracy runs on that set launch them (one
call over the batch).  Preferred orientations pile many images onto the
same central bricks, so the fast adjoint's packed LDS sums wrap their 32-bit
halves often there.

Compared with the oracle: the fast and the deterministic gradient and loss
(the runs on this set use the deterministic one), the Hutchinson probe pair,
and both from the kernel that forms them in one pass.  Bounds, written here: relative L2 <= 1e-4 and, per element,
max|got - want| <= 1e-4 max|want|.  The oracle's C loops run over chunks of
the batch in threads; the chunks' volumes are summed in chunk order (a split
of the sum over images of the definitions).
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

M, N_IMG, SEED, KAPPA = 320, 2048, 5320, 10.0
THREADS = 8


def close(got, want, tol, what):
    got = np.asarray(got, dtype=np.complex128).reshape(-1)
    want = np.asarray(want, dtype=np.complex128).reshape(-1)
    e_l2 = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    e_max = float(np.abs(got - want).max() / np.abs(want).max())
    print("[stress] %s: relative L2 %.2e, max element error / max %.2e" % (what, e_l2, e_max), flush=True)
    assert e_l2 <= tol and e_max <= tol, (what, e_l2, e_max)


def _chunks(n):
    step = (n + THREADS - 1) // THREADS
    return [list(range(s, min(n, s + step))) for s in range(0, n, step)]


def o_project(grid, opt, P, vol):
    with ThreadPoolExecutor(THREADS) as ex:
        outs = list(ex.map(lambda idx: oracle.project(grid, opt, P.subset(idx), vol), _chunks(P.n)))
    return np.concatenate(outs)


def o_backproject(grid, opt, P, img, scale):
    with ThreadPoolExecutor(THREADS) as ex:
        vols = list(ex.map(lambda idx: oracle.backproject(grid, opt, P.subset(idx), img[idx], ctf_power=1,
                                                          scale=scale), _chunks(P.n)))
    acc = vols[0]
    for v in vols[1:]:
        acc = acc + v
    return acc


@pytest.fixture(scope="module")
def stress():
    from paper_2311_16100_amd import binding as b
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    b.lib()
    grid = oracle.Grid(M)
    P = oracle.Poses(synth.vmf_rotations(N_IMG, KAPPA, SEED), synth.defocus_values(N_IMG, 0.5, 4.0, SEED))
    vol = synth.blob_volume(M, 1000, SEED)
    dev = torch.device("cuda:0")
    return b, grid, P, vol, torch.from_numpy(P.rot).to(dev), torch.from_numpy(P.defocus).to(dev), \
        torch.from_numpy(vol).to(dev)


def test_stress_batch_gradient_and_loss(stress):
    b, grid, P, vol, rot, df, v = stress
    ax = np.arange(M) - M // 2
    disk = (ax[:, None] ** 2 + ax[None, :] ** 2) <= grid.rmax ** 2
    # data near the model's images, plus noise
    y = o_project(grid, oracle.Optics(), P, vol)
    x = ((0.7 * y + 20.0 * synth.random_complex((N_IMG, M, M), 11, stream=17)) * disk[None]).astype(np.complex64)
    scale, lam = 244.1, 0.05
    r = y - x.astype(np.complex128)
    want = o_backproject(grid, oracle.Optics(), P, r, scale) + lam * vol.astype(np.complex128)
    vv = vol.astype(np.complex128)
    want_f = scale * 0.5 * np.vdot(r, r).real + 0.5 * lam * np.vdot(vv, vv).real
    xd = torch.from_numpy(x).cuda()
    for det in (True, False):
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        gr = b.gradient(b.Grid(M), b.Optics(), rot, df, v, xd, scale, lam, loss_out=loss, deterministic=det)
        close(gr.cpu().numpy(), want, 1e-4, "gradient (%s)" % ("deterministic" if det else "fast"))
        assert loss.item() == pytest.approx(want_f, rel=1e-5)
    # the gradient with the probe product in one kernel
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gr, _ = b.gradient_hutchinson(b.Grid(M), b.Optics(), rot, df, v, xd, scale, lam, 2, 23, probe0=40, loss_out=loss)
    close(gr.cpu().numpy(), want, 1e-4, "gradient (fused with the probe product)")
    assert loss.item() == pytest.approx(want_f, rel=1e-5)


def test_stress_batch_hutchinson(stress):
    b, grid, P, vol, rot, df, v = stress
    scale, lam, seed, p0 = 244.1, 0.05, 23, 40
    got = b.hutchinson_diag(b.Grid(M), b.Optics(), rot, df, 2, seed=seed, scale=scale, lam=lam, probe0=p0)
    want = np.zeros(M ** 3)
    for p in (p0, p0 + 1):
        z = oracle.rademacher(seed, p, M ** 3)
        hz = o_backproject(grid, oracle.Optics(), P, o_project(grid, oracle.Optics(), P, z.reshape(M, M, M)),
                           scale).reshape(-1) + lam * z
        want += z * hz.real / 2
    close(got.cpu().numpy(), want, 1e-4, "hutchinson probe pair")
    # the same pair's product from the kernel that also forms the gradient
    # (the diagonal depends on neither the volume nor the images)
    x0 = torch.zeros((N_IMG, M, M), dtype=torch.complex64, device="cuda")
    _, dg = b.gradient_hutchinson(b.Grid(M), b.Optics(), rot, df, v, x0, scale, lam, 2, seed, probe0=p0)
    close(dg.cpu().numpy(), want, 1e-4, "hutchinson probe pair (fused with the gradient)")
