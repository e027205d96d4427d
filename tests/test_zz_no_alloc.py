"""The allocation-free gradient (csg_gradient_noalloc, static per-GPU scratch)
against the workspace form csg_gradient (fast mode) on the same inputs,
called through the C ABI: two calls in a row, the second with a smaller
input, and a batch whose brick tables exceed the static scratch (processed in
sub-batches).  Bound: relative L2 <= 1e-4 and per element <= 1e-4 of the
largest value (the two differ only in the order of the float atomic flushes),
the loss to 1e-7 relative."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def b():
    from paper_2311_16100_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    binding.lib()
    return binding


def _case(b, M, n, seed, interp=1, shifts=False):
    dev = torch.device("cuda:0")
    rot = torch.from_numpy(synth.uniform_rotations(n, seed)).to(dev)
    df = torch.from_numpy(synth.defocus_values(n, 1.0, 3.0, seed)).to(dev)
    vol = torch.from_numpy(synth.blob_volume(M, 20, seed)).to(dev)
    x = torch.from_numpy(synth.random_complex((n, M, M), seed, stream=11)).to(dev)
    sh = None
    if shifts:
        rng = np.random.default_rng(seed)
        sh = torch.from_numpy(rng.uniform(-3, 3, size=(n, 2)).astype(np.float32)).to(dev)
    return b.Grid(M, interp=interp), rot, df, vol, x, sh


def _reference(b, grid, rot, df, vol, x, sh, scale, lam):
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = b.gradient(grid, b.Optics(), rot, df, vol, x, scale, lam, loss_out=loss, shift=sh)
    return g, loss


def _compare(got, want, loss_got, loss_want, what):
    got = got.cpu().numpy().reshape(-1).astype(np.complex128)
    want = want.cpu().numpy().reshape(-1).astype(np.complex128)
    l2 = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    el = float(np.abs(got - want).max() / np.abs(want).max())
    lr = abs(loss_got.item() - loss_want.item()) / abs(loss_want.item())
    print("[no-alloc] %s: relative L2 %.2e, max element %.2e, loss %.2e" % (what, l2, el, lr), flush=True)
    assert l2 <= 1e-4 and el <= 1e-4 and lr <= 1e-7, (what, l2, el, lr)


def _noalloc(b, grid, rot, df, vol, x, sh, scale, lam):
    out = torch.empty_like(vol)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    return out, loss


def test_two_calls_second_smaller(b):
    scale, lam = 37.5, 0.02
    big = _case(b, 64, 700, 41, shifts=True)
    small = _case(b, 36, 37, 42)
    outs = []
    for grid, rot, df, vol, x, sh in (big, small):
        out, loss = _noalloc(b, grid, rot, df, vol, x, sh, scale, lam)
        print("[no-alloc] call M=%d n=%d" % (grid.M, rot.shape[0]), flush=True)
        b.gradient_noalloc(grid, b.Optics(), rot, df, vol, x, scale, lam, out, loss_out=loss, shift=sh)
        outs.append((out, loss))
    torch.cuda.synchronize()
    for (grid, rot, df, vol, x, sh), (out, loss) in zip((big, small), outs):
        want, wl = _reference(b, grid, rot, df, vol, x, sh, scale, lam)
        _compare(out, want, loss, wl, "M=%d n=%d" % (grid.M, rot.shape[0]))


def test_sub_batches_when_the_tables_exceed_the_scratch(b):
    """256^3 with 1600 images: the brick tables of one launch would need more
    than the 64 MiB of static scratch, so the call runs two launches; then a
    smaller call on the same scratch."""
    scale, lam = 125.0, 0.01
    grid, rot, df, vol, x, sh = _case(b, 256, 1600, 43)
    need = b.workspace_bytes(grid, 1600, b.CSG_WS_GRADIENT)
    assert need > 64 * 2 ** 20, need
    out, loss = _noalloc(b, grid, rot, df, vol, x, sh, scale, lam)
    print("[no-alloc] call M=256 n=1600 (sub-batched)", flush=True)
    b.gradient_noalloc(grid, b.Optics(), rot, df, vol, x, scale, lam, out, loss_out=loss)
    g2 = _case(b, 40, 90, 44)
    out2, loss2 = _noalloc(b, *g2, scale, lam)
    print("[no-alloc] call M=40 n=90", flush=True)
    b.gradient_noalloc(g2[0], b.Optics(), *g2[1:5], scale, lam, out2, loss_out=loss2)
    torch.cuda.synchronize()
    want, wl = _reference(b, grid, rot, df, vol, x, sh, scale, lam)
    _compare(out, want, loss, wl, "M=256 n=1600")
    want2, wl2 = _reference(b, *g2, scale, lam)
    _compare(out2, want2, loss2, wl2, "M=40 n=90")


def test_nearest_neighbour_and_empty_batch(b):
    scale, lam = 3.0, 0.5
    grid, rot, df, vol, x, sh = _case(b, 32, 50, 45, interp=0)
    out, loss = _noalloc(b, grid, rot, df, vol, x, sh, scale, lam)
    print("[no-alloc] call M=32 n=50 nearest neighbour", flush=True)
    b.gradient_noalloc(grid, b.Optics(), rot, df, vol, x, scale, lam, out, loss_out=loss)
    want, wl = _reference(b, grid, rot, df, vol, x, sh, scale, lam)
    _compare(out, want, loss, wl, "nearest neighbour M=32 n=50")
    # no images: grad = lam v, loss = lam/2 |v|^2
    e = _case(b, 16, 1, 46)
    out0, loss0 = _noalloc(b, *e, scale, lam)
    b.gradient_noalloc(e[0], b.Optics(), e[1][:0], e[2][:0], e[3], e[4][:0], scale, lam, out0, loss_out=loss0)
    torch.cuda.synchronize()
    v = e[3].cpu().numpy().astype(np.complex128)
    np.testing.assert_allclose(out0.cpu().numpy(), lam * v, rtol=1e-6, atol=0)
    assert loss0.item() == pytest.approx(0.5 * lam * np.vdot(v, v).real, rel=1e-6)


def test_repeated_calls_leave_device_memory_unchanged(b):
    grid, rot, df, vol, x, sh = _case(b, 48, 300, 47)
    out, loss = _noalloc(b, grid, rot, df, vol, x, sh, 10.0, 0.1)
    b.gradient_noalloc(grid, b.Optics(), rot, df, vol, x, 10.0, 0.1, out, loss_out=loss)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(5):
        b.gradient_noalloc(grid, b.Optics(), rot, df, vol, x, 10.0, 0.1, out, loss_out=loss)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
