"""Streamed data sets (images regenerated per batch instead of resident) and
the deterministic adjoint inside Algorithm 1 (GPU)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_2311_16100_amd import binding, experiment
    binding.lib()
    return experiment


def test_streamed_images_equal_resident(E):
    res = E.make_dataset(32, 600, 20, 11, float("inf"), poses="vmf")
    st = E.make_dataset(32, 600, 20, 11, float("inf"), poses="vmf", stream=True)
    assert st.streamed and not res.streamed
    idx = torch.arange(0, 600, 7, device=res.device)
    assert torch.equal(st.images(idx), res.images(idx))
    assert st.lam == res.lam


def test_streamed_noise_is_a_function_of_the_image_index(E):
    """A noisy streamed set: an image carries the same noise in any batch
    and position; the noise has the set's variance on the disk (real and
    imaginary parts each half of it), none outside, no mean, and is
    uncorrelated between images; a few pixels against the generator's
    definition (Philox4x32-10 from the oracle's copy, then Box-Muller)."""
    import math

    import numpy as np

    import oracle
    import synth
    from synth import gpu_noise
    ds = E.make_dataset(48, 4000, 20, 15, 0.05, stream=True)
    assert ds.streamed and ds.sigma2 > 0
    clean = E.make_dataset(48, 4000, 20, 15, float("inf"), stream=True)
    a = torch.tensor([5, 3999, 17, 2048], device=ds.device)
    b = torch.tensor([17, 1, 5, 2, 3999, 6], device=ds.device)
    xa, xb = ds.images(a), ds.images(b)
    assert torch.equal(xa[0], xb[2]) and torch.equal(xa[2], xb[0]) and torch.equal(xa[1], xb[4])
    assert torch.equal(ds.images(slice(2040, 2050))[8], xa[3])
    idx = torch.arange(0, 4000, 3, device=ds.device)
    nz = (ds.images(idx) - clean.images(idx)).cpu().numpy()
    ax = np.arange(48) - 24
    disk = (ax[:, None] ** 2 + ax[None, :] ** 2) <= math.floor(ds.grid.rmax ** 2)
    assert np.all(nz[:, ~disk] == 0)
    v = nz[:, disk]
    n = v.size
    assert abs(np.mean(np.abs(v) ** 2) / ds.sigma2 - 1) < 6 / math.sqrt(n)
    assert abs(np.mean(v.real ** 2) / (ds.sigma2 / 2) - 1) < 8 / math.sqrt(n)
    assert abs(np.mean(v)) / math.sqrt(ds.sigma2) < 6 / math.sqrt(n)
    c = np.vdot(v[0], v[1]) / np.sqrt(np.vdot(v[0], v[0]).real * np.vdot(v[1], v[1]).real)
    assert abs(c) < 6 / math.sqrt(v.shape[1])
    key = gpu_noise.noise_seed(ds.seed, synth.STREAM_NOISE)
    sd = math.sqrt(ds.sigma2 / 2)
    for i_row, img in ((0, 0), (5, 15), (100, 300)):
        for p in (24 * 48 + 24, 10 * 48 + 30, 40 * 48 + 20):
            r = oracle.philox4x32_10([p, img, 0, gpu_noise.TAG], [key & 0xFFFFFFFF, key >> 32])
            u1 = ((int(r[0]) >> 8) + 1) * 2.0 ** -24
            u2 = (int(r[1]) >> 8) * 2.0 ** -24
            rad = sd * math.sqrt(-2 * math.log(u1))
            want = complex(rad * math.cos(2 * math.pi * u2), rad * math.sin(2 * math.pi * u2))
            got = complex(nz[i_row].reshape(-1)[p])
            assert abs(got - want) <= 1e-4 * sd + 1e-5 * abs(want), (img, p, got, want)


def test_streamed_run_matches_resident_run(E):
    res = E.make_dataset(32, 1000, 20, 12, float("inf"))
    st = E.make_dataset(32, 1000, 20, 12, float("inf"), stream=True)
    v_star, _, _ = E.ground_truth(res)
    a = E.run_arm(res, v_star, "hutchinson", 32, max_epochs=2, eval_every=5)
    b = E.run_arm(st, v_star, "hutchinson", 32, max_epochs=2, eval_every=5)
    assert a.iterations == b.iterations
    assert b.gen_seconds > 0.0 and a.gen_seconds == 0.0
    ea = [e[2] for e in a.errors]
    eb = [e[2] for e in b.errors]
    assert max(abs(x - y) / max(y, 1e-12) for x, y in zip(ea, eb)) < 1e-3


def test_deterministic_arm_is_reproducible(E):
    ds = E.make_dataset(32, 512, 20, 13, float("inf"), poses="vmf")
    v_star, _, _ = E.ground_truth(ds)
    a = E.run_arm(ds, v_star, "plain", 32, max_epochs=1, eval_every=4, deterministic=True)
    b = E.run_arm(ds, v_star, "plain", 32, max_epochs=1, eval_every=4, deterministic=True)
    # the gradient is bitwise reproducible; the step statistics and the
    # Armijo losses are double-precision sums whose order may vary
    ea, eb = [e[2] for e in a.errors], [e[2] for e in b.errors]
    assert len(ea) == len(eb) and max(abs(x - y) / y for x, y in zip(ea, eb)) < 1e-5


def test_queued_probes_leave_the_run_unchanged(E):
    """The look-ahead over batches (across the epoch boundary too: 31 batches
    of 32 per epoch) feeds the same poses and images as the plain loop."""
    ds = E.make_dataset(32, 1000, 20, 14, float("inf"))
    v_star, _, _ = E.ground_truth(ds)
    a = E.run_arm(ds, v_star, "hutchinson", 32, max_epochs=2, eval_every=5, target=1e-9, fused=False)
    b = E.run_arm(ds, v_star, "hutchinson", 32, max_epochs=2, eval_every=5, target=1e-9, queue_probes=False,
                  fused=False)
    # and the one-kernel gradient and probe product (no queue) on the same run
    c = E.run_arm(ds, v_star, "hutchinson", 32, max_epochs=2, eval_every=5, target=1e-9)
    assert a.iterations == b.iterations == 62
    # float atomics differ between the runs; a batch whose images and poses
    # did not belong together would move the errors far beyond this
    ea, eb, ec = [e[2] for e in a.errors], [e[2] for e in b.errors], [e[2] for e in c.errors]
    assert len(ea) == len(eb) and max(abs(x - y) / y for x, y in zip(ea, eb)) < 1e-3
    assert c.iterations == 62 and len(ec) == len(ea) and max(abs(x - y) / y for x, y in zip(ea, ec)) < 1e-3


def test_checkpoint_resume_is_bit_exact(E, tmp_path):
    """A run stopped mid-epoch and resumed from its checkpoint ends where the
    uninterrupted run ends, bit for bit, on the deterministic path (fixed
    diagonal, fixed-point gradient); across an epoch boundary with the step
    halving and iterate averaging too."""
    ds = E.make_dataset(24, 320, 12, 15, float("inf"))
    v_star, _, _ = E.ground_truth(ds)
    D = E.exact_diagonal(ds)
    kw = dict(D_fixed=D, max_epochs=3, eval_every=3, deterministic=True, target=1e-9, seed=3)
    for stop, extra in ((13, {}), (20, dict(decay_epochs=1, average_from_epoch=1))):
        full = E.run_arm(ds, v_star, "exact", 32, **kw, **extra)
        ck = str(tmp_path / ("ck%d.npz" % stop))
        part = E.run_arm(ds, v_star, "exact", 32, **kw, **extra, checkpoint=ck, stop_at=stop)
        assert part.note == "stopped" and part.iterations == stop
        rest = E.run_arm(ds, v_star, "exact", 32, **kw, **extra, resume=ck)
        assert rest.iterations == full.iterations == 30
        assert [e[:1] + e[2:] for e in rest.errors] == [e[:1] + e[2:] for e in full.errors]
        assert rest.halvings == full.halvings


def test_checkpoint_resume_hutchinson(E, tmp_path):
    """The Hutchinson arm resumed from a checkpoint (D and D_avg restored, the
    probes numbered by iteration) follows the uninterrupted run; its probe
    products sum with float atomics, so the match is to rounding."""
    ds = E.make_dataset(24, 320, 12, 16, float("inf"))
    v_star, _, _ = E.ground_truth(ds)
    kw = dict(max_epochs=2, eval_every=2, target=1e-9, seed=4)
    full = E.run_arm(ds, v_star, "hutchinson", 32, **kw)
    ck = str(tmp_path / "ckh.npz")
    E.run_arm(ds, v_star, "hutchinson", 32, **kw, checkpoint=ck, stop_at=7)
    rest = E.run_arm(ds, v_star, "hutchinson", 32, **kw, resume=ck)
    assert rest.iterations == full.iterations == 20
    ea, eb = [e[2] for e in rest.errors], [e[2] for e in full.errors]
    assert len(ea) == len(eb) and max(abs(x - y) / y for x, y in zip(ea, eb)) < 1e-4
