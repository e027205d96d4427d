"""What the trained preconditioner network gains over the method without it,
and its judge and fallback (GPU).

A small network is trained, with the library's own kernels, on Hutchinson
diagonals (100 probes) of six noise-free data sets at 32^3 and 48^3.  It is
then applied to a 64^3 data set of a size it never saw:
  - its diagonal is much closer to the exact diagonal (one squared-weight
    pass) than a Hutchinson estimate from a few probes;
  - the judge (shell means of a short Hutchinson estimate) accepts it, and
    rejects a corrupted network, after which the learned arm runs as the
    Hutchinson arm;
  - Algorithm 1 with the learned diagonal reaches 1e-2 relative error of the
    high-frequency band in fewer iterations than plain SGD and no more than
    the Hutchinson arm.
"""
import math

import pytest
import torch

pytestmark = pytest.mark.gpu

SPECS = [(32, 3000, 20, (0.5 + 0.5 * i, 2.0 + 0.5 * i)) for i in range(3)] + \
        [(48, 6000, 40, (0.8 + 0.5 * i, 2.5 + 0.5 * i)) for i in range(3)]


@pytest.fixture(scope="module")
def mods():
    from paper_2311_16100_amd import binding, experiment, learned, tta
    binding.lib()
    return binding, experiment, learned, tta


@pytest.fixture(scope="module")
def trained(mods):
    _, _, _, tta = mods
    print("[learned] training on %d sets" % len(SPECS), flush=True)
    params, hist = tta.train_network(SPECS, steps=600, n_probe=100, log=None)
    return params, hist


@pytest.fixture(scope="module")
def ds64(mods):
    _, E, _, _ = mods
    return E.make_dataset(64, 12000, 50, 4242, float("inf"), defocus_um=(1.0, 3.0))


def corrupted(params):
    p = params.clone()
    p[-1] += 2.0  # output bias: every predicted data term times e^2
    return p


def test_training_fits(trained):
    _, hist = trained
    assert all(math.isfinite(l) for _, l in hist)
    assert hist[-1][1] < 0.1, hist


def test_learned_diag_beats_short_hutchinson(mods, trained, ds64):
    _, E, L, _ = mods
    params, _ = trained
    exact = E.exact_diagonal(ds64)
    learned = L.predict(ds64, params)
    short = L.hutchinson_full(ds64, 2, 5, n_images=4096)
    e_learned = L.diag_rel_error(learned, exact, ds64)
    e_short = L.diag_rel_error(short, exact, ds64)
    print("[learned] rel err vs exact diagonal: learned %.4f, 2-probe Hutchinson %.4f" % (e_learned, e_short))
    assert e_learned < 0.3
    assert e_learned < 0.5 * e_short


def test_judge_accepts_trained_and_rejects_corrupted(mods, trained, ds64):
    _, _, L, _ = mods
    params, _ = trained
    ok = L.judge(ds64, L.predict(ds64, params))
    bad = L.judge(ds64, L.predict(ds64, corrupted(params)))
    print("[learned] judge: trained %.4f corrupted %.4f" % (ok, bad))
    assert ok < 0.2
    assert bad > 0.2


def test_fallback_runs_as_hutchinson(mods, trained, ds64):
    _, E, _, _ = mods
    params, _ = trained
    r = E.compare_arms(ds64, 128, params=corrupted(params), arms=("learned",), stop_on="high", log=None,
                       max_epochs=4, eval_every=2)
    arm = r["arms"]["learned"]
    assert "fallback" in arm.note
    assert arm.reached


def test_learned_arm_gains_iterations(mods, trained, ds64):
    _, E, _, _ = mods
    params, _ = trained
    r = E.compare_arms(ds64, 128, params=params, arms=("plain", "hutchinson", "learned"), stop_on="high",
                       log=None, max_epochs=6, eval_every=1)
    it = {k: (a.reached, a.iterations, a.note) for k, a in r["arms"].items()}
    print("[learned] iterations to 1e-2 (high band):", it)
    assert "fallback" not in r["arms"]["learned"].note
    assert all(a.reached for a in r["arms"].values()), it
    assert r["arms"]["learned"].iterations < r["arms"]["plain"].iterations
    assert r["arms"]["learned"].iterations <= r["arms"]["hutchinson"].iterations


def test_judge_sees_a_wrong_direction_dependence(mods, trained, ds64):
    """A prediction with the right shell means but the wrong dependence on
    direction (the data term doubled on one side of kz = 0 and zeroed on the
    other) passes the shell comparison and is rejected by the shell x sector
    comparison."""
    _, _, L, _ = mods
    params, _ = trained
    good = L.predict(ds64, params)
    M = ds64.M
    kz = (torch.arange(M, device=good.device) - M // 2)[:, None, None].expand(M, M, M)
    # voxels whose largest |k_d| is along z, on the two sides of kz = 0:
    # the data term doubled on one side, zeroed on the other; shell sums of
    # the two sides are equal by the symmetry of the sets' diagonal
    idx = L.sector_index(M, good.device).reshape(M, M, M)
    along_z = ((idx % 6) // 2 == 2)
    f = torch.ones_like(good)
    f[along_z & (kz > 0)] = 2.0
    f[along_z & (kz < 0)] = 0.0
    warped = ds64.lam + (good - ds64.lam) * f
    e, e_shell, e_sector = L.judge(ds64, warped, detail=True)
    e_ok, _, _ = L.judge(ds64, good, detail=True)
    print("[learned] warped prediction: shell %.4f sector %.4f (correct one %.4f)" % (e_shell, e_sector, e_ok))
    assert e_ok < 0.2
    assert e_shell < 0.2 < e_sector and e == e_sector
