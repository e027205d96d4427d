"""GPU parity of the preconditioner network's kernels (bfloat16 matrix-core
GEMMs, float32 accumulation) against the oracle network (bfloat16-rounded
weights and layer inputs, double accumulation).  Where a value sits near a
bfloat16 rounding boundary the two sides may round it differently, so the
tolerances are relative L2 <= 1e-2 for outputs and gradients."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2311_16100_amd import binding
    binding.lib()
    return binding


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def params(seed, scale=0.3):
    g = np.random.default_rng(seed)
    p = (g.standard_normal(oracle.MLP_NPARAM) * scale).astype(np.float32)
    return p


def test_param_count(B):
    assert B.mlp_param_count() == oracle.MLP_NPARAM


@pytest.mark.parametrize("n", [1, 31, 32, 33, 1000, 4099])
def test_forward_parity(B, n):
    p = params(1)
    X = (np.random.default_rng(2).standard_normal((n, 3)) * 1.5).astype(np.float32)
    y = B.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    want = oracle.mlp_forward(p, X)
    assert rel(y, want) <= 1e-2
    # and most samples agree to float rounding
    assert np.median(np.abs(y - want) / (np.abs(want) + 1e-3)) < 1e-3


@pytest.mark.parametrize("n", [37, 2048, 5000])
def test_gradient_parity(B, n):
    p = params(3)
    X = (np.random.default_rng(4).standard_normal((n, 3))).astype(np.float32)
    T = (np.random.default_rng(5).standard_normal(n)).astype(np.float32)
    g, L = B.mlp_grad(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    wantL, wantg = oracle.mlp_loss_grad(p, X, T)
    assert L.item() == pytest.approx(wantL, rel=1e-2)
    assert rel(g.cpu().numpy(), wantg) <= 2e-2


def test_adam_step(B):
    n = oracle.MLP_NPARAM
    rng = np.random.default_rng(7)
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    pd, gd, md, vd = (torch.from_numpy(a).cuda() for a in (p, g, m, v))
    B.mlp_adam(pd, md, vd, gd, 1, 1e-2)
    # first Adam step: m_hat = g, v_hat = g^2, update = lr g / (|g| + eps)
    want = p - 1e-2 * g / (np.abs(g) + 1e-8)
    assert np.allclose(pd.cpu().numpy(), want, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss(B):
    # regression of a smooth function of the inputs
    rng = np.random.default_rng(8)
    n = 8192
    X = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    T = (np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2]).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    p = torch.from_numpy(params(9, 0.2)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    L0 = None
    for step in range(1, 301):
        g, L = B.mlp_grad(p, Xd, Td)
        if L0 is None:
            L0 = L.item()
        B.mlp_adam(p, m, v, g, step, 3e-3)
    _, L1 = B.mlp_grad(p, Xd, Td)
    assert L1.item() < 0.1 * L0
    assert L1.item() == pytest.approx(oracle.mlp_loss_grad(p.cpu().numpy(), X, T)[0], rel=2e-2)


def test_learned_diag_fused(B):
    M, N, lam = 16, 50, 0.3
    rng = np.random.default_rng(10)
    ctf2 = rng.uniform(0.0, 5.0, (M, M, M)).astype(np.float32)
    cover = rng.integers(0, 30, (M, M, M)).astype(np.float32)
    p = params(11, 0.1)
    D = B.learned_diag(B.Grid(M), N, lam, torch.from_numpy(p).cuda(), torch.from_numpy(ctf2).cuda(),
                       torch.from_numpy(cover).cuda()).cpu().numpy()
    ax = np.arange(M) - M // 2
    k = np.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2) / (M // 2)
    X = np.stack([k.ravel(), np.log(np.maximum(ctf2.ravel() * M / N, 1e-30)),
                  np.log(np.maximum(cover.ravel() * M / N, 1e-30))], axis=1).astype(np.float32)
    y = oracle.mlp_forward(p, X)
    want = np.where(cover.ravel() > 0, lam + N / M * np.exp(y), lam)
    assert rel(D.ravel(), want) <= 1e-2
    assert np.all(D.ravel()[cover.ravel() == 0] == np.float32(lam))


def test_learned_diag_skips_unreached_tiles(B):
    """Voxels no image reaches (here: outside a ball, whole tiles of 32) get
    lambda without the network; the rest still matches the oracle network."""
    M, N, lam = 64, 400, 0.7
    rng = np.random.default_rng(12)
    ax = np.arange(M) - M // 2
    r = np.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2)
    ctf2 = rng.uniform(0.5, 5.0, (M, M, M)).astype(np.float32)
    cover = np.where(r <= 20, rng.integers(1, 30, (M, M, M)), 0).astype(np.float32)
    p = params(13, 0.1)
    D = B.learned_diag(B.Grid(M), N, lam, torch.from_numpy(p).cuda(), torch.from_numpy(ctf2).cuda(),
                       torch.from_numpy(cover).cuda()).cpu().numpy().ravel()
    X = np.stack([(r / (M // 2)).ravel(), np.log(np.maximum(ctf2.ravel() * M / N, 1e-30)),
                  np.log(np.maximum(cover.ravel() * M / N, 1e-30))], axis=1).astype(np.float32)
    inside = cover.ravel() > 0
    want = lam + N / M * np.exp(oracle.mlp_forward(p, X[inside]))
    assert rel(D[inside], want) <= 1e-2
    assert np.all(D[~inside] == np.float32(lam))


def test_gradient_is_bitwise_reproducible(B):
    """Fixed-order sums: equal inputs give equal bits (many blocks)."""
    n = 20000
    p = torch.from_numpy(params(14)).cuda()
    X = torch.from_numpy(np.random.default_rng(15).standard_normal((n, 3)).astype(np.float32)).cuda()
    T = torch.from_numpy(np.random.default_rng(16).standard_normal(n).astype(np.float32)).cuda()
    g1, L1 = B.mlp_grad(p, X, T)
    g1, L1 = g1.clone(), L1.clone()
    for _ in range(3):
        g2, L2 = B.mlp_grad(p, X, T)
        assert torch.equal(g1, g2) and torch.equal(L1, L2)


def test_training_is_reproducible(B):
    """Two trainings from the same seed give bitwise equal parameters."""
    from paper_2311_16100_amd import learned as L
    rng = np.random.default_rng(17)
    X = torch.from_numpy(rng.uniform(-1, 1, (6000, 3)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.standard_normal(6000).astype(np.float32)).cuda()
    sets = [L.TrainingSet(X, T)]
    p1, h1 = L.train(sets, steps=60, batch=2048, seed=3)
    p2, h2 = L.train(sets, steps=60, batch=2048, seed=3)
    assert torch.equal(p1, p2) and h1 == h2
