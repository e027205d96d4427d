"""Pins of the oracle's preconditioner network: bfloat16 rounding against the
format's definition, GELU against closed forms, the forward pass against a
hand-evaluated tiny case, and the gradient against central finite
differences (with the bfloat16 roundings switched off by choosing values that
are exactly representable)."""
import math

import numpy as np
import pytest


def test_bf16_rounding(orc):
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.0e38, 1e-40], dtype=np.float32)
    r = orc.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie -> even (1.0)
    assert r[2] == 1.0 + 2 ** -7            # exactly representable
    assert r[3] == 1.0 + 2 ** -6            # tie -> even (upper)
    assert r[4] == -2.5
    # 8 significant bits: relative error at most 2^-8 for normal numbers,
    # and the result is always a bfloat16 (low 16 bits zero)
    x = np.random.default_rng(1).standard_normal(10000).astype(np.float32)
    r = orc.bf16_round(x)
    assert np.max(np.abs(r - x) / np.abs(x)) <= 2 ** -8
    assert np.all(r.astype(np.float32).view(np.uint32) & 0xFFFF == 0)
    # and it is the nearer of the two neighbouring bfloat16 values
    lo = (x.view(np.uint32) & 0xFFFF0000).view(np.float32).astype(np.float64)
    hi = ((x.view(np.uint32) & 0xFFFF0000) + 0x10000).view(np.float32).astype(np.float64)
    best = np.where(np.abs(lo - x) <= np.abs(hi - x), lo, hi)
    assert np.all(np.abs(r - x) <= np.abs(best - x))


def test_gelu_closed_forms(orc):
    assert orc.gelu(np.array([0.0]))[0] == 0.0
    x = np.array([-3.0, -1.0, 0.5, 2.0])
    phi = 0.5 * (1 + np.array([math.erf(v / math.sqrt(2)) for v in x]))
    assert np.allclose(orc.gelu(x), x * phi, rtol=1e-15)
    # derivative by central differences
    h = 1e-6
    assert np.allclose(orc.gelu_grad(x), (orc.gelu(x + h) - orc.gelu(x - h)) / (2 * h), atol=1e-8)
    # large |x|: GELU -> relu
    assert orc.gelu(np.array([10.0]))[0] == pytest.approx(10.0)
    assert abs(orc.gelu(np.array([-10.0]))[0]) < 1e-20


def _params(seed, scale=0.25):
    g = np.random.default_rng(seed)
    p = (g.standard_normal(64 * 3 + 64 + 64 * 64 + 64 + 64 + 1) * scale).astype(np.float32)
    return p


def test_forward_tiny_case_by_hand(orc):
    # one hidden unit active in each layer, everything exactly representable
    p = np.zeros(orc.MLP_NPARAM, np.float32)
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(p)
    W1[0] = [1.0, 0.5, -0.25]
    b1[0] = 0.5
    W2[3, 0] = 2.0
    b2[3] = -0.5
    W3[3] = 1.5
    b3[0] = 0.25
    x = np.array([[1.0, 2.0, 4.0]], np.float32)
    z1 = 1.0 + 1.0 - 1.0 + 0.5
    h1 = z1 * 0.5 * (1 + math.erf(z1 / math.sqrt(2)))
    h1 = orc.bf16_round(np.array([h1], np.float32))[0]
    z2 = 2.0 * h1 - 0.5
    h2 = z2 * 0.5 * (1 + math.erf(z2 / math.sqrt(2)))
    h2 = orc.bf16_round(np.array([h2], np.float32))[0]
    want = 1.5 * h2 + 0.25
    # GELU(0) = 0 for all other hidden units
    assert orc.mlp_forward(p, x)[0] == pytest.approx(want, rel=1e-14)


def test_gradient_central_differences(orc, monkeypatch):
    # with the bfloat16 rounding replaced by the identity the network is
    # smooth, and the analytic gradient must match central differences
    monkeypatch.setattr(orc, "bf16_round", lambda a: np.asarray(a, dtype=np.float64))
    p = _params(3).astype(np.float64)
    X = np.random.default_rng(4).standard_normal((40, 3))
    t = np.random.default_rng(5).standard_normal(40)

    def L_of(q):
        y = orc.mlp_forward(q, X)
        return float(np.mean((y - t) ** 2))

    # evaluate with float64 parameters: patch the unpack dtype through a copy
    monkeypatch.setattr(orc, "mlp_unpack", _unpack64(orc))
    L, g = orc.mlp_loss_grad(p, X, t)
    rng = np.random.default_rng(6)
    h = 1e-6
    for k in rng.choice(len(p), 40, replace=False):
        q1 = p.copy(); q1[k] += h
        q2 = p.copy(); q2[k] -= h
        fd = (L_of(q1) - L_of(q2)) / (2 * h)
        assert fd == pytest.approx(g[k], abs=1e-7 + 1e-5 * abs(fd))
    assert L == pytest.approx(L_of(p))


def _unpack64(orc):
    def unpack(params):
        p = np.asarray(params, dtype=np.float64)
        H = orc.MLP_H
        o = 0
        W1 = p[o:o + 3 * H].reshape(H, 3); o += 3 * H
        b1 = p[o:o + H]; o += H
        W2 = p[o:o + H * H].reshape(H, H); o += H * H
        b2 = p[o:o + H]; o += H
        W3 = p[o:o + H]; o += H
        b3 = p[o:o + 1]
        return W1, b1, W2, b2, W3, b3
    return unpack
