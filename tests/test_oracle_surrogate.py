"""Pins of the surrogate oracle (oracle/surrogate.py) against brute force, closed forms and finite differences."""

import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S

TINY = dict(channels=(1, 2, 3, 2, 2), hidden=4, n_feat=1, n_out=3)


def loop_conv(a, W, b):
    """Brute-force stride-2 periodic 3x3x3 convolution, pure Python loops."""
    B, n, _, _, ci_n = a.shape
    m = n // 2
    co_n = W.shape[0]
    out = np.zeros((B, m, m, m, co_n))
    for bb in range(B):
        for oz in range(m):
            for oy in range(m):
                for ox in range(m):
                    for co in range(co_n):
                        s = b[co]
                        k = 0
                        for tz in range(3):
                            for ty in range(3):
                                for tx in range(3):
                                    iz, iy, ix = (2 * oz + tz - 1) % n, (2 * oy + ty - 1) % n, (2 * ox + tx - 1) % n
                                    for ci in range(ci_n):
                                        s += W[co, k, ci] * a[bb, iz, iy, ix, ci]
                                    k += 1
                        out[bb, oz, oy, ox, co] = s
    return out


def test_gelu_values():
    x = torch.tensor([0.0, 1.0, -1.0, 2.0, 40.0, -40.0], dtype=torch.float64)
    g = S.gelu(x).numpy()
    phi1 = 0.5 * (1.0 + math.erf(1.0 / math.sqrt(2.0)))
    assert g[0] == 0.0
    assert abs(g[1] - phi1) < 1e-16 and abs(g[1] - 0.8413447460685429) < 1e-15
    assert abs(g[2] + (1.0 - phi1)) < 1e-16
    assert abs(g[4] - 40.0) < 1e-12 and abs(g[5]) < 1e-12
    # x Phi(x) - (-x) Phi(-x) = x
    assert abs((g[3] - S.gelu(torch.tensor(-2.0, dtype=torch.float64)).item()) - 2.0) < 1e-15


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((2, 4, 4, 4, 2))
    W = rng.standard_normal((3, 27, 2))
    b = rng.standard_normal(3)
    out = S.conv_s2(torch.as_tensor(a), torch.as_tensor(W), torch.as_tensor(b)).numpy()
    assert np.abs(out - loop_conv(a, W, b)).max() < 1e-13


def test_conv_of_constant_field_and_shift_equivariance():
    rng = np.random.default_rng(1)
    W = rng.standard_normal((4, 27, 3))
    b = rng.standard_normal(4)
    a = np.full((1, 6, 6, 6, 3), 0.7)
    out = S.conv_s2(torch.as_tensor(a), torch.as_tensor(W), torch.as_tensor(b)).numpy()
    assert np.abs(out - (b + 0.7 * W.sum(axis=(1, 2)))).max() < 1e-13
    a = rng.standard_normal((1, 8, 8, 8, 3))
    shifted = np.roll(a, shift=(2, -2, 4), axis=(1, 2, 3))
    o1 = S.conv_s2(torch.as_tensor(a), torch.as_tensor(W), torch.as_tensor(b)).numpy()
    o2 = S.conv_s2(torch.as_tensor(shifted), torch.as_tensor(W), torch.as_tensor(b)).numpy()
    assert np.abs(np.roll(o1, shift=(1, -1, 2), axis=(1, 2, 3)) - o2).max() < 1e-13


def test_forward_matches_composition_of_brute_force_layers():
    rng = np.random.default_rng(2)
    theta = 0.3 * rng.standard_normal(S.n_params(**TINY))
    phase = (rng.random((2, 16, 16, 16)) < 0.3).astype(np.uint8)
    feat = rng.standard_normal((2, 1))
    y = S.predict(theta, phase, feat, **TINY)
    P = {k: v.numpy() for k, v in S.unflatten(torch.as_tensor(theta), **TINY).items()}
    gel = lambda x: 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))  # noqa: E731
    a = phase[..., None].astype(np.float64)
    for l in range(1, 5):
        a = gel(loop_conv(a, P["W%d" % l], P["b%d" % l]))
    g = a.reshape(2, -1, a.shape[-1]).mean(axis=1)
    h = gel(np.concatenate([g, feat], axis=1) @ P["W5"].T + P["b5"])
    ref = h @ P["W6"].T + P["b6"]
    assert np.abs(y - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = 0.3 * rng.standard_normal(S.n_params(**TINY))
    phase = (rng.random((3, 16, 16, 16)) < 0.4).astype(np.uint8)
    feat = rng.standard_normal((3, 1))
    target = rng.standard_normal((3, 3))
    L, g = S.loss_and_grad(theta, phase, feat, target, **TINY)
    # one coordinate in every parameter block
    sizes = [int(np.prod(s)) for _, s in S.param_shapes(**TINY)]
    starts = np.cumsum([0] + sizes[:-1])
    for st, sz in zip(starts, sizes):
        k = int(st + rng.integers(0, sz))
        hstep = 1e-5
        tp, tm = theta.copy(), theta.copy()
        tp[k] += hstep
        tm[k] -= hstep
        Lp, _ = S.loss_and_grad(tp, phase, feat, target, **TINY)
        Lm, _ = S.loss_and_grad(tm, phase, feat, target, **TINY)
        fd = (Lp - Lm) / (2 * hstep)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = S.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 0.01)
    assert np.abs(th + 0.01 * np.sign(g)).max() < 1e-7
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_stiffness_vector_round_trip():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((5, 6, 6))
    C = A + np.swapaxes(A, -1, -2)
    v = S.stiffness_to_vector(C)
    assert v.shape == (5, 21)
    assert np.array_equal(S.vector_to_stiffness(v), C)
    assert v[0, 0] == C[0, 0, 0] and v[0, 1] == C[0, 0, 1] and v[0, 6] == C[0, 1, 1] and v[0, 20] == C[0, 5, 5]


def test_parameter_count_of_the_full_network():
    # 4 conv blocks 1-32-64-128-256, MLP 257-256-21
    expect = (32 * 27 + 32) + (64 * 27 * 32 + 64) + (128 * 27 * 64 + 128) + (256 * 27 * 128 + 256) \
        + (256 * 257 + 256) + (21 * 256 + 21)
    assert S.n_params() == expect == 1234005
