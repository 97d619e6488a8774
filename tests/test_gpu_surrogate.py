"""Parity of the surrogate's HIP kernels (bf16 MFMA GEMMs, forward, backward, Adam, indicator).

Reference: the CPU oracle (oracle/surrogate.py, float64) evaluated with the same
parameters rounded to bf16, the precision the matrix cores consume.  The GPU
additionally rounds every activation and back-propagated gradient to bf16 before
each product (unit roundoff 2^-9 ~ 2e-3, accumulated over the 6 layers), so
outputs are compared to 2e-2 of their largest magnitude and gradients per
parameter block to 5e-2 in relative 2-norm; the GEMM alone (exact bf16
products, fp32 sums) to 5e-5 of the sum of the magnitudes of its terms.
"""

import numpy as np
import pytest
import torch

from oracle import closed_forms
from oracle import surrogate as OS

pytestmark = pytest.mark.gpu

SMALL = dict(n=16, channels=(1, 4, 8, 8, 16), hidden=16, n_feat=1, n_out=21)


def bf16_round(x):
    """Round float64 values to bf16 (nearest even), returned as float64."""
    return torch.as_tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def make(max_batch=8, **kw):
    from paper_2408_03804_amd.surrogate import CNN
    cfg = dict(SMALL)
    cfg.update(kw)
    return CNN(max_batch=max_batch, **cfg), cfg


def random_theta(cfg, seed, scale=0.25):
    rng = np.random.default_rng(seed)
    kw = dict(channels=cfg["channels"], hidden=cfg["hidden"], n_feat=cfg["n_feat"], n_out=cfg["n_out"])
    shapes = OS.param_shapes(**kw)
    parts = []
    for name, shape in shapes:
        fan = int(np.prod(shape[1:])) if name.startswith("W") else 1
        parts.append(rng.uniform(-1, 1, int(np.prod(shape))) * (scale if fan == 1 else np.sqrt(3.0 / fan)))
    return np.concatenate(parts).astype(np.float32), kw


def rounded_weights(theta, kw):
    """The oracle's view of theta: weights at bf16, biases kept at fp32 (the GPU adds them in fp32)."""
    th = theta.astype(np.float64).copy()
    off = 0
    for name, shape in OS.param_shapes(**kw):
        m = int(np.prod(shape))
        if name.startswith("W"):
            th[off:off + m] = bf16_round(th[off:off + m])
        off += m
    return th


@pytest.mark.parametrize("M,N,K,ak,bk,splits", [(70, 45, 50, True, True, 1), (64, 64, 64, True, False, 1),
                                                (33, 130, 96, False, True, 1), (100, 20, 1000, False, False, 7),
                                                (5, 3, 2000, False, False, 16), (300, 21, 27, True, True, 1)])
def test_gemm_matches_numpy(M, N, K, ak, bk, splits):
    h, _ = make()
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((N, K)).astype(np.float32)
    Ad = torch.as_tensor(A if ak else A.T.copy()).to(torch.bfloat16).cuda()
    Bd = torch.as_tensor(B if bk else B.T.copy()).to(torch.bfloat16).cuda()
    sam, sak = (K, 1) if ak else (1, M)
    sbn, sbk = (K, 1) if bk else (1, N)
    C = h.debug_gemm(M, N, K, Ad, sam, sak, Bd, sbn, sbk, splits).sum(dim=0).cpu().numpy().astype(np.float64)
    Ar, Br = bf16_round(A), bf16_round(B)
    ref = Ar @ Br.T
    mag = np.abs(Ar) @ np.abs(Br).T
    assert np.all(np.abs(C - ref) <= 5e-5 * mag + 1e-30)


def test_forward_matches_oracle_small():
    h, cfg = make()
    theta, kw = random_theta(cfg, 1)
    h.set_params(theta)
    rng = np.random.default_rng(2)
    B = 3
    phase = (rng.random((B, 16, 16, 16)) < 0.35).astype(np.uint8)
    feat = rng.standard_normal((B, 1)).astype(np.float32)
    y = h.forward(phase, feat).cpu().numpy()
    ref = OS.predict(rounded_weights(theta, kw), phase, bf16_round(feat), **kw)
    assert np.abs(y - ref).max() < 2e-2 * np.abs(ref).max()
    scale = np.array([2.0, 0.5, 3.0], np.float32)
    ys = h.forward(phase, feat, scale).cpu().numpy()
    assert np.allclose(ys, y * scale[:, None], rtol=1e-6, atol=0)
    offset = rng.standard_normal(y.shape).astype(np.float32)
    yo = h.forward(phase, feat, scale, offset).cpu().numpy()
    assert np.allclose(yo, offset + y * scale[:, None], rtol=1e-6, atol=1e-6)


def test_gradient_matches_oracle_small():
    h, cfg = make()
    theta, kw = random_theta(cfg, 3)
    h.set_params(theta)
    rng = np.random.default_rng(4)
    B = 4
    phase = (rng.random((B, 16, 16, 16)) < 0.4).astype(np.uint8)
    feat = rng.standard_normal((B, 1)).astype(np.float32)
    target = rng.standard_normal((B, 21)).astype(np.float32)
    loss, g = h.loss_grad(phase, feat, target)
    Lr, gr = OS.loss_and_grad(rounded_weights(theta, kw), phase, bf16_round(feat), target, **kw)
    assert abs(loss - Lr) < 2e-2 * abs(Lr)
    g = g.cpu().numpy()
    off = 0
    for name, shape in OS.param_shapes(**kw):
        m = int(np.prod(shape))
        a, b = g[off:off + m], gr[off:off + m]
        assert np.linalg.norm(a - b) < 5e-2 * np.linalg.norm(b) + 1e-12, name
        off += m


def test_full_network_forward_and_gradient_match_oracle():
    from paper_2408_03804_amd.surrogate import CNN
    kw = dict(channels=OS.CHANNELS, hidden=256, n_feat=1, n_out=21)
    h = CNN(n=32, max_batch=2, **kw)
    theta, _ = random_theta(dict(n=32, **kw), 5)
    h.set_params(theta)
    rng = np.random.default_rng(6)
    phase = (rng.random((2, 32, 32, 32)) < 0.3).astype(np.uint8)
    feat = rng.standard_normal((2, 1)).astype(np.float32)
    target = rng.standard_normal((2, 21)).astype(np.float32)
    th_r = rounded_weights(theta, kw)
    y = h.forward(phase, feat).cpu().numpy()
    ref = OS.predict(th_r, phase, bf16_round(feat), **kw)
    assert np.abs(y - ref).max() < 2e-2 * np.abs(ref).max()
    loss, g = h.loss_grad(phase, feat, target)
    Lr, gr = OS.loss_and_grad(th_r, phase, bf16_round(feat), target, **kw)
    assert abs(loss - Lr) < 2e-2 * abs(Lr)
    g = g.cpu().numpy()
    assert np.linalg.norm(g - gr) < 5e-2 * np.linalg.norm(gr)


def test_adam_step_matches_oracle_and_training_reduces_loss():
    h, cfg = make(max_batch=16)
    theta, kw = random_theta(cfg, 7)
    h.set_params(theta)
    rng = np.random.default_rng(8)
    phase = (rng.random((16, 16, 16, 16)) < 0.4).astype(np.uint8)
    feat = rng.standard_normal((16, 1)).astype(np.float32)
    target = rng.standard_normal((16, 21)).astype(np.float32) * 0.1
    loss0, g = h.loss_grad(phase, feat, target)
    h.adam_step(1e-3)
    p1 = h.get_params().cpu().numpy()
    ref, _, _ = OS.adam_step(theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size),
                             g.cpu().numpy().astype(np.float64), 1, 1e-3)
    assert np.abs(p1 - ref).max() < 1e-6
    for _ in range(150):
        loss, _ = h.loss_grad(phase, feat, target, want_grad=False)
        h.adam_step(3e-3)
    assert loss < 0.2 * loss0


def test_training_step_is_bitwise_reproducible():
    outs = []
    for _ in range(2):
        h, cfg = make(max_batch=8)
        theta, kw = random_theta(cfg, 9)
        h.set_params(theta)
        rng = np.random.default_rng(10)
        phase = (rng.random((8, 16, 16, 16)) < 0.4).astype(np.uint8)
        feat = rng.standard_normal((8, 1)).astype(np.float32)
        target = rng.standard_normal((8, 21)).astype(np.float32)
        for _ in range(3):
            h.loss_grad(phase, feat, target, want_grad=False)
            h.adam_step(1e-3)
        outs.append(h.get_params().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_phase_ids_above_one_are_rejected():
    from paper_2408_03804_amd.binding import FFTHomogError
    h, _ = make()
    h.set_params(random_theta(SMALL, 11)[0])
    phase = np.zeros((1, 16, 16, 16), np.uint8)
    phase[0, 3, 4, 5] = 2
    with pytest.raises(FFTHomogError):
        h.forward(phase, np.zeros((1, 1), np.float32))


def test_indicator_accepts_inside_bounds_and_rejects_outside():
    from paper_2408_03804_amd.surrogate import upper21
    h, _ = make()
    rng = np.random.default_rng(12)
    phase = (rng.random((5, 16, 16, 16)) < 0.3).astype(np.uint8)
    f1 = phase.reshape(5, -1).mean(axis=1)
    tables = np.array([[[1.0, 0.8], [6.0, 4.0]]] * 5)
    Cs = []
    for b in range(5):
        CV, CR = closed_forms.voigt_reuss([closed_forms.isotropic_matrix(1.0, 0.8, 3),
                                           closed_forms.isotropic_matrix(6.0, 4.0, 3)], [1 - f1[b], f1[b]])
        Cs.append([0.5 * (CV + CR), CV * 1.0, 2.0 * CV, 0.5 * CR, 0.5 * (CV + CR)][b])
    Cs = np.array(Cs)
    feat = np.array([[1.0], [1.0], [1.0], [1.0], [5.0]], np.float32)
    ok = h.check(phase, tables.reshape(5, 4), feat, upper21(Cs), 1e-3, 0.0, 2.0).cpu().numpy()
    assert list(ok) == [1, 1, 0, 0, 0]


def test_indicator_with_a_second_member_averages_and_tests_the_spread():
    from paper_2408_03804_amd.surrogate import upper21
    h, _ = make()
    rng = np.random.default_rng(13)
    phase = (rng.random((2, 16, 16, 16)) < 0.3).astype(np.uint8)
    f1 = phase.reshape(2, -1).mean(axis=1)
    tables = np.array([[[1.0, 0.8], [6.0, 4.0]]] * 2)
    C = []
    for b in range(2):
        CV, CR = closed_forms.voigt_reuss([closed_forms.isotropic_matrix(1.0, 0.8, 3),
                                           closed_forms.isotropic_matrix(6.0, 4.0, 3)], [1 - f1[b], f1[b]])
        C.append(0.5 * (CV + CR))
    C1 = upper21(np.array(C)).astype(np.float32)
    C2 = C1 * np.array([[1.02], [1.2]], np.float32)
    feat = np.ones((2, 1), np.float32)
    Ct = torch.as_tensor(C1).cuda()
    ok = h.check(phase, tables.reshape(2, 4), feat, Ct, 0.0, 0.0, 2.0, C2=C2, max_spread=0.05).cpu().numpy()
    # spreads 0.02 / 1.01 and 0.2 / 1.1 of the mean
    assert list(ok) == [1, 0]
    assert np.allclose(Ct.cpu().numpy(), 0.5 * (C1 + C2), rtol=1e-6)
    # the per-sample spread the caller calibrates its limit on
    Ct = torch.as_tensor(C1).cuda()
    ok2, sp = h.check(phase, tables.reshape(2, 4), feat, Ct, 0.0, 0.0, 2.0, C2=C2, max_spread=0.05, want_spread=True)
    assert list(ok2.cpu().numpy()) == [1, 0]
    assert np.allclose(sp.cpu().numpy(), [0.02 / 1.01, 0.2 / 1.1], rtol=1e-5)
    ok1, sp1 = h.check(phase, tables.reshape(2, 4), feat, torch.as_tensor(C1).cuda(), 0.0, 0.0, 2.0, want_spread=True)
    assert np.all(sp1.cpu().numpy() == 0.0)
