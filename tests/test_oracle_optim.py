"""Pins of the oracle's inverse-loop pieces (Sec. "Parameterization and
constraints", Sec. "Loss function", Sec. "Optimization procedure"): closed
forms, finite differences and torch.optim.Adam. CPU only."""
import numpy as np
import pytest

import oracle
from oracle import optim


def test_param_map_closed_forms():
    lo, hi = np.array([1.0, -2.0, 5.0, 3.0]), np.array([3.0, 2.0, 5.0, 7.0])
    u = np.array([0.5, -0.3, 0.7, 1.4])
    th = optim.param_map(u, lo, hi)
    assert th[0] == 2.0            # midpoint
    assert th[1] == -2.0           # clipped at the lower bound
    assert th[2] == 5.0            # fixed parameter (lo == hi)
    assert th[3] == 7.0            # clipped at the upper bound


def test_clip_derivative_against_finite_differences():
    rng = np.random.default_rng(0)
    lo, hi = rng.uniform(-1, 0, 6), rng.uniform(1, 2, 6)
    u = np.array([0.2, 0.9, -0.1, 1.3, 0.5, 0.0])
    g_theta = rng.standard_normal(6)
    g_u = optim.unconstrained_grad(g_theta, u, lo, hi)
    h = 1e-6
    for j in range(6):
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        # L = g_theta . theta(u): central difference inside, one-sided beyond a bound
        fd = (g_theta @ optim.param_map(up, lo, hi) - g_theta @ optim.param_map(um, lo, hi)) / (2 * h)
        if 0.0 < u[j] < 1.0:
            assert g_u[j] == pytest.approx(fd, rel=1e-8)
        else:
            assert g_u[j] == 0.0
    # a bound itself counts as saturated (Eq. clip_grad uses strict inequalities)
    assert optim.unconstrained_grad([1.0], [1.0], [0.0], [1.0])[0] == 0.0


def test_first_adam_step_is_signed_learning_rate():
    """With m_0 = v_0 = 0 the bias-corrected moments are g and g^2, so the
    first step moves each variable by lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    lr = np.array([0.1, 0.2, 0.05, 0.1])
    u, m, v = optim.adam_update(np.zeros(4), np.zeros(4), np.zeros(4), g, lr, 1)
    assert np.allclose(u, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    u0 = rng.uniform(0.2, 0.8, 5)
    p = torch.tensor(u0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.03, betas=(0.8, 0.95), eps=1e-7)
    u, m, v = u0.copy(), np.zeros(5), np.zeros(5)
    for k in range(1, 8):
        g = rng.standard_normal(5)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        u, m, v = optim.adam_update(u, m, v, g, np.full(5, 0.03), k, 0.8, 0.95, 1e-7)
    assert np.allclose(u, p.detach().numpy(), rtol=0, atol=1e-14)


def test_clip_norm():
    g = np.array([3.0, 4.0])
    assert np.allclose(optim.clip_norm(g, 1.0), [0.6, 0.8], rtol=1e-15)
    assert np.array_equal(optim.clip_norm(g, 10.0), g)
    assert np.array_equal(optim.clip_norm(g, 0.0), g)   # disabled


def test_image_loss_closed_form_and_gradient():
    B = np.array([[-10.0, -3.0], [0.0, -60.0]])
    R = np.array([[-12.0, -3.0], [-1.0, -55.0]])
    L, g = optim.image_loss(B, R, 0.3, 0.7)
    d = B - R   # 2, 0, 1, -5
    assert L == pytest.approx((0.3 * (2 + 0 + 1 + 5) + 0.7 * (4 + 0 + 1 + 25)) / 4, rel=1e-15)
    assert np.allclose(g, (0.3 * np.sign(d) + 1.4 * d) / 4, rtol=1e-15)
    # pure L2 is the oracle's mean squared error
    assert optim.image_loss(B, R, 0.0, 1.0)[0] == pytest.approx(oracle.mse(B, R), rel=1e-15)
    # gradient by central differences away from the L1 kink
    rng = np.random.default_rng(2)
    B, R = rng.standard_normal((3, 4)), rng.standard_normal((3, 4))
    _, g = optim.image_loss(B, R, 0.4, 0.6)
    h = 1e-6
    for idx in np.ndindex(B.shape):
        bp, bm = B.copy(), B.copy()
        bp[idx] += h
        bm[idx] -= h
        fd = (optim.image_loss(bp, R, 0.4, 0.6)[0] - optim.image_loss(bm, R, 0.4, 0.6)[0]) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6)
