"""Pins of the oracle's parameter gradients (paper Sec. 3.2, Eq. chain_rule):
forward-mode dual numbers at fixed ray realizations against central finite
differences of the oracle's own FP64 forward, at the transport level and
through the whole image chain. CPU only.

The function differentiated is the fixed-sample estimator whose branch
probabilities are sampling densities: they decide the branch and divide the
weight, but are not differentiated (so the gradient is unbiased for the
expected image). Finite differences therefore perturb theta with the branch
probabilities recorded at the unperturbed theta.

Finite differences use a relative step of 1e-7 (1e-8 through the image chain;
absolute 1e-9 for zero parameters): small enough that hardly any discrete
choice (element under a returning ray, sphere hit or miss) flips and hardly any
deposit crosses a sample boundary, large enough that FP64 cancellation stays
far below the tolerance."""
import numpy as np
import pytest

import oracle
from paper_2604_15017_amd import workloads as W


def _small_phantom(rays_per_elem=48, n_tx=3):
    wl = W.layered_phantom()
    ang = np.radians(np.linspace(-10, 10, n_tx))
    return wl.replace(rays_per_elem=rays_per_elem, angles=ang,
                      tx_ids=np.arange(n_tx, dtype=np.uint32),
                      grid=W.Grid.span(24, 48, -19.2e-3, 19.2e-3, 0.0, 60e-3))


def _smooth_field(shape, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(shape)
    k = np.exp(-0.5 * (np.arange(-30, 31) / 10.0) ** 2)
    return np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1, g)


def _fd(fun, theta, j, rel=1e-7):
    h = rel * abs(theta[j]) if theta[j] != 0 else 1e-2 * rel
    tp, tm = theta.copy(), theta.copy()
    tp[j] += h; tm[j] -= h
    return (fun(tp) - fun(tm)) / (2 * h)


def test_transport_gradient_matches_finite_differences():
    wl = _small_phantom()
    p = wl.probe
    theta = wl.scene.theta()
    g_h = _smooth_field((wl.n_tx, p.n_elem, p.n_t), 7)

    probs = oracle.trace(wl.scene, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                         wl.max_bounces, theta=theta, record_probs=True).probs

    def L(th):
        tr = oracle.trace(wl.scene, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                          wl.max_bounces, theta=th, probs=probs)
        return float(np.sum(g_h * tr.splat(wl.n_tx, p.n_elem, p.n_t, p.fs)))

    tr = oracle.trace(wl.scene, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                      wl.max_bounces, theta=theta, g_h=g_h)
    ad = tr.g_theta
    # compare sensitivities per unit relative change (metres vs m/s vs MRayl)
    unit = np.where(theta != 0, np.abs(theta), 1e-3)
    scale = np.abs(ad * unit).max()
    checked = 0
    for j in range(theta.shape[0]):
        fd = _fd(L, theta, j)
        assert abs(fd - ad[j]) * unit[j] <= 1e-3 * abs(ad[j]) * unit[j] + 1e-7 * scale, (j, fd, ad[j])
        checked += abs(ad[j]) * unit[j] > 1e-4 * scale
    assert checked >= 28          # most parameters carry real signal here


def test_full_chain_gradient_matches_finite_differences():
    """MSE between B-mode images in dB (target from seeded +-5 % parameters)."""
    wl = _small_phantom(rays_per_elem=32, n_tx=2)
    target = W.layered_phantom_target(wl)
    B_ref = oracle.render(wl, theta=target.theta())["B"]
    theta = wl.scene.theta()
    idx = W.perturbed_indices(wl.scene)
    out = oracle.grad_theta(wl, B_ref, theta=theta, grad_params=idx)
    ad = out["g_theta"]

    probs = oracle.render(wl, theta=theta, record_probs=True)["trace"].probs

    def L(th):
        return oracle.mse(oracle.render(wl, theta=th, probs=probs)["B"], B_ref)

    assert out["loss"] == pytest.approx(L(theta), rel=1e-12)
    unit = np.where(theta != 0, np.abs(theta), 1e-3)
    scale = np.abs(ad[idx] * unit[idx]).max()
    for j in idx:
        # the image chain makes dL/dh rough on the sample scale, so the step is
        # kept small enough that no deposit crosses a sample boundary
        fd = _fd(L, theta, j, rel=1e-8)
        assert abs(fd - ad[j]) * unit[j] <= 1e-3 * abs(ad[j]) * unit[j] + 1e-6 * scale, (j, fd, ad[j])
