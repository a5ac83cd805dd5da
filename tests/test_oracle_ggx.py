"""Pins of the oracle's rough reflection (Eq. GGX_PDF): the mirror at zero
roughness, the distribution of the sampled microfacet normals against the
normal distribution function integrated numerically, the mean estimator
factor against the directional albedo of the microfacet BRDF by quadrature,
and the roughness gradients against central finite differences of the
transport. CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_2604_15017_amd import workloads as W

WATER, TISSUE = (1480.0, 1.48), (1540.0, 1.63)


def _dir(theta_deg, phi_deg=0.0):
    t, p = math.radians(theta_deg), math.radians(phi_deg)
    return np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])


@pytest.mark.parametrize("theta_i", [0.0, 25.0, 60.0])
def test_zero_roughness_is_the_mirror(theta_i):
    w = _dir(theta_i, 30.0)
    n = np.array([0.2, -0.1, -0.97]) / np.linalg.norm([0.2, -0.1, -0.97])   # faces the incoming ray
    _, w_refl, _ = oracle.interface(w, n, *WATER, *TISSUE)
    for u1, u2 in ((0.3, 0.7), (0.99, 0.01)):
        d, g, ok = oracle.glossy(w, n, *WATER, *TISSUE, 0.0, u1, u2)
        assert ok and np.array_equal(d, w_refl)
        assert g == pytest.approx(1.0, abs=1e-15)


def _cap_integral(a, rho, m=20000):
    """Integral of D(h) cos(theta_h) over the cap theta_h <= a (quadrature)."""
    t = (np.arange(m) + 0.5) / m * a
    c = np.cos(t)
    d = rho ** 2 / (np.pi * (c ** 2 * (rho ** 2 - 1.0) + 1.0) ** 2)
    return float(np.sum(d * c * np.sin(t)) * 2 * np.pi * a / m)


@pytest.mark.parametrize("rho", [0.05, 0.3, 0.8])
def test_microfacet_normals_follow_the_distribution(rho):
    """At normal incidence every sampled microfacet faces the incident ray, so
    the half vector of (incident, reflected) recovers it for all samples; over
    a stratified grid of (u1, u2) the fraction with theta_h <= a matches the
    integral of D(h) cos(theta_h) over that cap (Eq. GGX_PDF by quadrature;
    the whole hemisphere integrates to 1)."""
    n = np.array([0.0, 0.0, -1.0])
    w = np.array([0.0, 0.0, 1.0])
    m = 64
    grid = (np.arange(m) + 0.5) / m
    theta_h = []
    for u1 in grid:
        for u2 in grid:
            d, _, _ = oracle.glossy(w, n, *WATER, *TISSUE, rho, u1, u2)
            h = d - w
            h /= np.linalg.norm(h)
            theta_h.append(math.acos(min(1.0, -h[2])))
    theta_h = np.array(theta_h)
    assert _cap_integral(math.pi / 2, rho) == pytest.approx(1.0, abs=2e-4)
    for a in (0.5 * rho, rho, 2.0 * rho, 4.0 * rho):
        a = min(math.atan(a), 1.5)
        # the grid is stratified in the cap probability: at most one row off
        assert np.mean(theta_h <= a) == pytest.approx(_cap_integral(a, rho), abs=1.0 / m + 1e-3)


@pytest.mark.parametrize("rho,theta_i", [(0.1, 10.0), (0.3, 30.0), (0.6, 45.0), (0.9, 60.0)])
def test_mean_factor_is_the_directional_albedo(rho, theta_i):
    """E[g] over the sampled microfacets equals the albedo of the microfacet
    BRDF with unit Fresnel, int D G1(i) G1(o) / (4 cos_i cos_o) cos_o do,
    computed by quadrature over the reflected hemisphere; it is below 1
    (shadowing and masking)."""
    n = np.array([0.0, 0.0, -1.0])
    w = _dir(theta_i)
    i = -w
    cos_i = float(-n @ w)
    m = 256
    u = (np.arange(m) + 0.5) / m
    mc = np.mean([oracle.glossy(w, n, *WATER, *TISSUE, rho, a, b)[1] for a in u for b in u])
    nt, nphi = 1600, 512
    t = (np.arange(nt) + 0.5) / nt * (np.pi / 2)
    ph = (np.arange(nphi) + 0.5) / nphi * 2 * np.pi
    T, P = np.meshgrid(t, ph, indexing="ij")
    o = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), -np.cos(T)], axis=-1)
    h = o + i
    h /= np.linalg.norm(h, axis=-1, keepdims=True)
    ch, co = -h[..., 2], np.cos(T)
    d = rho ** 2 / (np.pi * (ch ** 2 * (rho ** 2 - 1.0) + 1.0) ** 2)
    g1 = lambda c: 2.0 * c / (c + np.sqrt(rho ** 2 + (1.0 - rho ** 2) * c ** 2))
    f = d * g1(cos_i) * g1(co) / (4 * cos_i * co)
    albedo = float(np.sum(f * co * np.sin(T)) * (np.pi / 2 / nt) * (2 * np.pi / nphi))
    assert albedo < 1.0
    assert mc == pytest.approx(albedo, rel=3e-3)


def test_roughness_gradient_matches_finite_differences():
    """Rough spheres and planes: dual-number gradients of the roughness (and of
    the geometry they couple to) against central differences of the fp64
    transport at fixed branch probabilities."""
    wl = W.rough_layered_phantom().replace(rays_per_elem=96, angles=np.radians([-6.0, 0.0, 4.0]),
                                           tx_ids=np.arange(3, dtype=np.uint32))
    sc, p = wl.scene, wl.probe
    theta = sc.theta()
    rng = np.random.default_rng(3)
    k = np.exp(-0.5 * (np.arange(-30, 31) / 10.0) ** 2)
    g_h = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1,
                              rng.standard_normal((wl.n_tx, p.n_elem, p.n_t)))
    probs = oracle.trace(sc, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                         theta=theta, record_probs=True).probs
    idx = [sc.idx_rough("plane", j) for j in range(sc.n_planes)]
    idx += [sc.idx_rough("sphere", j) for j in range(sc.n_spheres)]
    idx += [sc.idx_sphere(0, "r"), sc.idx_plane(1), sc.idx_region(2, "Z")]
    ad = oracle.trace(sc, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                      theta=theta, g_h=g_h, grad_params=idx).g_theta

    def L(th):
        tr = oracle.trace(sc, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                          theta=th, probs=probs)
        return float(np.sum(g_h * tr.splat(wl.n_tx, p.n_elem, p.n_t, p.fs)))

    unit = np.abs(theta)
    scale = max(abs(ad[j]) * unit[j] for j in idx)
    significant = 0
    for j in idx:
        h = 1e-7 * unit[j]
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        assert abs(fd - ad[j]) * unit[j] <= 1e-3 * abs(ad[j]) * unit[j] + 1e-7 * scale, (j, fd, ad[j])
        significant += abs(ad[j]) * unit[j] > 1e-3 * scale
    print(f"{significant} of {len(idx)} parameters significant", flush=True)
    # the deepest plane reflects too rarely at this ray count to matter
    assert significant >= 6
