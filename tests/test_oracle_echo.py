"""Closed-form pins of the oracle's transport: every ray's fate in a planar
scene is predicted here from numpy's Philox stream (a library generator, not
the oracle's), the normal-incidence impedance formulas, straight-line
geometry and Beer-Lambert attenuation; the oracle must reproduce each
contribution to rounding. CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_2604_15017_amd import workloads as W


def philox_blocks(seed: int, tx_id: int, event: int, n_rays: int) -> np.ndarray:
    """Blocks Philox4x64-10(key=(seed, 0), counter=(r, tx_id, event, 0)) for
    r = 0..n_rays-1, from numpy's generator: its stream visits consecutive
    counters, starting one past its state, so the state is set one before."""
    c = [2**64 - 1, tx_id, event, 0]
    # borrow through the higher words
    i = 1
    while True:
        if c[i] == 0:
            c[i] = 2**64 - 1
            i += 1
        else:
            c[i] -= 1
            break
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array([seed, 0], dtype=np.uint64))
    return bg.random_raw(4 * n_rays).reshape(n_rays, 4)


def uniforms(blocks: np.ndarray) -> np.ndarray:
    return ((blocks >> np.uint64(41)).astype(np.float64) + 0.5) / 2**23


def test_philox_blocks_helper_matches_oracle():
    b = philox_blocks(0, 0, 1, 3)
    for r in range(3):
        assert np.array_equal(b[r], oracle.philox4x64_10([r, 0, 1, 0], [0, 0]))
    b = philox_blocks(7, 5, 0, 2)
    assert np.array_equal(b[1], oracle.philox4x64_10([1, 5, 0, 0], [7, 0]))


def _contribs_by_ray(tr):
    return {int(r): (int(e), t, a) for r, e, t, a in zip(tr.ray, tr.elem, tr.t, tr.a)}


def test_planar_echo_time_and_amplitude_normal_incidence():
    """Water over tissue, interface at 30 mm, 0 deg: a ray reflects iff its first
    interaction uniform is below R = ((Z2-Z1)/(Z2+Z1))^2, returns to its own
    element at t = 2d/c with amplitude (1/N)(A_r/R_E). Everything else escapes."""
    wl = W.two_layer(rays_per_elem=1 << 12)
    sc, p = wl.scene, wl.probe
    tr = oracle.trace(sc, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces)
    n = p.n_elem * wl.rays_per_elem
    Z1, Z2, c1, d = 1.48, 1.63, 1480.0, 30e-3
    Ar = (Z2 - Z1) / (Z2 + Z1)
    u_branch = uniforms(philox_blocks(wl.seed, 0, 1, n))[:, 0]
    reflect = np.nonzero(u_branch < Ar * Ar)[0]
    got = _contribs_by_ray(tr)
    assert len(got) == len(reflect) and len(tr.t) == len(reflect)
    t_echo = 2 * d / c1
    for r in reflect:
        e, t, a = got[int(r)]
        assert e == r // wl.rays_per_elem
        assert t == pytest.approx(t_echo, rel=1e-14)
        assert a == pytest.approx(Ar / (Ar * Ar) / wl.rays_per_elem, rel=1e-13)
    # the splatted histogram: k_e rays per element at sample t fs = 1621.62
    h = tr.splat(1, p.n_elem, p.n_t, p.fs)
    k = np.bincount(reflect // wl.rays_per_elem, minlength=p.n_elem)
    x = t_echo * p.fs
    j0, f = int(math.floor(x)), x - math.floor(x)
    assert j0 == 1621
    amp = k * (1.0 / Ar) / wl.rays_per_elem
    assert np.allclose(h[0, :, j0], amp * (1 - f), rtol=1e-12, atol=0)
    assert np.allclose(h[0, :, j0 + 1], amp * f, rtol=1e-12, atol=0)
    assert np.count_nonzero(h) == 2 * np.count_nonzero(k)
    # segments: every ray makes one segment to the interface and one more
    assert tr.segments == 2 * n


@pytest.mark.parametrize("deg", [10.0, -7.5])
def test_planar_echo_oblique_steering(deg):
    """Steered plane wave over a flat interface at d: the reflected ray from x0
    lands at x0 + 2 d tan(th) at t = x0 sin(th)/c + 2 d / (c cos th), on the
    element under it, with weight cos(th)/N * A_r/R_E."""
    wl = W.two_layer(rays_per_elem=1 << 10)
    th = math.radians(deg)
    d = 20e-3
    sc = wl.scene.with_theta(np.r_[wl.scene.regions.reshape(-1), [d], [0.0]])   # depth, roughness
    p = wl.probe
    tr = oracle.trace(sc, p, [th], [3], 11, wl.rays_per_elem, 4)
    n = p.n_elem * wl.rays_per_elem
    emit = uniforms(philox_blocks(11, 3, 0, n))
    u_branch = uniforms(philox_blocks(11, 3, 1, n))[:, 0]
    coef, _, _ = oracle.interface([math.sin(th), 0, math.cos(th)], [0, 0, 1.0],
                                  1480.0, 1.48, 1540.0, 1.63)
    Ar, RE = coef[0], coef[2]
    got = _contribs_by_ray(tr)
    half = 0.5 * p.n_elem * p.pitch
    expected = 0
    for r in np.nonzero(u_branch < RE)[0]:
        e = r // wl.rays_per_elem
        x0 = (e - 0.5 * (p.n_elem - 1)) * p.pitch + (emit[r, 0] - 0.5) * p.elem_width
        x1 = x0 + 2 * d * math.tan(th)
        if abs(x1) >= half:
            assert int(r) not in got
            continue
        expected += 1
        e1, t, a = got[int(r)]
        assert e1 == int(math.floor((x1 + half) / p.pitch))
        assert t == pytest.approx(x0 * math.sin(th) / 1480.0 + 2 * d / (1480.0 * math.cos(th)),
                                  rel=1e-13)
        assert a == pytest.approx(math.cos(th) / wl.rays_per_elem * Ar / RE, rel=1e-12)
    assert expected == len(got) == len(tr.t) and expected > 0


def test_attenuation_and_transmission_two_interfaces():
    """Water / attenuating tissue / stiff layer at normal incidence, 4 bounces.
    Only two families reach the array: the echo of the first interface (R) and
    the echo of the second seen through the first (T, R, T). The latter carries
    (A_t/T_E)(A_r'/R_E')(A_t''/T_E'') exp(-2 a L) with A_t = 2 Z2/(Z1 + Z2) and
    amplitude attenuation a = alpha f0[MHz] * 100 ln(10)/20 per metre."""
    rpe = 1 << 11
    wl = W.two_layer(rays_per_elem=rpe)
    d1, d2 = 10e-3, 25e-3
    Zw, Zt, Zb = 1.48, 1.63, 3.0
    cw, ct, cb = 1480.0, 1540.0, 2800.0
    alpha = 0.7
    sc = W.Scene(regions=np.array([[cw, Zw, 0.0], [ct, Zt, alpha], [cb, Zb, 0.2]]),
                 planes=np.array([d1, d2]), plane_regions=np.array([[0, 1], [1, 2]], np.int32),
                 plane_kd=np.zeros(2), spheres=np.zeros((0, 4)),
                 sphere_regions=np.zeros((0, 2), np.int32), sphere_kd=np.zeros(0))
    p = wl.probe
    tr = oracle.trace(sc, p, [0.0], [0], 5, rpe, 4)
    n = p.n_elem * rpe
    u = [None] + [uniforms(philox_blocks(5, 0, k, n))[:, 0] for k in (1, 2, 3)]

    def coeffs(Za, Zb_):
        return (Zb_ - Za) / (Zb_ + Za), 2 * Zb_ / (Za + Zb_)

    r1, t1 = coeffs(Zw, Zt)       # water -> tissue
    r2, _ = coeffs(Zt, Zb)        # tissue -> stiff, seen from above
    _, t3 = coeffs(Zt, Zw)        # tissue -> water on the way up
    R1, R2, R3 = r1 * r1, r2 * r2, ((Zw - Zt) / (Zw + Zt)) ** 2
    a_np = alpha * (p.f0 * 1e-6) * 100 * math.log(10) / 20
    got = _contribs_by_ray(tr)
    fam_R = np.nonzero(u[1] < R1)[0]
    fam_TRT = np.nonzero((u[1] >= R1) & (u[2] < R2) & (u[3] >= R3))[0]
    assert len(got) == len(fam_R) + len(fam_TRT) and len(fam_TRT) > 0
    for r in fam_R:
        e, t, a = got[int(r)]
        assert t == pytest.approx(2 * d1 / cw, rel=1e-14)
        assert a == pytest.approx(r1 / R1 / rpe, rel=1e-13)
    expect_a = (t1 / (1 - R1)) * (r2 / R2) * (t3 / (1 - R3)) * math.exp(-2 * a_np * (d2 - d1)) / rpe
    expect_t = 2 * d1 / cw + 2 * (d2 - d1) / ct
    for r in fam_TRT:
        e, t, a = got[int(r)]
        assert e == r // rpe
        assert t == pytest.approx(expect_t, rel=1e-14)
        assert a == pytest.approx(expect_a, rel=1e-12)


def test_das_peak_at_point_reflector():
    """A small, fully diffuse, nearly rigid sphere in water (so that almost no
    energy enters it and its far wall stays dark) images at its near surface
    (x_c, z_c - r), to within one pixel."""
    wl = W.two_layer(rays_per_elem=1 << 12)
    xc, zc, rad = 2.4e-3, 18e-3, 0.2e-3
    sc = W.Scene(regions=np.array([[1480.0, 1.48, 0.0], [1480.0, 1000.0, 0.0]]),
                 planes=np.zeros(0), plane_regions=np.zeros((0, 2), np.int32),
                 plane_kd=np.zeros(0), spheres=np.array([[xc, 0.0, zc, rad]]),
                 sphere_regions=np.array([[1, 0]], np.int32), sphere_kd=np.array([1.0]))
    wl = wl.replace(scene=sc, angles=np.radians([-5.0, 0.0, 5.0]),
                    tx_ids=np.arange(3, dtype=np.uint32))
    out = oracle.render(wl)
    B, g = out["B"], wl.grid
    a, b = np.unravel_index(np.argmax(B), B.shape)
    x, z = g.x0 + a * g.dx, g.z0 + b * g.dz
    assert abs(x - xc) <= g.dx and abs(z - (zc - rad)) <= g.dz
    assert out["trace"].t.shape[0] > 100
