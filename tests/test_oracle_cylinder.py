"""Pins of the oracle's cylinders (the hollow-cylinder scene of the paper's
forward check and inversion): every echo of a mirror cylinder under a 0 deg
plane wave predicted in closed form from numpy's Philox stream and circle
geometry; the dual-number gradients of the axis, radius, impedance and
roughness against central finite differences. CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_2604_15017_amd import workloads as W
from test_oracle_echo import philox_blocks, uniforms


def test_mirror_cylinder_echoes_in_closed_form():
    """0 deg, one interaction: a ray from x0 with |x0| < R meets the wall at
    z_h = z_c - sqrt(R^2 - x0^2) with normal n = (x0, 0, z_h - z_c)/R, and if
    its branch uniform is below R_E there, returns along w' = w - 2 (w.n) n to
    the element under x0 + z_h w'_x / (-w'_z), at t = (z_h + z_h / (-w'_z)) / c
    with amplitude (1/N)(A_r/R_E) f_d; rays missing the cylinder, refracted
    or landing beside the array leave nothing."""
    rpe = 1 << 9
    wl = W.cylinder_phantom(rough=0.0, kd=0.0).replace(rays_per_elem=rpe, angles=np.array([0.0]),
                                                      tx_ids=np.array([2], dtype=np.uint32))
    sc, p = wl.scene, wl.probe
    xc, zc, R = sc.cylinders[0]
    c1 = sc.regions[0, 0]
    tr = oracle.trace(sc, p, wl.angles, wl.tx_ids, 17, rpe, 1)
    got = {int(r): (int(e), t, a) for r, e, t, a in zip(tr.ray, tr.elem, tr.t, tr.a)}
    n = p.n_elem * rpe
    emit = uniforms(philox_blocks(17, 2, 0, n))
    u_branch = uniforms(philox_blocks(17, 2, 1, n))[:, 0]
    half = 0.5 * p.n_elem * p.pitch
    expected = 0
    for r in range(n):
        e = r // rpe
        x0 = (e - 0.5 * (p.n_elem - 1)) * p.pitch + (emit[r, 0] - 0.5) * p.elem_width
        if abs(x0 - xc) >= R:
            assert r not in got
            continue
        zh = zc - math.sqrt(R * R - (x0 - xc) ** 2)
        nrm = np.array([x0 - xc, 0.0, zh - zc]) / R
        w = np.array([0.0, 0.0, 1.0])
        coef, w_refl, _ = oracle.interface(w, nrm, c1, sc.regions[0, 1], sc.regions[1, 0], sc.regions[1, 1])
        Ar, RE = coef[0], coef[2]
        assert np.allclose(w_refl, w - 2 * (w @ nrm) * nrm, atol=1e-15)
        if u_branch[r] >= RE or w_refl[2] >= 0:
            assert r not in got
            continue
        x1 = x0 + zh * w_refl[0] / (-w_refl[2])
        if abs(x1) >= half:
            assert r not in got
            continue
        cos_a = -w_refl[2]
        fd = oracle.directivity(p, cos_a)
        if fd == 0.0:
            assert r not in got
            continue
        expected += 1
        e1, t, a = got[r]
        assert e1 == int(math.floor((x1 + half) / p.pitch))
        assert t == pytest.approx((zh + zh / cos_a) / c1, rel=1e-12)
        assert a == pytest.approx(1.0 / rpe * Ar / RE * fd, rel=1e-11)
    assert expected == len(got) == len(tr.t) and expected > 20


def test_cylinder_gradients_match_finite_differences():
    wl = W.cylinder_phantom().replace(rays_per_elem=64, angles=np.radians([-8.0, 0.0, 6.0]),
                                      tx_ids=np.arange(3, dtype=np.uint32))
    sc, p = wl.scene, wl.probe
    theta = sc.theta()
    rng = np.random.default_rng(6)
    k = np.exp(-0.5 * (np.arange(-30, 31) / 10.0) ** 2)
    g_h = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1,
                              rng.standard_normal((wl.n_tx, p.n_elem, p.n_t)))
    probs = oracle.trace(sc, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                         theta=theta, record_probs=True).probs
    idx = [sc.idx_cylinder(0, "x"), sc.idx_cylinder(0, "z"), sc.idx_cylinder(0, "R"),
           sc.idx_rough("cylinder", 0), sc.idx_region(1, "Z"), sc.idx_region(1, "c")]
    ad = oracle.trace(sc, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                      theta=theta, g_h=g_h, grad_params=idx).g_theta

    def L(th):
        tr = oracle.trace(sc, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                          theta=th, probs=probs)
        return float(np.sum(g_h * tr.splat(wl.n_tx, p.n_elem, p.n_t, p.fs)))

    unit = np.where(theta != 0, np.abs(theta), 1e-3)
    scale = max(abs(ad[j]) * unit[j] for j in idx)
    for j in idx:
        h = 1e-7 * unit[j]
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        assert abs(fd - ad[j]) * unit[j] <= 1e-3 * abs(ad[j]) * unit[j] + 1e-7 * scale, (j, fd, ad[j])
        assert abs(ad[j]) * unit[j] > 1e-4 * scale, j   # each parameter moves the signal here


def test_fd_step_sweep_of_the_cylinder_image_loss():
    """The paper's AD-versus-FD comparison on the simulated-reference cylinder
    problem: dual-number gradients of the B-mode MSE with respect to R, Z and
    the roughness against central differences over steps of 1e-2 .. 1e-9
    (relative), at fixed branch probabilities. Large steps carry truncation
    error (and discrete changes of the paths), the smallest cancellation; the
    agreement is best in between, where it reaches 1e-3."""
    wl = W.cylinder_phantom().replace(rays_per_elem=24, angles=np.radians([-5.0, 5.0]),
                                      tx_ids=np.arange(2, dtype=np.uint32),
                                      grid=W.Grid.span(32, 64, -6.4e-3, 6.4e-3, 5e-3, 25e-3))
    sc = wl.scene
    idx = [sc.idx_cylinder(0, "R"), sc.idx_region(1, "Z"), sc.idx_rough("cylinder", 0)]
    tgt = sc.theta().copy()
    tgt[idx] = [5.2e-3, 1.8, 0.25]
    B_ref = oracle.render(wl, theta=tgt)["B"]
    theta = sc.theta()
    ad = oracle.grad_theta(wl, B_ref, theta=theta, grad_params=idx)["g_theta"]
    probs = oracle.render(wl, theta=theta, record_probs=True)["trace"].probs

    def L(th):
        return oracle.mse(oracle.render(wl, theta=th, probs=probs)["B"], B_ref)

    steps = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9]
    for j, name in zip(idx, ("R", "Z", "rho")):
        errs = []
        for rel in steps:
            h = rel * abs(theta[j])
            tp, tm = theta.copy(), theta.copy()
            tp[j] += h
            tm[j] -= h
            fd = (L(tp) - L(tm)) / (2 * h)
            errs.append(abs(fd - ad[j]) / abs(ad[j]))
        print(f"{name}: AD {ad[j]:.6e}; |FD - AD| / |AD| over steps {steps}: "
              + " ".join(f"{e:.1e}" for e in errs), flush=True)
        assert min(errs) <= 1e-3
        assert errs[0] > min(errs)        # truncation at the largest step
