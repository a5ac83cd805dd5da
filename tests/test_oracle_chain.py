"""Pins of the oracle's image chain: a library Hilbert transform, closed forms,
adjoint identities <K x, y> = <x, K^T y>, and finite differences. CPU only."""
import math

import numpy as np
import pytest
import scipy.signal

import oracle
from paper_2604_15017_amd import workloads as W


def test_analytic_signal_matches_scipy_hilbert():
    rng = np.random.default_rng(0)
    for n in (64, 2048, 4097):
        x = rng.standard_normal((3, n))
        assert np.allclose(oracle.analytic(x), scipy.signal.hilbert(x, axis=-1), atol=1e-12)


def test_analytic_tone_has_unit_envelope():
    n, k = 4096, 300
    t = np.arange(n)
    A = oracle.analytic(np.cos(2 * np.pi * k * t / n))
    assert np.allclose(np.abs(A), 1.0, atol=1e-12)
    assert np.allclose(A.imag, np.sin(2 * np.pi * k * t / n), atol=1e-12)


def _real_inner(a, b):
    return float(np.sum(np.real(np.conj(a) * b)))


def test_pulse_adjoint_identity():
    rng = np.random.default_rng(1)
    _, s = oracle.pulse_taps(5e6, 2.0, 40e6)
    x = rng.standard_normal((2, 3, 500)); y = rng.standard_normal((2, 3, 500))
    assert _real_inner(oracle.pulse(x, s), y) == pytest.approx(_real_inner(x, oracle.pulse_vjp(y, s)), rel=1e-12)


def test_pulse_of_single_impulse_is_the_pulse():
    _, s = oracle.pulse_taps(5e6, 2.0, 40e6)
    h = np.zeros(300); h[150] = 2.0
    rf = oracle.pulse(h, s)
    M = (len(s) - 1) // 2
    assert np.allclose(rf[150 - M:150 + M + 1], 2.0 * s)
    assert np.count_nonzero(rf) == np.count_nonzero(s)


def test_analytic_adjoint_identity():
    rng = np.random.default_rng(2)
    for n in (256, 257):
        x = rng.standard_normal((4, n))
        y = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
        assert _real_inner(oracle.analytic(x), y) == pytest.approx(_real_inner(x, oracle.analytic_vjp(y)), rel=1e-12)


def _small_geometry():
    wl = W.two_layer()
    probe = W.Probe(n_elem=8, pitch=0.3e-3, elem_width=0.3e-3, elem_height=5e-3, f0=5e6,
                    n_cycles=2, fs=40e6, n_t=400, c_ref=1540.0)
    grid = W.Grid.span(9, 21, -2e-3, 2e-3, 2e-3, 7e-3)
    return probe, grid, np.radians([-6.0, 0.0, 9.0])


def test_das_adjoint_identity():
    rng = np.random.default_rng(3)
    probe, grid, angles = _small_geometry()
    A = rng.standard_normal((3, 8, 400)) + 1j * rng.standard_normal((3, 8, 400))
    gI = rng.standard_normal((9, 21)) + 1j * rng.standard_normal((9, 21))
    lhs = _real_inner(oracle.das(A, probe, grid, angles), gI)
    rhs = _real_inner(A, oracle.das_vjp(gI, probe, grid, angles, 400))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_das_brute_force_single_pixel():
    """One pixel by the printed sum, term by term, with explicit interpolation."""
    rng = np.random.default_rng(4)
    probe, grid, angles = _small_geometry()
    A = rng.standard_normal((3, 8, 400)) + 1j * rng.standard_normal((3, 8, 400))
    I = oracle.das(A, probe, grid, angles)
    a, b = 4, 13
    x, z = grid.x0 + a * grid.dx, grid.z0 + b * grid.dz
    acc = 0j
    for i, th in enumerate(angles):
        for e in range(8):
            xe = (e - 3.5) * 0.3e-3
            tau = (x * math.sin(th) + z * math.cos(th)) / 1540.0 + math.hypot(x - xe, z) / 1540.0
            k = tau * 40e6
            k0 = int(math.floor(k))
            acc += (k0 + 1 - k) * A[i, e, k0] + (k - k0) * A[i, e, k0 + 1]
    assert I[a, b] == pytest.approx(acc, rel=1e-12)


def test_bmode_values_and_clip():
    I = np.array([[3 + 4j, 0.5, 0.0], [1e-5, -5.0, 2.5j]])
    B = oracle.bmode(I, 60.0)
    assert B[0, 0] == 0.0 and B[1, 1] == 0.0
    assert B[0, 1] == pytest.approx(20 * math.log10(0.1))
    assert B[0, 2] == -60.0 and B[1, 0] == -60.0
    assert B[1, 2] == pytest.approx(20 * math.log10(0.5))


def test_bmode_vjp_finite_differences():
    """Directional derivatives of L(B(I)) against central differences in FP64,
    including the normalisation by the frame maximum."""
    rng = np.random.default_rng(5)
    I = rng.standard_normal((6, 7)) + 1j * rng.standard_normal((6, 7))
    I[2, 3] = 10 + 2j                       # a clear maximum
    I[0, 0] = 1e-4                          # a clipped pixel
    g_B = rng.standard_normal(I.shape)
    L = lambda J: float(np.sum(g_B * oracle.bmode(J, 60.0)))
    g = oracle.bmode_vjp(I, g_B, 60.0)
    for _ in range(6):
        dI = rng.standard_normal(I.shape) + 1j * rng.standard_normal(I.shape)
        eps = 1e-7
        fd = (L(I + eps * dI) - L(I - eps * dI)) / (2 * eps)
        assert _real_inner(g, dI) == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_nee_matches_bsdf_sampling_in_expectation():
    """Receiver-directed secondary rays and plain lobe sampling estimate the same
    expected signal: a fully diffuse stiff plane seen by small elements
    (point-element approximation error ~ (size/range)^2 ~ 1e-3). Totals per
    element agree within 4 standard errors of the noisier estimator."""
    probe = W.Probe(n_elem=16, pitch=0.4e-3, elem_width=0.4e-3, elem_height=0.4e-3, f0=5e6,
                    n_cycles=2, fs=40e6, n_t=2048, c_ref=1480.0)
    sc = W.Scene(regions=np.array([[1480.0, 1.48, 0.0], [1480.0, 15.0, 0.0]]),
                 planes=np.array([15e-3]), plane_regions=np.array([[0, 1]], np.int32),
                 plane_kd=np.array([1.0]), spheres=np.zeros((0, 4)),
                 sphere_regions=np.zeros((0, 2), np.int32), sphere_kd=np.zeros(0))
    rpe = 1 << 17
    nee = oracle.trace(sc, probe, [0.0], [0], 3, rpe, 1, nee_mode=0)
    bsdf = oracle.trace(sc, probe, [0.0], [0], 3, rpe, 1, nee_mode=1)
    tot_nee = np.bincount(nee.elem, weights=nee.a, minlength=16)
    tot_bsdf = np.bincount(bsdf.elem, weights=bsdf.a, minlength=16)
    # standard error of the lobe-sampling total from its per-ray weights
    se = np.sqrt(np.bincount(bsdf.elem, weights=bsdf.a ** 2, minlength=16))
    assert np.all(np.abs(tot_nee - tot_bsdf) < 4 * se + 2e-3 * tot_nee)
    assert abs(tot_nee.sum() - tot_bsdf.sum()) < 4 * math.sqrt(np.sum(se ** 2)) + 2e-3 * tot_nee.sum()
    # arrival times: both spread over the same window
    assert abs(np.average(nee.t, weights=nee.a) - np.average(bsdf.t, weights=bsdf.a)) < 0.1e-6


def test_das_acquisition_gradients_match_finite_differences():
    """dL/d(angles, c_ref, pitch) of L = Re <g, I> at fixed analytic signal,
    against central differences of the oracle's delay-and-sum with the
    parameter moved (Eq. das; I is piecewise linear in each sample index,
    and a step of 1e-7 relative crosses a sample boundary at too few pixels
    to matter)."""
    import dataclasses
    rng = np.random.default_rng(17)
    wl = W.two_layer()
    p = dataclasses.replace(wl.probe, n_elem=12, n_t=1024)
    g = W.Grid.span(10, 14, -3e-3, 3e-3, 8e-3, 14e-3)
    angles = np.radians([-7.0, 2.0, 9.0])
    k = np.exp(-0.5 * (np.arange(-9, 10) / 3.0) ** 2)
    rf = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1,
                             rng.standard_normal((3, p.n_elem, p.n_t)))
    A = oracle.analytic(rf)
    g_I = rng.standard_normal((g.n_x, g.n_z)) + 1j * rng.standard_normal((g.n_x, g.n_z))
    g_th, g_c, g_p = oracle.das_acq_vjp(A, g_I, p, g, angles)

    def L(probe, ang):
        return _real_inner(g_I, oracle.das(A, probe, g, ang))

    fd_th = []
    for i in range(len(angles)):
        h = 1e-7
        ap, am = angles.copy(), angles.copy()
        ap[i] += h
        am[i] -= h
        fd_th.append((L(p, ap) - L(p, am)) / (2 * h))
    hc = 1e-7 * p.c_ref
    fd_c = (L(dataclasses.replace(p, c_ref=p.c_ref + hc), angles)
            - L(dataclasses.replace(p, c_ref=p.c_ref - hc), angles)) / (2 * hc)
    hp = 1e-7 * p.pitch
    fd_p = (L(dataclasses.replace(p, pitch=p.pitch + hp), angles)
            - L(dataclasses.replace(p, pitch=p.pitch - hp), angles)) / (2 * hp)
    got = np.array([*g_th, g_c, g_p])
    want = np.array([*fd_th, fd_c, fd_p])
    print("acquisition gradients", got, "finite differences", want)
    assert np.all(np.abs(got) > 0)
    assert np.allclose(got, want, rtol=2e-4, atol=0.0)
