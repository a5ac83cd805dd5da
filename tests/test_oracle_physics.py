"""Pins of the oracle's building blocks against things other than itself:
a library generator, conservation laws, Snell's law, closed forms, and
distributional facts. CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_2604_15017_amd import workloads as W


# ------------------------------------------------------------------ Philox
def test_philox_matches_numpy_library():
    """numpy's Philox is the 4x64-10 variant of Salmon et al. (SC'11); its first
    output block for state counter c is the block for counter c + 1."""
    for key, ctr in [((0, 0), (0, 0, 0, 0)), ((12345, 0), (7, 3, 2, 0)),
                     ((2**63 + 5, 0), (2**64 - 2, 11, 8, 0)), ((1, 0), (99, 0, 0, 5))]:
        bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64),
                              key=np.array(key, dtype=np.uint64))
        ref = bg.random_raw(4)
        nxt = list(ctr)
        nxt[0] = (nxt[0] + 1) % 2**64
        carry = nxt[0] == 0
        for i in range(1, 4):
            if not carry:
                break
            nxt[i] = (nxt[i] + 1) % 2**64
            carry = nxt[i] == 0
        ours = oracle.philox4x64_10(nxt, key)
        assert np.array_equal(ours, ref), (key, ctr)


def test_uniform_exact_in_float32_and_open_interval():
    for x in [0, 1, 2**41 - 1, 2**41, 2**64 - 1, 0x123456789ABCDEF0]:
        u = oracle.uniform(x)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
        assert u == ((x >> 41) + 0.5) / 2**23


# ------------------------------------------------------------------ interface physics
def _independent_transmitted_energy(c1, Z1, c2, Z2, cos_i, At):
    """Energy flux carried across the interface by a transmitted pressure wave of
    amplitude A_t: intensity p^2 / (2 Z) times the projected area ratio."""
    cos_t = math.sqrt(1.0 - (c2 / c1) ** 2 * (1.0 - cos_i ** 2))
    return (Z1 * cos_t) / (Z2 * cos_i) * At ** 2


@pytest.mark.parametrize("c1,Z1,c2,Z2", [(1480, 1.48, 1540, 1.63), (1540, 1.63, 1480, 1.48),
                                         (1450, 1.8, 1600, 1.3), (1600, 1.3, 1450, 1.8),
                                         (1500, 1.5, 1500, 1.5)])
def test_energy_conservation_and_snell(c1, Z1, c2, Z2):
    rng = np.random.default_rng(0)
    crit = math.asin(min(1.0, c1 / c2)) if c2 > c1 else math.pi / 2
    for _ in range(200):
        th = rng.uniform(0, min(crit, math.radians(89.0)) - 1e-6)
        phi = rng.uniform(0, 2 * math.pi)
        n = np.array([0.3, -0.2, 0.93]); n /= np.linalg.norm(n)
        # incident direction making angle th with -n
        t1 = np.cross(n, [1.0, 0, 0]); t1 /= np.linalg.norm(t1); t2 = np.cross(n, t1)
        w = -math.cos(th) * n + math.sin(th) * (math.cos(phi) * t1 + math.sin(phi) * t2)
        # normal given either way round must not matter
        for nn in (n, -n):
            coef, wr, wt = oracle.interface(w, nn, c1, Z1, c2, Z2)
            Ar, At, RE, tir = coef
            assert tir == 0.0
            assert RE == pytest.approx(Ar * Ar, rel=1e-15)
            TE = _independent_transmitted_energy(c1, Z1, c2, Z2, math.cos(th), At)
            assert RE + TE == pytest.approx(1.0, abs=1e-13)
            # mirror: same angle, tangential part kept, normal part flipped
            assert np.linalg.norm(wr) == pytest.approx(1.0, abs=1e-14)
            assert np.dot(wr, n) == pytest.approx(-np.dot(w, n), abs=1e-14)
            assert np.allclose(wr - np.dot(wr, n) * n, w - np.dot(w, n) * n, atol=1e-14)
            # Snell: sin(th_t) / c2 = sin(th_i) / c1, unit length, coplanar, other side
            assert np.linalg.norm(wt) == pytest.approx(1.0, abs=1e-14)
            sin_t = np.linalg.norm(np.cross(wt, n))
            assert sin_t / c2 == pytest.approx(math.sin(th) / c1, rel=1e-10, abs=1e-16)
            assert np.dot(np.cross(w, n), wt) == pytest.approx(0.0, abs=1e-14)
            assert np.sign(np.dot(wt, n)) == np.sign(np.dot(w, n))


def test_normal_incidence_closed_form():
    """Pressure reflection (Z2 - Z1)/(Z2 + Z1) and transmission 2 Z2/(Z2 + Z1)."""
    for Z1, Z2 in [(1.48, 1.63), (1.63, 1.48), (1.3, 1.8)]:
        coef, wr, wt = oracle.interface([0, 0, 1.0], [0, 0, 1.0], 1500, Z1, 1520, Z2)
        assert coef[0] == pytest.approx((Z2 - Z1) / (Z2 + Z1), rel=1e-14)
        assert coef[1] == pytest.approx(2 * Z2 / (Z2 + Z1), rel=1e-14)
        assert np.allclose(wr, [0, 0, -1.0]) and np.allclose(wt, [0, 0, 1.0])
    # round trip through an interface: A_t A_t' = 1 - R_E at normal incidence
    a = oracle.interface([0, 0, 1.0], [0, 0, 1.0], 1480, 1.48, 1540, 1.63)[0]
    b = oracle.interface([0, 0, -1.0], [0, 0, 1.0], 1540, 1.63, 1480, 1.48)[0]
    assert a[1] * b[1] == pytest.approx(1.0 - a[2], rel=1e-14)


def test_total_internal_reflection_at_critical_angle():
    c1, c2 = 1480.0, 1540.0
    crit = math.asin(c1 / c2)
    assert math.degrees(crit) == pytest.approx(73.95, abs=0.01)
    n = np.array([0, 0, 1.0])
    for th, expect_tir in [(crit - 1e-9, 0.0), (crit + 1e-9, 1.0), (math.radians(85), 1.0)]:
        w = np.array([math.sin(th), 0, math.cos(th)])
        coef, wr, wt = oracle.interface(w, n, c1, 1.48, c2, 1.63)
        assert coef[3] == expect_tir
        if expect_tir:
            assert coef[0] == 1.0 and coef[2] == 1.0 and coef[1] == 0.0


def test_cosine_lobe_distribution():
    """Cosine-weighted hemisphere: unit vectors on the normal's side with
    E[cos] = 2/3 and E[cos^2] = 1/2, tangential mean zero."""
    rng = np.random.default_rng(1)
    for n in ([0, 0, 1.0], [0, 0, -1.0], [0.6, 0.0, -0.8], [0.1, 0.7, 0.7071]):
        n = np.array(n) / np.linalg.norm(n)
        d = np.array([oracle.cosine_dir(n, *rng.random(2)) for _ in range(20000)])
        assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
        c = d @ n
        assert c.min() > 0
        assert c.mean() == pytest.approx(2 / 3, abs=0.01)
        assert (c ** 2).mean() == pytest.approx(0.5, abs=0.01)
        assert np.linalg.norm((d - np.outer(c, n)).mean(axis=0)) < 0.02


def test_receive_directivity_piecewise():
    """Eq. cutoff with alpha_m = 20 deg, alpha_c = 60 deg."""
    p = W.two_layer().probe
    for deg, expect in [(0, 1.0), (19.9, 1.0), (20.0, 1.0), (40.0, 0.5), (50.0, 0.25),
                        (60.0, 0.0), (75.0, 0.0), (120.0, 0.0)]:
        assert oracle.directivity(p, math.cos(math.radians(deg))) == pytest.approx(expect, abs=1e-12)


def test_pulse_envelope_fwhm_matches_cycles():
    """Reading of Eq. axial_sig: the Gaussian envelope's FWHM is n_cycles / f0,
    and the taps stop at the first one whose envelope is at or below 1e-7. The envelope is recovered
    from the oracle's taps by dividing out the carrier."""
    for f0, nc, fs in [(5e6, 2.0, 40e6), (7.5e6, 2.0, 60e6), (3e6, 3.0, 50e6)]:
        m, s = oracle.pulse_taps(f0, nc, fs)
        t = m / fs
        carrier = np.sin(2 * math.pi * f0 * t)
        ok = np.abs(carrier) > 0.3
        env = s[ok] / carrier[ok]
        # log-envelope is -t^2 / sigma: fit sigma by least squares
        sigma = -np.sum(t[ok] ** 2 * t[ok] ** 2) / np.sum(t[ok] ** 2 * np.log(env))
        fwhm = 2 * math.sqrt(sigma * math.log(2))
        assert fwhm == pytest.approx(nc / f0, rel=1e-9)
        M = m[-1]
        # M is the first tap whose envelope is at or below 1e-7
        assert math.exp(-(M / fs) ** 2 / sigma) <= 1e-7 < math.exp(-((M - 1) / fs) ** 2 / sigma)
        assert np.allclose(s, -s[::-1], atol=1e-15)   # odd: sine carrier, even envelope
