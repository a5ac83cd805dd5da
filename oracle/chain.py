"""FP64 image-formation chain and its adjoints (numpy), for the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Forward (paper Sec. 2.3.4 and Sec. 3.3):
  h   --pulse-->  rf   (Eq. axial_sig, a linear filter of the deposited impulses)
  rf  --analytic-> A   (demodulation: analytic signal along time, FFT method)
  A   --DAS-->     I   (Eq. das: plane-wave delay-and-sum, linear interpolation,
                        coherent over transmits)
  I   --bmode-->   B   (envelope |I|, log compression normalised by the frame
                        maximum, dynamic-range clip)
Backward: the adjoint of each step (Eq. das_adjoint for DAS; the envelope/log
adjoint is derived here, as the paper refers to it without printing it).

Readings (where the paper is silent):
  * pulse width: sigma chosen so that the Gaussian envelope's full width at
    half maximum equals n_cycles / f0; taps |m| <= M, M the first whose
    envelope is at or below 1e-7;
  * pulse filter: linear (zero-padded) convolution, kept to [0, n_t);
  * analytic signal per channel along time (the Hilbert transform commutes
    with the per-channel delays), FFT multiplier 1, 2, ..., 2, 1, 0, ... 0;
  * DAS: unit apodisation; samples outside [0, n_t) read as zero; transmit
    delay (x sin th + z cos th)/c_ref, receive delay |x - x_e|/c_ref;
  * B-mode: B = max(20 log10(|I| / max|I|), -DR); pixels at the clip get no
    gradient; the normalising maximum is the first pixel (row-major) of
    largest |I|.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

__all__ = ["pulse_taps", "pulse", "pulse_vjp", "analytic", "analytic_vjp", "das_index", "das",
           "das_vjp", "das_acq_vjp", "bmode", "bmode_vjp", "mse", "mse_grad", "simulate_rf", "render",
           "grad_theta", "analytic_multiplier"]

LOG_SCALE = 20.0 / math.log(10.0)


# ---------------------------------------------------------------- pulse (Eq. axial_sig)
def pulse_taps(f0: float, n_cycles: float, fs: float):
    """Taps s[m] = s(m / fs), m = -M..M, of s(t) = sin(2 pi f0 t) exp(-t^2 / sigma)."""
    sigma = (n_cycles / (2.0 * f0)) ** 2 / math.log(2.0)
    M = int(math.ceil(fs * math.sqrt(sigma * math.log(1e7))))
    m = np.arange(-M, M + 1)
    t = m / fs
    return m, np.sin(2.0 * math.pi * f0 * t) * np.exp(-t * t / sigma)


def pulse(h: np.ndarray, s: np.ndarray) -> np.ndarray:
    """rf[..., k] = sum_m h[..., k - m] s[m], h read as zero outside [0, n_t)."""
    M = (s.shape[0] - 1) // 2
    n = h.shape[-1]
    rf = np.zeros_like(h)
    for i, m in enumerate(range(-M, M + 1)):
        if m >= 0:
            rf[..., m:] += s[i] * h[..., :n - m]
        else:
            rf[..., :n + m] += s[i] * h[..., -m:]
    return rf


def pulse_vjp(g_rf: np.ndarray, s: np.ndarray) -> np.ndarray:
    """g_h[..., j] = sum_m g_rf[..., j + m] s[m] (adjoint of `pulse`)."""
    M = (s.shape[0] - 1) // 2
    n = g_rf.shape[-1]
    g = np.zeros_like(g_rf)
    for i, m in enumerate(range(-M, M + 1)):
        if m >= 0:
            g[..., :n - m] += s[i] * g_rf[..., m:]
        else:
            g[..., -m:] += s[i] * g_rf[..., :n + m]
    return g


# ---------------------------------------------------------------- analytic signal
def analytic_multiplier(n: int) -> np.ndarray:
    H = np.zeros(n)
    H[0] = 1.0
    if n % 2 == 0:
        H[1:n // 2] = 2.0
        H[n // 2] = 1.0
    else:
        H[1:(n + 1) // 2] = 2.0
    return H


def analytic(rf: np.ndarray) -> np.ndarray:
    """A = IFFT(H * FFT(rf)) along the last axis; Re(A) = rf."""
    n = rf.shape[-1]
    return np.fft.ifft(np.fft.fft(rf, axis=-1) * analytic_multiplier(n), axis=-1)


def analytic_vjp(g_A: np.ndarray) -> np.ndarray:
    """Adjoint under the real inner product Re<g, A>: the map is F^-1 diag(H) F
    with a real multiplier, hence self-adjoint, so g_rf = Re(T g_A)."""
    n = g_A.shape[-1]
    return np.real(np.fft.ifft(np.fft.fft(g_A, axis=-1) * analytic_multiplier(n), axis=-1))


# ---------------------------------------------------------------- delay-and-sum (Eq. das)
def _pixels(grid):
    x = grid.x0 + np.arange(grid.n_x) * grid.dx
    z = grid.z0 + np.arange(grid.n_z) * grid.dz
    return np.meshgrid(x, z, indexing="ij")


def das_index(probe, grid, angle: float, e: int) -> np.ndarray:
    """Fractional sample index fs * tau_e(x, z) for one transmit angle and element."""
    X, Z = _pixels(grid)
    xe = (e - 0.5 * (probe.n_elem - 1)) * probe.pitch
    tau = (X * math.sin(angle) + Z * math.cos(angle)) / probe.c_ref \
        + np.sqrt((X - xe) ** 2 + Z ** 2) / probe.c_ref
    return tau * probe.fs


def das(A: np.ndarray, probe, grid, angles) -> np.ndarray:
    """I(x, z) = sum_tx sum_e lerp(A[tx, e], fs tau) (unit weights)."""
    n_t = A.shape[-1]
    I = np.zeros((grid.n_x, grid.n_z), dtype=np.complex128)
    for i, th in enumerate(angles):
        for e in range(probe.n_elem):
            k = das_index(probe, grid, th, e)
            k0 = np.floor(k).astype(np.int64)
            f = k - k0
            row = A[i, e]
            v0 = np.where((k0 >= 0) & (k0 < n_t), row[np.clip(k0, 0, n_t - 1)], 0.0)
            v1 = np.where((k0 + 1 >= 0) & (k0 + 1 < n_t), row[np.clip(k0 + 1, 0, n_t - 1)], 0.0)
            I += (1.0 - f) * v0 + f * v1
    return I


def das_vjp(g_I: np.ndarray, probe, grid, angles, n_t: int) -> np.ndarray:
    """Eq. das_adjoint: scatter the image gradient back onto the two samples
    each pixel interpolated from, with the same weights."""
    g_A = np.zeros((len(angles), probe.n_elem, n_t), dtype=np.complex128)
    gr = g_I.reshape(-1)
    for i, th in enumerate(angles):
        for e in range(probe.n_elem):
            k = das_index(probe, grid, th, e).reshape(-1)
            k0 = np.floor(k).astype(np.int64)
            f = k - k0
            for idx, wgt in ((k0, 1.0 - f), (k0 + 1, f)):
                ok = (idx >= 0) & (idx < n_t)
                g_A[i, e] += np.bincount(idx[ok], weights=(wgt[ok] * gr[ok].real), minlength=n_t) \
                    + 1j * np.bincount(idx[ok], weights=(wgt[ok] * gr[ok].imag), minlength=n_t)
    return g_A


def das_acq_vjp(A: np.ndarray, g_I: np.ndarray, probe, grid, angles):
    """Gradient of L = Re sum conj(g_I) I with respect to the acquisition
    parameters of Eq. das at fixed analytic signal A: each transmit's steering
    angle, the beamforming speed of sound c_ref and the element pitch.

    I depends on them only through the fractional sample index k = fs tau, and
    the linear interpolation lerp(A, k) has slope A[k0 + 1] - A[k0] in k on
    each sample interval, so dL/dk = Re(conj(g_I) (A[k0 + 1] - A[k0])). With
    k = fs ((x sin th + z cos th) + r_e) / c_ref, r_e = |(x, z) - (x_e, 0)| and
    x_e = (e - (N - 1)/2) pitch:
        dk/dth    = fs (x cos th - z sin th) / c_ref
        dk/dc_ref = -k / c_ref
        dk/dpitch = -fs (x - x_e) (e - (N - 1)/2) / (r_e c_ref).
    Returns (g_angles [n_tx], g_c_ref, g_pitch)."""
    n_t = A.shape[-1]
    X, Z = _pixels(grid)
    half = 0.5 * (probe.n_elem - 1)
    g_th = np.zeros(len(angles))
    g_c = 0.0
    g_p = 0.0
    for i, th in enumerate(angles):
        dk_dth = probe.fs * (X * math.cos(th) - Z * math.sin(th)) / probe.c_ref
        for e in range(probe.n_elem):
            k = das_index(probe, grid, th, e)
            k0 = np.floor(k).astype(np.int64)
            row = A[i, e]
            v0 = np.where((k0 >= 0) & (k0 < n_t), row[np.clip(k0, 0, n_t - 1)], 0.0)
            v1 = np.where((k0 + 1 >= 0) & (k0 + 1 < n_t), row[np.clip(k0 + 1, 0, n_t - 1)], 0.0)
            dL_dk = (np.conj(g_I) * (v1 - v0)).real
            xe = (e - half) * probe.pitch
            r = np.sqrt((X - xe) ** 2 + Z ** 2)
            g_th[i] += float(np.sum(dL_dk * dk_dth))
            g_c += float(np.sum(dL_dk * (-k / probe.c_ref)))
            g_p += float(np.sum(dL_dk * (-probe.fs * (X - xe) * (e - half) / (r * probe.c_ref))))
    return g_th, g_c, g_p


# ---------------------------------------------------------------- B-mode
def bmode(I: np.ndarray, dr_db: float) -> np.ndarray:
    env = np.abs(I)
    m = env.max()
    with np.errstate(divide="ignore"):
        v = LOG_SCALE * np.log(np.where(env > 0, env, 1.0) / m)
    v = np.where(env > 0, v, -dr_db)
    return np.maximum(v, -dr_db)


def bmode_vjp(I: np.ndarray, g_B: np.ndarray, dr_db: float) -> np.ndarray:
    """Complex gradient g = dL/dRe I + i dL/dIm I of L(B(I)).

    For an unclipped pixel, B = (20/ln 10)(log|I| - log m) gives
    dB/dI = (20/ln 10) I/|I|^2 plus, through m = |I_am| at the arg-max pixel,
    -(20/ln 10) I_am / m^2 for every unclipped pixel."""
    env = np.abs(I)
    am = int(np.argmax(env.reshape(-1)))
    m = env.reshape(-1)[am]
    with np.errstate(divide="ignore", invalid="ignore"):
        v = LOG_SCALE * np.log(np.where(env > 0, env, 1.0) / m)
    unclipped = (env > 0) & (v > -dr_db)
    g = np.zeros_like(I)
    g[unclipped] = g_B[unclipped] * LOG_SCALE * I[unclipped] / env[unclipped] ** 2
    S = g_B[unclipped].sum()
    g.reshape(-1)[am] += -LOG_SCALE * S * I.reshape(-1)[am] / m ** 2
    return g


def mse(B: np.ndarray, B_ref: np.ndarray) -> float:
    return float(np.mean((B - B_ref) ** 2))


def mse_grad(B: np.ndarray, B_ref: np.ndarray) -> np.ndarray:
    return 2.0 * (B - B_ref) / B.size


# ---------------------------------------------------------------- whole chain
def simulate_rf(wl, theta: Optional[np.ndarray] = None, ray_begin: int = 0,
                ray_count: Optional[int] = None, nee_mode: int = 0, want_hashes: bool = False,
                n_threads: int = 0, probs=None, record_probs: bool = False):
    """Transport + splat + pulse for a workload-like object (attributes scene,
    probe, angles, tx_ids, seed, rays_per_elem, max_bounces). Returns (rf, h, trace)."""
    from . import trace as _trace
    p = wl.probe
    tr = _trace(wl.scene, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                ray_begin=ray_begin, ray_count=ray_count, theta=theta, nee_mode=nee_mode,
                want_hashes=want_hashes, n_threads=n_threads, probs=probs,
                record_probs=record_probs)
    h = tr.splat(len(wl.angles), p.n_elem, p.n_t, p.fs)
    _, s = pulse_taps(p.f0, p.n_cycles, p.fs)
    return pulse(h, s), h, tr


def render(wl, theta: Optional[np.ndarray] = None, **kw):
    rf, h, tr = simulate_rf(wl, theta=theta, **kw)
    A = analytic(rf)
    I = das(A, wl.probe, wl.grid, wl.angles)
    B = bmode(I, wl.dr_db)
    return dict(h=h, rf=rf, A=A, I=I, B=B, trace=tr)


def grad_theta(wl, B_ref: np.ndarray, theta: Optional[np.ndarray] = None,
               grad_params=None, ray_begin: int = 0, ray_count: Optional[int] = None,
               n_threads: int = 0):
    """MSE(B(theta), B_ref) and its gradient with respect to theta[grad_params]
    at fixed ray realisations (Sec. 3.2): image-chain adjoints in numpy, then
    the transport's dual-number derivatives contracted with dL/dh."""
    from . import trace as _trace
    out = render(wl, theta=theta, ray_begin=ray_begin, ray_count=ray_count, n_threads=n_threads)
    p = wl.probe
    g_B = mse_grad(out["B"], B_ref)
    g_I = bmode_vjp(out["I"], g_B, wl.dr_db)
    g_A = das_vjp(g_I, p, wl.grid, wl.angles, p.n_t)
    g_rf = analytic_vjp(g_A)
    _, s = pulse_taps(p.f0, p.n_cycles, p.fs)
    g_h = pulse_vjp(g_rf, s)
    th = wl.scene.theta() if theta is None else np.asarray(theta, dtype=np.float64)
    params = list(range(th.shape[0])) if grad_params is None else list(grad_params)
    g = np.zeros(th.shape[0])
    for c0 in range(0, len(params), 64):
        sel = params[c0:c0 + 64]
        tr = _trace(wl.scene, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                    wl.max_bounces, ray_begin=ray_begin, ray_count=ray_count, theta=th,
                    g_h=g_h, grad_params=sel, n_threads=n_threads)
        g += tr.g_theta
    out.update(loss=mse(out["B"], B_ref), g_theta=g, g_B=g_B, g_I=g_I, g_A=g_A, g_rf=g_rf, g_h=g_h)
    return out
