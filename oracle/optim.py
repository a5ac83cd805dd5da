"""Inverse loop of the paper, plain numpy FP64 (TEST INFRASTRUCTURE ONLY, as
the rest of this package).

  param_map            Eq. clip01 then Eq. scale_phys
  unconstrained_grad   chain rule through Eq. scale_phys with Eq. clip_grad
  clip_norm            gradient clipping (the paper names it without a form;
                       reading: the global L2 norm over the optimised
                       variables is capped at max_norm)
  adam_update          Eq. adam with the standard bias corrections
  image_loss           Eq. weighted_l1_l2_loss and its gradient
  iteration            one micro-batched iteration (Algorithm opt, Eq.
                       microbatch_loss): per micro-batch render, loss,
                       adjoints down to dL/dh, dual-number transport
                       gradient; sum; Adam on the unconstrained variables

Pinned in tests/test_oracle_optim.py (closed forms, torch.optim.Adam,
finite differences); `iteration` is pinned by its parts.
"""
from __future__ import annotations

import numpy as np

from . import chain


def param_map(u, lo, hi):
    """theta = lo + clip(u, 0, 1) (hi - lo); lo == hi fixes the parameter."""
    u, lo, hi = (np.asarray(a, dtype=np.float64) for a in (u, lo, hi))
    return np.where(lo == hi, lo, lo + np.clip(u, 0.0, 1.0) * (hi - lo))


def unconstrained_grad(g_theta, u, lo, hi):
    """dL/du = dL/dtheta (hi - lo) inside (0, 1), zero at or beyond a bound
    (Eq. clip_grad) and for fixed parameters."""
    g_theta, u, lo, hi = (np.asarray(a, dtype=np.float64) for a in (g_theta, u, lo, hi))
    inside = (u > 0.0) & (u < 1.0) & (lo < hi)
    return np.where(inside, g_theta * (hi - lo), 0.0)


def clip_norm(g, max_norm):
    g = np.asarray(g, dtype=np.float64)
    n = float(np.sqrt(np.sum(g * g)))
    if max_norm > 0.0 and n > max_norm:
        return g * (max_norm / n)
    return g


def adam_update(u, m, v, g, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """Returns (u, m, v) after one step; step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return u - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def image_loss(B, B_ref, l1, l2):
    """L = (1/N) [l1 sum |d| + l2 sum d^2], d = B - B_ref, and dL/dB
    (sign(0) = 0)."""
    d = np.asarray(B, dtype=np.float64) - np.asarray(B_ref, dtype=np.float64)
    n = d.size
    L = float((l1 * np.abs(d).sum() + l2 * (d * d).sum()) / n)
    return L, (l1 * np.sign(d) + 2.0 * l2 * d) / n


def iteration(batches, refs, u, m, v, lo, hi, lr, step, l1=0.0, l2=1.0, beta1=0.9, beta2=0.999,
              eps=1e-8, max_norm=0.0, n_threads=0):
    """One optimisation iteration. `batches` is a list of (workload, ray_begin,
    ray_count); each workload carries the micro-batch's transmits. `refs[b]`
    is the reference B-mode image of micro-batch b. Returns (u, m, v, total
    loss, dL/dtheta)."""
    from . import trace as _trace
    theta = param_map(u, lo, hi)
    params = [j for j in range(theta.shape[0]) if lo[j] < hi[j]]
    g_theta = np.zeros(theta.shape[0])
    total = 0.0
    for (wl, rb, rc), B_ref in zip(batches, refs):
        out = chain.render(wl, theta=theta, ray_begin=rb, ray_count=rc, n_threads=n_threads)
        L, g_B = image_loss(out["B"], B_ref, l1, l2)
        total += L
        p = wl.probe
        g_I = chain.bmode_vjp(out["I"], g_B, wl.dr_db)
        g_A = chain.das_vjp(g_I, p, wl.grid, wl.angles, p.n_t)
        g_rf = chain.analytic_vjp(g_A)
        _, s = chain.pulse_taps(p.f0, p.n_cycles, p.fs)
        g_h = chain.pulse_vjp(g_rf, s)
        for c0 in range(0, len(params), 64):
            sel = params[c0:c0 + 64]
            tr = _trace(wl.scene, p, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                        wl.max_bounces, ray_begin=rb, ray_count=rc, theta=theta, g_h=g_h,
                        grad_params=sel, n_threads=n_threads)
            g_theta += tr.g_theta
    g_u = clip_norm(unconstrained_grad(g_theta, u, lo, hi), max_norm)
    u, m, v = adam_update(np.asarray(u, dtype=np.float64), m, v, g_u, np.asarray(lr, dtype=np.float64),
                          step, beta1, beta2, eps)
    return u, m, v, total, g_theta
