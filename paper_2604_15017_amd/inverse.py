"""Inverse loop of the paper on the GPU (Algorithm opt, Sec. "Optimization
procedure"): for every micro-batch (a subset of the transmits and a range of
rays, Sec. "Micro-batched acquisition", Eq. microbatch_loss) the forward
frame, the weighted L1 + L2 image loss against that micro-batch's reference
(Eq. weighted_l1_l2_loss) and the VJP chain down to dL/dtheta, accumulated
over the micro-batches; then one Adam step (Eq. adam) on the unconstrained
variables and the clip-and-scale map (Eq. clip01, Eq. scale_phys) back to the
scene, all through the C-ABI on one stream. The ray realisations stay fixed
across iterations (common random numbers)."""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L


@dataclasses.dataclass
class MicroBatch:
    tx: Sequence[int]                 # indices into the workload's transmits
    ray_begin: int = 0
    ray_count: Optional[int] = None   # None: every ray from ray_begin


def unconstrained_start(theta0, lo, hi):
    """u with lo + u (hi - lo) = theta0 (0 for fixed parameters)."""
    theta0, lo, hi = (np.asarray(a, dtype=np.float64) for a in (theta0, lo, hi))
    span = np.where(hi > lo, hi - lo, 1.0)
    return np.where(hi > lo, (theta0 - lo) / span, 0.0)


class InverseLoop:
    """Optimises the scene parameters theta = lo + clip(u, 0, 1) (hi - lo);
    parameters with lo == hi stay fixed. `lr` holds one learning rate per
    parameter (groups are runs of equal values). With `recorded`, each
    micro-batch's forward keeps its path records and the backward reads them
    (us_simulate_rf_recorded, us_simulate_rf_vjp_recorded: the same gradient
    bit for bit, device memory for the records of the largest micro-batch)."""

    def __init__(self, ctx, wl, lo, hi, lr, u0, batches: List[MicroBatch], refs=None, target=None,
                 lambda1: float = 0.0, lambda2: float = 1.0, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8, max_norm: float = 0.0, stream=None,
                 recorded: bool = False):
        import torch
        self.ctx, self.wl, self.batches = ctx, wl, batches
        self.l1, self.l2, self.b1, self.b2, self.eps, self.max_norm = (lambda1, lambda2, beta1, beta2,
                                                                       eps, max_norm)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        dev = ctx.torch_device
        f64 = dict(dtype=torch.float64, device=dev)
        self.lo, self.hi, self.lr = (torch.tensor(np.asarray(a, dtype=np.float64), **f64) for a in (lo, hi, lr))
        self.u = torch.tensor(np.asarray(u0, dtype=np.float64), **f64)
        self.m, self.v = torch.zeros_like(self.u), torch.zeros_like(self.u)
        self.g_theta = torch.zeros_like(self.u)
        self.theta = L.us_param_map(ctx, self.u, self.lo, self.hi, stream=self.stream)
        self.scene = L.Scene(ctx, wl.scene)
        self.scene.set_params(self.theta, stream=self.stream)
        self.probe = L.Probe(ctx, wl.probe)
        self.step_count = 0
        p, g = wl.probe, wl.grid
        self._views = []
        for b in batches:
            tx = np.asarray(b.tx, dtype=np.int64)
            count = wl.rays_per_tx - b.ray_begin if b.ray_count is None else b.ray_count
            self._views.append((wl.angles[tx], wl.tx_ids[tx], b.ray_begin, count))
        n_tx = max(len(v[0]) for v in self._views)
        count = max(v[3] for v in self._views)
        self.rf = torch.empty((n_tx, p.n_elem, p.n_t), dtype=torch.float32, device=dev)
        self.iq = torch.empty((g.n_x, g.n_z, 2), dtype=torch.float32, device=dev)
        self.bm = torch.empty((g.n_x, g.n_z), dtype=torch.float32, device=dev)
        self.g_b, self.g_iq = torch.empty_like(self.bm), torch.empty_like(self.iq)
        self.g_rf = torch.empty_like(self.rf)
        self.loss = torch.zeros(len(batches), dtype=torch.float64, device=dev)
        lib = L.load()
        self.ws_t = L._workspace(L.us_simulate_rf_workspace_size(self.scene, self.probe, n_tx, count,
                                                                 wl.max_bounces), dev)
        self.ws_b = L._workspace(lib.us_beamform_workspace_size(self.probe.handle, n_tx), dev)
        self.ws_m = L._workspace(lib.us_bmode_workspace_size(g.n_px), dev)
        self.ws_l = L._workspace(lib.us_image_loss_workspace_size(g.n_px), dev)
        self.recorded = recorded
        if recorded:
            self.ws_rec = L._workspace(L.us_recorded_workspace_size(self.scene, self.probe, n_tx, count,
                                                                    wl.max_bounces), dev)
        else:
            self.ws_r = L._workspace(L.us_simulate_rf_vjp_workspace_size(self.scene, self.probe, n_tx, count,
                                                                         wl.max_bounces), dev)
        if refs is None:
            if target is None:
                raise ValueError("give the reference images or a target scene")
            refs = self.render_all(target)
        self.refs = refs

    def _frame(self, scene, b, record=False):
        wl, (ang, ids, rb, rc) = self.wl, self._views[b]
        rf = self.rf[:len(ang)]
        rec = None
        if record:
            _, rec = L.us_simulate_rf_recorded(self.ctx, scene, self.probe, ang, ids, wl.seed, wl.rays_per_elem,
                                               wl.max_bounces, ray_begin=rb, ray_count=rc, rf=rf,
                                               workspace=self.ws_rec, stream=self.stream)
        else:
            L.us_simulate_rf(self.ctx, scene, self.probe, ang, ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                             ray_begin=rb, ray_count=rc, rf=rf, workspace=self.ws_t, stream=self.stream)
        L.us_beamform(self.ctx, self.probe, wl.grid, ang, ids, rf, iq=self.iq, workspace=self.ws_b,
                      stream=self.stream)
        L.us_bmode(self.ctx, self.iq, wl.dr_db, out=self.bm, workspace=self.ws_m, stream=self.stream)
        return rf, rec

    def render_all(self, scene_desc):
        """B-mode image of every micro-batch for a scene description."""
        sc = L.Scene(self.ctx, scene_desc)
        out = []
        for b in range(len(self.batches)):
            self._frame(sc, b)
            out.append(self.bm.clone())
        return out

    def iterate(self):
        """One iteration; returns the summed loss (float64 device tensor, at
        the parameters before the update)."""
        wl = self.wl
        self.g_theta.zero_()
        for b, (ang, ids, rb, rc) in enumerate(self._views):
            rf, rec = self._frame(self.scene, b, record=self.recorded)
            L.us_image_loss(self.ctx, self.bm, self.refs[b], self.l1, self.l2, loss=self.loss[b:b + 1],
                            g_bmode=self.g_b, workspace=self.ws_l, stream=self.stream)
            L.us_bmode_vjp(self.ctx, self.iq, self.g_b, wl.dr_db, g_iq=self.g_iq, workspace=self.ws_m,
                           stream=self.stream)
            g_rf = self.g_rf[:len(ang)]
            L.us_beamform_vjp(self.ctx, self.probe, wl.grid, ang, ids, self.g_iq, g_rf=g_rf,
                              workspace=self.ws_b, stream=self.stream)
            if rec is not None:
                L.us_simulate_rf_vjp_recorded(self.ctx, rec, g_rf, g_theta=self.g_theta, stream=self.stream)
            else:
                L.us_simulate_rf_vjp(self.ctx, self.scene, self.probe, ang, ids, wl.seed, wl.rays_per_elem,
                                     wl.max_bounces, g_rf, g_theta=self.g_theta, ray_begin=rb, ray_count=rc,
                                     workspace=self.ws_r, stream=self.stream)
        self.step_count += 1
        L.us_adam_step(self.ctx, self.u, self.m, self.v, self.g_theta, self.lo, self.hi, self.lr,
                       self.step_count, self.b1, self.b2, self.eps, self.max_norm, stream=self.stream)
        L.us_param_map(self.ctx, self.u, self.lo, self.hi, theta=self.theta, stream=self.stream)
        self.scene.set_params(self.theta, stream=self.stream)
        return self.loss.sum()
