"""torch.autograd wrappers over the C-ABI (paper Sec. 3.2-3.3).

    theta --SimulateRF--> rf --Beamform--> iq --BMode--> bmode

Each Function's forward and backward is one call into the HIP library (the
backward calls are the vector-Jacobian products: us_simulate_rf_vjp replays
the rays from their Philox counters, us_beamform_vjp is the transposed DAS
gather, us_bmode_vjp the log/envelope adjoint). PyTorch only supplies device
memory, the current stream and the graph bookkeeping.

Fixed ray realisations (common random numbers): the seed and ray range are
attributes of the Renderer, constants of the differentiation.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import _lib as L


class Renderer:
    """Resident scene, probe and workspaces for one workload."""

    def __init__(self, wl, ctx: Optional[L.Context] = None, ray_begin: int = 0,
                 ray_count: Optional[int] = None):
        self.wl = wl
        self.ctx = ctx or L.Context(0)
        self.scene = L.Scene(self.ctx, wl.scene)
        self.probe = L.Probe(self.ctx, wl.probe)
        self.ray_begin = ray_begin
        self.ray_count = wl.rays_per_tx - ray_begin if ray_count is None else ray_count
        dev = self.ctx.torch_device
        n_tx, p = wl.n_tx, wl.probe
        self.ws_trace = L._workspace(L.us_simulate_rf_workspace_size(
            self.scene, self.probe, n_tx, self.ray_count, wl.max_bounces), dev)
        self.ws_replay = L._workspace(L.us_simulate_rf_vjp_workspace_size(
            self.scene, self.probe, n_tx, self.ray_count, wl.max_bounces), dev)
        self.ws_beam = L._workspace(L.load().us_beamform_workspace_size(self.probe.handle, n_tx), dev)
        self.ws_beam_vjp = L._workspace(L.load().us_beamform_vjp_workspace_size(self.probe.handle, n_tx), dev)
        self.ws_bmode = L._workspace(L.load().us_bmode_workspace_size(wl.grid.n_px), dev)
        self.theta0 = torch.tensor(wl.scene.theta(), dtype=torch.float64, device=dev)

    # -- the three differentiable stages
    def simulate_rf(self, theta: torch.Tensor) -> torch.Tensor:
        return SimulateRF.apply(theta, self)

    def beamform(self, rf: torch.Tensor) -> torch.Tensor:
        return Beamform.apply(rf, self)

    def bmode(self, iq: torch.Tensor) -> torch.Tensor:
        return BMode.apply(iq, self)

    def render(self, theta: Optional[torch.Tensor] = None) -> torch.Tensor:
        theta = self.theta0 if theta is None else theta
        return self.bmode(self.beamform(self.simulate_rf(theta)))


class SimulateRF(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta: torch.Tensor, r: Renderer):
        theta = theta.detach().to(torch.float64).contiguous()
        r.scene.set_params(theta)
        wl = r.wl
        rf = L.us_simulate_rf(r.ctx, r.scene, r.probe, wl.angles, wl.tx_ids, wl.seed,
                              wl.rays_per_elem, wl.max_bounces, ray_begin=r.ray_begin,
                              ray_count=r.ray_count, workspace=r.ws_trace)
        fctx.r = r
        fctx.save_for_backward(theta)
        return rf

    @staticmethod
    def backward(fctx, g_rf: torch.Tensor):
        r = fctx.r
        (theta,) = fctx.saved_tensors
        wl = r.wl
        r.scene.set_params(theta)           # the parameters this forward ran with
        g_theta = L.us_simulate_rf_vjp(r.ctx, r.scene, r.probe, wl.angles, wl.tx_ids, wl.seed,
                                       wl.rays_per_elem, wl.max_bounces,
                                       g_rf.to(torch.float32).contiguous(),
                                       ray_begin=r.ray_begin, ray_count=r.ray_count,
                                       workspace=r.ws_replay)
        return g_theta, None


class Beamform(torch.autograd.Function):
    @staticmethod
    def forward(fctx, rf: torch.Tensor, r: Renderer):
        wl = r.wl
        iq = L.us_beamform(r.ctx, r.probe, wl.grid, wl.angles, wl.tx_ids,
                           rf.detach().to(torch.float32).contiguous(), workspace=r.ws_beam)
        fctx.r = r
        return iq

    @staticmethod
    def backward(fctx, g_iq: torch.Tensor):
        r = fctx.r
        wl = r.wl
        g_rf = L.us_beamform_vjp(r.ctx, r.probe, wl.grid, wl.angles, wl.tx_ids,
                                 g_iq.to(torch.float32).contiguous(), workspace=r.ws_beam_vjp)
        return g_rf, None


class BMode(torch.autograd.Function):
    @staticmethod
    def forward(fctx, iq: torch.Tensor, r: Renderer):
        iq = iq.detach().to(torch.float32).contiguous()
        b = L.us_bmode(r.ctx, iq, r.wl.dr_db, workspace=r.ws_bmode)
        fctx.r = r
        fctx.save_for_backward(iq)
        return b

    @staticmethod
    def backward(fctx, g_b: torch.Tensor):
        r = fctx.r
        (iq,) = fctx.saved_tensors
        g_iq = L.us_bmode_vjp(r.ctx, iq, g_b.to(torch.float32).contiguous(), r.wl.dr_db,
                              workspace=r.ws_bmode)
        return g_iq, None


class ImageLoss(torch.autograd.Function):
    """Weighted L1 + L2 image loss (Eq. weighted_l1_l2_loss) by us_image_loss."""

    @staticmethod
    def forward(fctx, b: torch.Tensor, b_ref: torch.Tensor, r: Renderer, l1: float, l2: float):
        loss, g = L.us_image_loss(r.ctx, b.detach().contiguous(), b_ref.detach().to(torch.float32).contiguous(),
                                  l1, l2)
        fctx.save_for_backward(g)
        return loss[0]

    @staticmethod
    def backward(fctx, g_out: torch.Tensor):
        (g,) = fctx.saved_tensors
        return g * g_out.to(g.dtype), None, None, None, None


def mse(b: torch.Tensor, b_ref: torch.Tensor, r: Renderer) -> torch.Tensor:
    """Mean squared dB difference (the forward+backward workload's loss)."""
    return ImageLoss.apply(b, b_ref, r, 0.0, 1.0)


def l1_l2(b: torch.Tensor, b_ref: torch.Tensor, r: Renderer, l1: float, l2: float) -> torch.Tensor:
    return ImageLoss.apply(b, b_ref, r, l1, l2)
