"""torch.autograd wrappers over the C-ABI (paper Sec. 3.2-3.3).

    theta --SimulateRF--> rf --Beamform--> iq --BMode--> bmode

Each Function's forward and backward is one call into the HIP library (the
backward calls are the vector-Jacobian products: us_simulate_rf_vjp replays
the rays from their Philox counters, us_beamform_vjp is the transposed DAS
gather, us_bmode_vjp the log/envelope adjoint). PyTorch only supplies device
memory, the current stream and the graph bookkeeping.

Frame (Renderer.render_frame) is the same chain as one Function: its forward
makes the three forward calls, its backward is one us_frame_vjp call, which
takes dL/dB to the parameters with the intermediate gradients in its
workspace (the analytic-signal and pulse adjoints fused into one kernel);
the gradient is bit for bit that of the three-Function chain. With
render_frame(theta, recorded=True) the forward keeps the path records and the
backward reads them (us_frame_vjp_recorded), the same gradient again.

Fixed ray realisations (common random numbers): the seed and ray range are
attributes of the Renderer, constants of the differentiation.

Acquisition parameters: SimulateRF and Beamform also take an optional vector
acq = (steering angle of each transmit [rad], c_ref [m/s], pitch [m], f0 [Hz])
(Renderer.acquisition() gives the current one). Passed with requires_grad, it
receives the transport's gradient (us_simulate_rf_vjp_acq: emission, element
centres, pulse and the f0-scaled attenuation) and the image chain's
(us_beamform_acq_vjp: the delays of Eq. das, which do not depend on f0). A
changed c_ref, pitch or f0 uploads a new probe; the element width stays.
"""
from __future__ import annotations

import dataclasses
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

    # -- acquisition parameters
    def acquisition(self) -> torch.Tensor:
        """(steering angle of each transmit, c_ref, pitch, f0) as float64 [n_tx + 3]."""
        return torch.tensor(self._acquisition_host(), dtype=torch.float64, device=self.ctx.torch_device)

    def _acquisition_host(self) -> np.ndarray:
        p = self.wl.probe
        return np.concatenate([np.asarray(self.wl.angles, dtype=np.float64), [p.c_ref, p.pitch, p.f0]])

    def set_acquisition(self, acq) -> None:
        """Use these acquisition parameters from now on (uploads a new probe when
        c_ref, pitch or f0 change)."""
        a = acq.detach().to("cpu", torch.float64).numpy() if isinstance(acq, torch.Tensor) \
            else np.asarray(acq, dtype=np.float64)
        n = self.wl.n_tx
        if a.shape != (n + 3,):
            raise ValueError(f"acq must hold {n + 3} values (n_tx angles, c_ref, pitch, f0)")
        p = self.wl.probe
        q = dataclasses.replace(p, c_ref=float(a[n]), pitch=float(a[n + 1]), f0=float(a[n + 2]))
        if (q.c_ref, q.pitch, q.f0) != (p.c_ref, p.pitch, p.f0):
            self.probe = L.Probe(self.ctx, q)
        self.wl = self.wl.replace(angles=a[:n].copy(), probe=q)

    # -- the three differentiable stages
    def simulate_rf(self, theta: torch.Tensor, acq: Optional[torch.Tensor] = None) -> torch.Tensor:
        return SimulateRF.apply(theta, acq, self)

    def beamform(self, rf: torch.Tensor, acq: Optional[torch.Tensor] = None) -> torch.Tensor:
        return Beamform.apply(rf, acq, self)

    def bmode(self, iq: torch.Tensor) -> torch.Tensor:
        return BMode.apply(iq, self)

    def render(self, theta: Optional[torch.Tensor] = None, acq: Optional[torch.Tensor] = None) -> torch.Tensor:
        theta = self.theta0 if theta is None else theta
        return self.bmode(self.beamform(self.simulate_rf(theta, acq), acq))

    def render_frame(self, theta: Optional[torch.Tensor] = None, recorded: bool = False) -> torch.Tensor:
        """theta -> B-mode as one Function whose backward is us_frame_vjp. With
        `recorded`, the forward keeps the path records (device memory for the
        whole frame, one workspace per Renderer) and the backward reads them
        (us_frame_vjp_recorded, the same gradient bit for bit); a backward
        whose records were overwritten or whose parameters changed since
        traces the paths again."""
        theta = self.theta0 if theta is None else theta
        return Frame.apply(theta, self, recorded)

    def record_workspace(self) -> torch.Tensor:
        if getattr(self, "_ws_record", None) is None:
            wl = self.wl
            n = L.us_recorded_workspace_size(self.scene, self.probe, wl.n_tx, self.ray_count, wl.max_bounces)
            if n == 0:
                raise ValueError("a recorded frame takes at most 64 transmits and at least one ray")
            self._ws_record = L._workspace(n, self.ctx.torch_device)
        return self._ws_record

    def frame_workspace(self) -> torch.Tensor:
        if getattr(self, "_ws_frame", None) is None:
            wl = self.wl
            self._ws_frame = L._workspace(L.us_frame_vjp_workspace_size(
                self.scene, self.probe, wl.grid, wl.n_tx, self.ray_count, wl.max_bounces), self.ctx.torch_device)
        return self._ws_frame


class SimulateRF(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta: torch.Tensor, acq: Optional[torch.Tensor], r: Renderer):
        theta = theta.detach().to(torch.float64).contiguous()
        r.scene.set_params(theta)
        if acq is not None:
            r.set_acquisition(acq)
        fctx.acq = r._acquisition_host()
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
        r.scene.set_params(theta)           # the parameters this forward ran with
        r.set_acquisition(fctx.acq)
        wl = r.wl
        g_acq = None
        if fctx.needs_input_grad[1]:
            g_acq = torch.zeros(wl.n_tx + 3, dtype=torch.float64, device=r.ctx.torch_device)
        g_theta = L.us_simulate_rf_vjp(r.ctx, r.scene, r.probe, wl.angles, wl.tx_ids, wl.seed,
                                       wl.rays_per_elem, wl.max_bounces,
                                       g_rf.to(torch.float32).contiguous(),
                                       ray_begin=r.ray_begin, ray_count=r.ray_count,
                                       workspace=r.ws_replay, g_acq=g_acq)
        return g_theta, g_acq, None


class Beamform(torch.autograd.Function):
    @staticmethod
    def forward(fctx, rf: torch.Tensor, acq: Optional[torch.Tensor], r: Renderer):
        if acq is not None:
            r.set_acquisition(acq)
        fctx.acq = r._acquisition_host()
        wl = r.wl
        rf = rf.detach().to(torch.float32).contiguous()
        iq = L.us_beamform(r.ctx, r.probe, wl.grid, wl.angles, wl.tx_ids, rf, workspace=r.ws_beam)
        fctx.r = r
        fctx.save_for_backward(rf)
        return iq

    @staticmethod
    def backward(fctx, g_iq: torch.Tensor):
        r = fctx.r
        (rf,) = fctx.saved_tensors
        r.set_acquisition(fctx.acq)
        wl = r.wl
        g_iq = g_iq.to(torch.float32).contiguous()
        g_rf = L.us_beamform_vjp(r.ctx, r.probe, wl.grid, wl.angles, wl.tx_ids, g_iq,
                                 workspace=r.ws_beam_vjp)
        g_acq = None
        if fctx.needs_input_grad[1]:
            g = L.us_beamform_acq_vjp(r.ctx, r.probe, wl.grid, wl.angles, wl.tx_ids, rf, g_iq)
            g_acq = torch.cat([g, g.new_zeros(1)])   # the delays do not depend on f0
        return g_rf, g_acq, None


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


class Frame(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta: torch.Tensor, r: Renderer, recorded: bool = False):
        theta = theta.detach().to(torch.float64).contiguous()
        r.scene.set_params(theta)
        wl = r.wl
        fctx.rec = None
        if recorded:
            # the Renderer's one record workspace: a later recorded forward overwrites it
            r._record_serial = getattr(r, "_record_serial", 0) + 1
            fctx.serial = r._record_serial
            rf, fctx.rec = L.us_simulate_rf_recorded(r.ctx, r.scene, r.probe, wl.angles, wl.tx_ids, wl.seed,
                                                     wl.rays_per_elem, wl.max_bounces, ray_begin=r.ray_begin,
                                                     ray_count=r.ray_count, workspace=r.record_workspace())
        else:
            rf = L.us_simulate_rf(r.ctx, r.scene, r.probe, wl.angles, wl.tx_ids, wl.seed,
                                  wl.rays_per_elem, wl.max_bounces, ray_begin=r.ray_begin,
                                  ray_count=r.ray_count, workspace=r.ws_trace)
        iq = L.us_beamform(r.ctx, r.probe, wl.grid, wl.angles, wl.tx_ids, rf, workspace=r.ws_beam)
        b = L.us_bmode(r.ctx, iq, wl.dr_db, workspace=r.ws_bmode)
        fctx.r = r
        fctx.save_for_backward(theta, iq)
        return b

    @staticmethod
    def backward(fctx, g_b: torch.Tensor):
        r = fctx.r
        theta, iq = fctx.saved_tensors
        wl = r.wl
        g_b = g_b.to(torch.float32).contiguous()
        if fctx.rec is not None and fctx.serial == r._record_serial:
            try:
                # the records hold while the scene keeps this forward's parameters
                g_theta = L.us_frame_vjp_recorded(r.ctx, fctx.rec, wl.grid, iq, g_b, wl.dr_db)
                return g_theta, None, None
            except L.USError as e:
                if e.code != L.US_EINVAL:
                    raise
        r.scene.set_params(theta)
        g_theta = L.us_frame_vjp(r.ctx, r.scene, r.probe, wl.grid, wl.angles, wl.tx_ids, wl.seed,
                                 wl.rays_per_elem, wl.max_bounces, iq, g_b,
                                 wl.dr_db, ray_begin=r.ray_begin, ray_count=r.ray_count,
                                 workspace=r.frame_workspace())
        return g_theta, None, None


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
