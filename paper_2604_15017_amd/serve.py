"""Serving loop: continuous batching of simulate and simulate+gradient requests.

A persistent loop (one host thread issues all GPU work) keeps scenes and
probes resident, admits requests first-in first-out as soon as an execution
slot and enough device memory are free, runs every admitted request on its
slot's own HIP stream so that requests overlap on the device, and records per
request the arrival, admission and completion times.

Gradient requests take the whole backward in one call (us_frame_vjp). One
whose path records fit RECORD_MAX_BYTES is rendered by the recorded forward
and its backward reads those records instead of tracing the paths again
(us_frame_vjp_recorded); the result is the same bits either way.

Admission accounting: a request reserves the bytes of everything it
allocates (RF, analytic-signal and queue workspaces, image buffers, and for
gradient requests the adjoint buffers and the replay or record workspace), as
reported by the library's *_workspace_size calls; a request larger than the
cap is rejected with an error result and the loop goes on.

The executor is pluggable: GpuExecutor calls the C-ABI; tests of admission,
ordering, latency accounting and failure handling use a host-only executor.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Dict, List, Optional

import numpy as np


# The replay workspace of a gradient request is sized for chunks of this many
# rays (some 5 GB at twelve interactions): a whole-frame chunk would save a few
# launches but reserve up to 20 GB per request in flight.
REPLAY_CHUNK_RAYS = 1 << 21

# A gradient request records its paths (about 3 KB of device memory per ray
# at twelve interactions) when the records take at most this many bytes:
# some 2.8 million rays.
RECORD_MAX_BYTES = 8 << 30


@dataclasses.dataclass
class Request:
    rid: int
    workload: object                  # workloads.Workload
    want_grad: bool = False
    # reference image of the gradient's loss: a float32 device tensor
    # [n_x][n_z] (build_requests makes it one), or a host array that launch()
    # stages through pinned memory without blocking
    b_ref: Optional[object] = None
    arrival: float = 0.0


@dataclasses.dataclass
class Result:
    rid: int
    ok: bool
    error: str = ""
    bmode: Optional[object] = None    # device tensor [n_x][n_z]
    loss: Optional[float] = None
    g_theta: Optional[object] = None  # device tensor [n_params]
    segments: int = 0
    bytes_reserved: int = 0
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Server:
    """First-in first-out admission into `n_slots` concurrent slots under a
    memory cap; completions are polled, slots and memory are released at once."""

    def __init__(self, executor, n_slots: int = 8, mem_cap_bytes: int = 200 * 10**9,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.n_slots = n_slots
        self.cap = int(mem_cap_bytes)
        self.clock = clock
        self.pending: "collections.deque[Request]" = collections.deque()
        self.lock = threading.Lock()
        self.free_slots = list(range(n_slots))
        self.inflight: List[tuple] = []
        self.reserved = 0
        self.results: Dict[int, Result] = {}
        self.max_reserved = 0
        self.max_concurrent = 0

    def submit(self, req: Request):
        req.arrival = self.clock()
        with self.lock:
            self.pending.append(req)

    def _admit(self):
        while True:
            with self.lock:
                if not self.pending:
                    return
                req = self.pending[0]
            need = self.ex.bytes_needed(req)
            if need > self.cap:
                with self.lock:
                    self.pending.popleft()
                self.results[req.rid] = Result(req.rid, False, f"request needs {need} bytes, cap {self.cap}",
                                               t_arrival=req.arrival, t_admit=self.clock(),
                                               t_done=self.clock())
                continue
            if not self.free_slots or self.reserved + need > self.cap:
                return
            with self.lock:
                self.pending.popleft()
            slot = self.free_slots.pop()
            t_admit = self.clock()
            try:
                handle = self.ex.launch(req, slot)
            except Exception as e:   # launch failure: report, release, continue
                self.free_slots.append(slot)
                self.results[req.rid] = Result(req.rid, False, f"{type(e).__name__}: {e}",
                                               t_arrival=req.arrival, t_admit=t_admit,
                                               t_done=self.clock())
                continue
            self.reserved += need
            self.max_reserved = max(self.max_reserved, self.reserved)
            self.inflight.append((req, slot, handle, need, t_admit))
            self.max_concurrent = max(self.max_concurrent, len(self.inflight))

    def _poll(self) -> bool:
        done_any = False
        still = []
        for req, slot, handle, need, t_admit in self.inflight:
            if self.ex.done(handle):
                res = self.ex.finish(req, handle)
                res.t_arrival, res.t_admit, res.t_done = req.arrival, t_admit, self.clock()
                res.bytes_reserved = need
                self.results[req.rid] = res
                self.reserved -= need
                self.free_slots.append(slot)
                done_any = True
            else:
                still.append((req, slot, handle, need, t_admit))
        self.inflight = still
        return done_any

    def step(self) -> bool:
        """One loop iteration; True while anything is pending or in flight."""
        self._admit()
        self._poll()
        with self.lock:
            busy = bool(self.pending) or bool(self.inflight)
        return busy

    def run(self, n_expected: int, idle_sleep: float = 2e-5, timeout: float = 3600.0):
        """Serve until n_expected results exist (requests may keep arriving)."""
        t0 = self.clock()
        while len(self.results) < n_expected:
            if not self.step():
                time.sleep(idle_sleep)
            if self.clock() - t0 > timeout:
                raise TimeoutError("serving loop did not finish")


def latency_stats(results: List[Result]) -> dict:
    ok = [r for r in results if r.ok]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    span = (max(r.t_done for r in ok) - min(r.t_arrival for r in ok)) if ok else 0.0
    segs = sum(r.segments for r in ok)
    return {"completed": len(ok), "failed": len(results) - len(ok),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "span_s": span,
            "ray_segments_per_s": segs / span if span > 0 else 0.0}


class GpuExecutor:
    """Runs requests through the C-ABI on one stream per slot."""

    def __init__(self, ctx=None, n_slots: int = 8, record_max_bytes: int = RECORD_MAX_BYTES,
                 replay_chunk_rays: int = REPLAY_CHUNK_RAYS):
        import torch
        from . import _lib as L
        self.L, self.torch = L, torch
        self.record_max_bytes = int(record_max_bytes)
        self.replay_chunk_rays = int(replay_chunk_rays)
        self.ctx = ctx or L.Context(0)
        self.streams = [torch.cuda.Stream(device=self.ctx.torch_device) for _ in range(n_slots)]
        self.scenes: Dict[int, object] = {}
        self.probes: Dict[int, object] = {}
        self._sizes: Dict[tuple, int] = {}

    def resident(self, wl):
        """Scene and probe uploaded once per distinct description object."""
        ks, kp = id(wl.scene), id(wl.probe)
        if ks not in self.scenes:
            self.scenes[ks] = (self.L.Scene(self.ctx, wl.scene), wl.scene)
        if kp not in self.probes:
            self.probes[kp] = (self.L.Probe(self.ctx, wl.probe), wl.probe)
        return self.scenes[ks][0], self.probes[kp][0]

    def record_bytes(self, req: Request) -> int:
        """Bytes of the path records of a gradient request, 0 when it is
        traced again in its backward (no gradient, records over the cap, or
        more transmits than one recorded forward takes)."""
        if not req.want_grad:
            return 0
        wl = req.workload
        scene, probe = self.resident(wl)
        n = self.L.us_recorded_workspace_size(scene, probe, wl.n_tx, wl.rays_per_tx, wl.max_bounces)
        return n if 0 < n <= self.record_max_bytes else 0

    def sizes(self, req: Request) -> dict:
        wl = req.workload
        scene, probe = self.resident(wl)
        L, p, g = self.L, wl.probe, wl.grid
        n_tx = wl.n_tx
        rows = n_tx * p.n_elem * p.n_t
        rec = self.record_bytes(req)
        s = {"rf": 4 * rows, "iq": 8 * g.n_px, "bmode": 4 * g.n_px,
             "ws_beam": L.load().us_beamform_workspace_size(probe.handle, n_tx),
             "ws_bmode": L.load().us_bmode_workspace_size(g.n_px), "counters": 40}
        if rec:
            s["ws_record"] = rec
        else:
            s["ws_trace"] = L.us_simulate_rf_workspace_size(scene, probe, n_tx, wl.rays_per_tx, wl.max_bounces)
        if req.want_grad:
            s.update({"b_ref": 4 * g.n_px, "g_b": 4 * g.n_px, "loss": 8, "g_theta": 8 * scene.n_params,
                      "ws_loss": L.load().us_image_loss_workspace_size(g.n_px)})
            if rec:
                s["ws_frame_vjp"] = L.us_frame_vjp_recorded_workspace_size(probe, g, n_tx)
            else:
                s["ws_frame_vjp"] = L.us_frame_vjp_workspace_size(
                    scene, probe, g, n_tx, min(wl.rays_per_tx, max(1, self.replay_chunk_rays // n_tx)),
                    wl.max_bounces)
        return s

    def bytes_needed(self, req: Request) -> int:
        return int(sum(self.sizes(req).values()))

    def launch(self, req: Request, slot: int):
        L, torch = self.L, self.torch
        wl = req.workload
        scene, probe = self.resident(wl)
        st = self.streams[slot]
        p, g = wl.probe, wl.grid
        dev = self.ctx.torch_device
        sz = self.sizes(req)
        with torch.cuda.stream(st):
            t = {}
            t["counters"] = torch.zeros(5, dtype=torch.int64, device=dev)
            t["rf"] = torch.empty((wl.n_tx, p.n_elem, p.n_t), dtype=torch.float32, device=dev)
            t["iq"] = torch.empty((g.n_x, g.n_z, 2), dtype=torch.float32, device=dev)
            t["bmode"] = torch.empty((g.n_x, g.n_z), dtype=torch.float32, device=dev)
            for k in ("ws_trace", "ws_record", "ws_beam", "ws_bmode", "ws_loss", "ws_frame_vjp"):
                if k in sz:
                    t[k] = torch.empty(max(256, sz[k]), dtype=torch.uint8, device=dev)
            rec = None
            if "ws_record" in sz:
                _, rec = L.us_simulate_rf_recorded(self.ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed,
                                                   wl.rays_per_elem, wl.max_bounces, rf=t["rf"],
                                                   counters=t["counters"], workspace=t["ws_record"], stream=st)
            else:
                L.us_simulate_rf(self.ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                                 wl.max_bounces, rf=t["rf"], counters=t["counters"], workspace=t["ws_trace"],
                                 stream=st)
            L.us_beamform(self.ctx, probe, g, wl.angles, wl.tx_ids, t["rf"], iq=t["iq"],
                          workspace=t["ws_beam"], stream=st)
            L.us_bmode(self.ctx, t["iq"], wl.dr_db, out=t["bmode"], workspace=t["ws_bmode"], stream=st)
            if req.want_grad:
                t["b_ref"] = self._device_ref(req.b_ref, t)
                t["loss"] = torch.empty(1, dtype=torch.float64, device=dev)
                t["g_b"] = torch.empty_like(t["bmode"])
                t["g_theta"] = torch.zeros(scene.n_params, dtype=torch.float64, device=dev)
                L.us_image_loss(self.ctx, t["bmode"], t["b_ref"], 0.0, 1.0, loss=t["loss"],
                                g_bmode=t["g_b"], workspace=t["ws_loss"], stream=st)
                if rec is not None:
                    L.us_frame_vjp_recorded(self.ctx, rec, g, t["iq"], t["g_b"], wl.dr_db, g_theta=t["g_theta"],
                                            workspace=t["ws_frame_vjp"], stream=st)
                else:
                    L.us_frame_vjp(self.ctx, scene, probe, g, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                                   wl.max_bounces, t["iq"], t["g_b"], wl.dr_db, g_theta=t["g_theta"],
                                   workspace=t["ws_frame_vjp"], stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return (t, ev)

    def _device_ref(self, b_ref, t):
        """The reference image on the device without a host-blocking copy:
        a device tensor is used as it is; a host array is copied into pinned
        memory and sent with an asynchronous copy on the current (slot)
        stream, its pinned buffer kept in the request's handle until the
        request completes."""
        torch = self.torch
        if isinstance(b_ref, torch.Tensor) and b_ref.is_cuda:
            return b_ref
        host = torch.from_numpy(np.ascontiguousarray(b_ref, dtype=np.float32)).pin_memory()
        t["b_ref_host"] = host
        return host.to(self.ctx.torch_device, non_blocking=True)

    def done(self, handle) -> bool:
        return handle[1].query()

    def finish(self, req: Request, handle) -> Result:
        t, _ = handle
        c = t["counters"].cpu().numpy()
        res = Result(req.rid, True, bmode=t["bmode"], segments=int(c[0] + c[1]))
        if req.want_grad:
            res.loss = float(t["loss"].item())
            res.g_theta = t["g_theta"]
        return res


def poisson_arrivals(n: int, rate_hz: float, seed: int = 0) -> np.ndarray:
    """Arrival offsets [s] of a Poisson process (exponential gaps)."""
    rng = np.random.Generator(np.random.Philox(key=[seed, 7]))
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def replay_stream(server: Server, requests: List[Request], offsets: np.ndarray):
    """Submits requests at their arrival offsets (a client thread) while the
    calling thread runs the serving loop; returns the results in request order."""
    t0 = server.clock()

    def client():
        for req, off in zip(requests, offsets):
            delay = t0 + off - server.clock()
            if delay > 0:
                time.sleep(delay)
            server.submit(req)

    th = threading.Thread(target=client, daemon=True)
    th.start()
    server.run(len(requests))
    th.join()
    return [server.results[r.rid] for r in requests]


def reference_image(ex: GpuExecutor, wl, target_scene):
    """B-mode of `target_scene` under workload `wl` (the reference image of a
    gradient request), rendered through the library on the default stream;
    a float32 device tensor [n_x][n_z] that stays resident."""
    L, torch = ex.L, ex.torch
    scene = L.Scene(ex.ctx, target_scene)
    _, probe = ex.resident(wl)
    rf = L.us_simulate_rf(ex.ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                          wl.max_bounces)
    iq = L.us_beamform(ex.ctx, probe, wl.grid, wl.angles, wl.tx_ids, rf)
    b = L.us_bmode(ex.ctx, iq, wl.dr_db)
    torch.cuda.synchronize()
    return b


def build_requests(ex: GpuExecutor, specs) -> List[Request]:
    """Requests from workloads.serving_requests specs (reference images rendered)."""
    reqs = []
    for i, sp in enumerate(specs):
        b_ref = reference_image(ex, sp.workload, sp.target) if sp.want_grad else None
        reqs.append(Request(i, sp.workload, sp.want_grad, b_ref))
    return reqs
