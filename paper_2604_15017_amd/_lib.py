"""ctypes binding of libusrt.so (include/usrt.h), same names as the C-ABI.

Argument marshalling only: every step of the path runs in the HIP kernels of
the library. PyTorch provides device memory (outputs and workspaces) and
streams. If the library is not built, every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libusrt.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "usrt.h")

US_OK, US_EINVAL, US_ENOMEM, US_EDEVICE, US_ETOOBIG = 0, -1, -2, -3, -4


class USError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class us_probe_desc(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int32), ("pitch", ctypes.c_double),
                ("elem_width", ctypes.c_double), ("elem_height", ctypes.c_double),
                ("f0", ctypes.c_double), ("n_cycles", ctypes.c_double), ("fs", ctypes.c_double),
                ("n_t", ctypes.c_int32), ("c_ref", ctypes.c_double),
                ("alpha_main", ctypes.c_double), ("alpha_cut", ctypes.c_double)]


class us_scene_desc(ctypes.Structure):
    _fields_ = [("n_regions", ctypes.c_int32), ("n_planes", ctypes.c_int32),
                ("n_spheres", ctypes.c_int32), ("theta", ctypes.c_void_p),
                ("plane_regions", ctypes.c_void_p), ("plane_kd", ctypes.c_void_p),
                ("sphere_regions", ctypes.c_void_p), ("sphere_kd", ctypes.c_void_p),
                ("start_region", ctypes.c_int32),
                ("n_meshes", ctypes.c_int32), ("n_basis", ctypes.c_int32),
                ("mesh_regions", ctypes.c_void_p), ("mesh_kd", ctypes.c_void_p),
                ("n_vertices", ctypes.c_int64), ("n_triangles", ctypes.c_int64),
                ("vertices", ctypes.c_void_p), ("vnormal", ctypes.c_void_p),
                ("vbasis", ctypes.c_void_p), ("vmesh", ctypes.c_void_p),
                ("triangles", ctypes.c_void_p), ("tmesh", ctypes.c_void_p),
                ("n_cylinders", ctypes.c_int32), ("cylinder_regions", ctypes.c_void_p),
                ("cylinder_kd", ctypes.c_void_p)]


class us_tx_desc(ctypes.Structure):
    _fields_ = [("angle", ctypes.c_double), ("id", ctypes.c_uint32)]


class us_grid_desc(ctypes.Structure):
    _fields_ = [("n_x", ctypes.c_int32), ("n_z", ctypes.c_int32), ("x0", ctypes.c_double),
                ("dx", ctypes.c_double), ("z0", ctypes.c_double), ("dz", ctypes.c_double)]


_lib = None
vp, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t

_SIGNATURES = {
    "us_last_error": (ctypes.c_char_p, []),
    "us_create": (ctypes.c_int, [ctypes.c_int, vp]),
    "us_destroy": (ctypes.c_int, [vp]),
    "us_probe_upload": (ctypes.c_int, [vp, vp, vp]),
    "us_probe_destroy": (ctypes.c_int, [vp]),
    "us_scene_upload": (ctypes.c_int, [vp, vp, vp, vp]),
    "us_scene_destroy": (ctypes.c_int, [vp]),
    "us_scene_set_params": (ctypes.c_int, [vp, vp, i32, vp]),
    "us_simulate_rf_workspace_size": (sz, [vp, vp, i32, i64, i32]),
    "us_simulate_rf": (ctypes.c_int, [vp, vp, vp, vp, i32, u64, i32, i64, i64, i32, vp, vp, vp,
                                      vp, sz, vp]),
    "us_beamform_workspace_size": (sz, [vp, i32]),
    "us_beamform": (ctypes.c_int, [vp, vp, vp, vp, i32, vp, vp, vp, sz, vp]),
    "us_beamform_static": (ctypes.c_int, [vp, vp, vp, vp, i32, vp, vp, vp]),
    "us_bmode_workspace_size": (sz, [i64]),
    "us_bmode": (ctypes.c_int, [vp, vp, i64, ctypes.c_float, vp, vp, sz, vp]),
    "us_bmode_vjp": (ctypes.c_int, [vp, vp, vp, i64, ctypes.c_float, vp, vp, sz, vp]),
    "us_beamform_vjp_workspace_size": (sz, [vp, i32]),
    "us_beamform_vjp": (ctypes.c_int, [vp, vp, vp, vp, i32, vp, vp, vp, sz, vp]),
    "us_beamform_acq_vjp_workspace_size": (sz, [vp, vp, i32]),
    "us_beamform_acq_vjp": (ctypes.c_int, [vp, vp, vp, vp, i32, vp, vp, vp, vp, sz, vp]),
    "us_simulate_rf_vjp_workspace_size": (sz, [vp, vp, i32, i64, i32]),
    "us_simulate_rf_vjp": (ctypes.c_int, [vp, vp, vp, vp, i32, u64, i32, i64, i64, i32, vp, vp,
                                          vp, sz, vp]),
    "us_simulate_rf_vjp_acq": (ctypes.c_int, [vp, vp, vp, vp, i32, u64, i32, i64, i64, i32, vp, vp, vp, vp, sz, vp]),
    "us_frame_vjp_workspace_size": (sz, [vp, vp, vp, i32, i64, i32]),
    "us_frame_vjp": (ctypes.c_int, [vp, vp, vp, vp, vp, i32, u64, i32, i64, i64, i32, vp, vp,
                                    ctypes.c_float, vp, vp, sz, vp]),
    "us_recorded_workspace_size": (sz, [vp, vp, i32, i64, i32]),
    "us_simulate_rf_recorded": (ctypes.c_int, [vp, vp, vp, vp, i32, u64, i32, i64, i64, i32, vp, vp, vp, sz, vp]),
    "us_simulate_rf_vjp_recorded": (ctypes.c_int, [vp, vp, vp, vp, i32, u64, i32, i64, i64, i32, vp, vp,
                                                   vp, sz, vp]),
    "us_frame_vjp_recorded_workspace_size": (sz, [vp, vp, i32]),
    "us_frame_vjp_recorded": (ctypes.c_int, [vp, vp, vp, vp, vp, i32, u64, i32, i64, i64, i32, vp, vp,
                                             ctypes.c_float, vp, vp, sz, vp, sz, vp]),
    "us_image_loss_workspace_size": (sz, [i64]),
    "us_image_loss": (ctypes.c_int, [vp, vp, vp, i64, ctypes.c_double, ctypes.c_double, vp, vp,
                                     vp, sz, vp]),
    "us_param_map": (ctypes.c_int, [vp, vp, vp, vp, i32, vp, vp]),
    "us_adam_step": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, vp]),
    "us_profile_enable": (ctypes.c_int, [vp, ctypes.c_int]),
    "us_profile_read": (ctypes.c_int, [vp, i32, vp, vp, vp, vp]),
}


def header_symbols():
    """Function names declared in include/usrt.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(us_[a-z_]+)\s*\(", text)) - {"us_probe_desc", "us_scene_desc"})


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # torch ships its own HIP runtime under the same soname; it has to be
        # the one loaded first so that torch and the library share one runtime
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, name: str):
    if rc != US_OK:
        msg = load().us_last_error().decode()
        raise USError(rc, f"{name}: {msg}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP library needs a visible GPU")
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _expect(t, n: int, dtype, name: str):
    """Raise unless `t` is a contiguous device tensor of `n` elements of `dtype`:
    the library reads and writes exactly that many through the raw pointer."""
    if t is None:
        raise ValueError(f"{name}: missing")
    if t.dtype != dtype or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of {n} elements "
                         f"(got {t.dtype}, {t.numel()} elements, contiguous={t.is_contiguous()})")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    return t


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _expect_ws(ws, name: str = "workspace"):
    """A caller workspace is a contiguous uint8 device tensor: its element
    count is passed to the library as its size in bytes."""
    import torch
    return _expect(ws, ws.numel() if ws is not None else 0, torch.uint8, name)


def _tx_array(angles, tx_ids):
    angles = np.asarray(angles, dtype=np.float64).reshape(-1)
    ids = np.asarray(tx_ids if tx_ids is not None else np.arange(len(angles)), dtype=np.uint32).reshape(-1)
    if ids.shape[0] != angles.shape[0]:
        raise ValueError(f"tx_ids has {ids.shape[0]} entries for {angles.shape[0]} steering angles")
    arr = (us_tx_desc * len(angles))()
    for i, (a, k) in enumerate(zip(angles, ids)):
        arr[i].angle = float(a)
        arr[i].id = int(k)
    return arr, len(angles)


class Context:
    """us_create / us_destroy."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(load().us_create(device, ctypes.byref(h)), "us_create")
        self.handle, self.device = h, device
        self.torch_device = _torch().device("cuda", device)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.us_destroy(self.handle)
            self.handle = None


class Probe:
    """us_probe_upload of a workloads.Probe-like object."""

    def __init__(self, ctx: Context, p):
        d = us_probe_desc(int(p.n_elem), float(p.pitch), float(p.elem_width),
                          float(p.elem_height), float(p.f0), float(p.n_cycles), float(p.fs),
                          int(p.n_t), float(p.c_ref), float(p.alpha_main), float(p.alpha_cut))
        h = ctypes.c_void_p()
        _check(load().us_probe_upload(ctx.handle, ctypes.byref(d), ctypes.byref(h)), "us_probe_upload")
        self.ctx, self.handle, self.desc = ctx, h, p

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.us_probe_destroy(self.handle)
            self.handle = None


class Scene:
    """us_scene_upload of a workloads.Scene-like object."""

    def __init__(self, ctx: Context, s, theta: Optional[np.ndarray] = None):
        th = np.ascontiguousarray(s.theta() if theta is None else theta, dtype=np.float64)
        pr = np.ascontiguousarray(s.plane_regions, dtype=np.int32)
        pk = np.ascontiguousarray(s.plane_kd, dtype=np.float64)
        sr = np.ascontiguousarray(s.sphere_regions, dtype=np.int32)
        sk = np.ascontiguousarray(s.sphere_kd, dtype=np.float64)
        d = us_scene_desc(int(s.regions.shape[0]), int(s.planes.shape[0]),
                          int(s.spheres.shape[0]), th.ctypes.data, pr.ctypes.data, pk.ctypes.data,
                          sr.ctypes.data, sk.ctypes.data, int(s.start_region))
        n_c = int(getattr(s, "n_cylinders", 0))
        if n_c:
            cr = np.ascontiguousarray(s.cylinder_regions, dtype=np.int32).reshape(-1)
            ck = np.ascontiguousarray(s.cylinder_kd, dtype=np.float64).reshape(-1)
            if cr.shape[0] != 2 * n_c or ck.shape[0] != n_c:
                raise ValueError("cylinder arrays disagree")
            d.n_cylinders, d.cylinder_regions, d.cylinder_kd = n_c, cr.ctypes.data, ck.ctypes.data
            self._keep = (cr, ck)
        meshes = list(getattr(s, "meshes", None) or [])
        if meshes:
            # concatenate the meshes: global vertex ids, owning mesh per vertex / triangle
            offs = np.cumsum([0] + [len(m.vertices) for m in meshes])
            arr = dict(
                regions=np.array([[m.region_in, m.region_out] for m in meshes], np.int32),
                kd=np.array([m.kd for m in meshes], np.float64),
                v=np.concatenate([m.vertices for m in meshes]).astype(np.float64),
                n=np.concatenate([m.normals for m in meshes]).astype(np.float64),
                b=np.concatenate([m.basis for m in meshes]).astype(np.float64),
                vm=np.concatenate([np.full(len(m.vertices), k, np.int32) for k, m in enumerate(meshes)]),
                t=np.concatenate([np.asarray(m.triangles) + offs[k] for k, m in enumerate(meshes)]).astype(np.int32),
                tm=np.concatenate([np.full(len(m.triangles), k, np.int32) for k, m in enumerate(meshes)]))
            arr = {k: np.ascontiguousarray(v) for k, v in arr.items()}
            nb = {m.basis.shape[1] for m in meshes}
            if len(nb) != 1:
                raise ValueError("all meshes need the same number of basis functions")
            d.n_meshes, d.n_basis = len(meshes), nb.pop()
            d.mesh_regions, d.mesh_kd = arr["regions"].ctypes.data, arr["kd"].ctypes.data
            d.n_vertices, d.n_triangles = len(arr["v"]), len(arr["t"])
            d.vertices, d.vnormal, d.vbasis = arr["v"].ctypes.data, arr["n"].ctypes.data, arr["b"].ctypes.data
            d.vmesh, d.triangles, d.tmesh = arr["vm"].ctypes.data, arr["t"].ctypes.data, arr["tm"].ctypes.data
        h = ctypes.c_void_p()
        n = ctypes.c_int32()
        _check(load().us_scene_upload(ctx.handle, ctypes.byref(d), ctypes.byref(h), ctypes.byref(n)),
               "us_scene_upload")
        self.ctx, self.handle, self.n_params, self.desc = ctx, h, n.value, s

    def set_params(self, theta_dev, stream=None):
        """us_scene_set_params from a float64 device tensor of n_params entries."""
        _expect(theta_dev, self.n_params, _torch().float64, "theta")
        _check(load().us_scene_set_params(self.handle, _ptr(theta_dev), int(theta_dev.numel()),
                                          _stream(stream)), "us_scene_set_params")

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.us_scene_destroy(self.handle)
            self.handle = None


def us_simulate_rf_workspace_size(scene: Scene, probe: Probe, n_tx: int, ray_count: int,
                                  max_bounces: int) -> int:
    return int(load().us_simulate_rf_workspace_size(scene.handle, probe.handle, n_tx, ray_count,
                                                    max_bounces))


def us_simulate_rf(ctx: Context, scene: Scene, probe: Probe, angles, tx_ids, seed: int,
                   rays_per_elem: int, max_bounces: int, ray_begin: int = 0,
                   ray_count: Optional[int] = None, rf=None, counters=None, ray_hash=None,
                   workspace=None, stream=None):
    torch = _torch()
    p = probe.desc
    tx, n_tx = _tx_array(angles, tx_ids)
    if ray_count is None:
        ray_count = int(p.n_elem) * int(rays_per_elem) - ray_begin
    if rf is None:
        rf = torch.empty((n_tx, p.n_elem, p.n_t), dtype=torch.float32, device=ctx.torch_device)
    _expect(rf, n_tx * p.n_elem * p.n_t, torch.float32, "rf")
    if counters is not None:
        _expect(counters, 5, torch.int64, "counters")
    if ray_hash is not None:
        _expect(ray_hash, n_tx * int(ray_count), torch.int64, "ray_hash")
    if workspace is None:
        workspace = _workspace(us_simulate_rf_workspace_size(scene, probe, n_tx, ray_count,
                                                             max_bounces), ctx.torch_device)
    _expect_ws(workspace)
    _check(load().us_simulate_rf(ctx.handle, scene.handle, probe.handle, tx, n_tx, int(seed),
                                 int(rays_per_elem), int(ray_begin), int(ray_count),
                                 int(max_bounces), _ptr(rf), _ptr(counters), _ptr(ray_hash),
                                 _ptr(workspace), workspace.numel(), _stream(stream)),
           "us_simulate_rf")
    return rf


def _grid(g) -> us_grid_desc:
    return us_grid_desc(int(g.n_x), int(g.n_z), float(g.x0), float(g.dx), float(g.z0), float(g.dz))


def us_beamform(ctx: Context, probe: Probe, grid, angles, tx_ids, rf, iq=None, workspace=None,
                stream=None):
    torch = _torch()
    tx, n_tx = _tx_array(angles, tx_ids)
    g = _grid(grid)
    if iq is None:
        iq = torch.empty((g.n_x, g.n_z, 2), dtype=torch.float32, device=ctx.torch_device)
    p = probe.desc
    _expect(rf, n_tx * p.n_elem * p.n_t, torch.float32, "rf")
    _expect(iq, 2 * g.n_x * g.n_z, torch.float32, "iq")
    if workspace is None:
        workspace = _workspace(load().us_beamform_workspace_size(probe.handle, n_tx), ctx.torch_device)
    _expect_ws(workspace)
    _check(load().us_beamform(ctx.handle, probe.handle, ctypes.byref(g), tx, n_tx, _ptr(rf),
                              _ptr(iq), _ptr(workspace), workspace.numel(), _stream(stream)),
           "us_beamform")
    return iq


def us_beamform_static(ctx: Context, probe: Probe, grid, angles, tx_ids, rf, iq=None, stream=None):
    """us_beamform without a workspace (the library's static scratch; calls on
    one GPU must not overlap)."""
    torch = _torch()
    tx, n_tx = _tx_array(angles, tx_ids)
    g = _grid(grid)
    if iq is None:
        iq = torch.empty((g.n_x, g.n_z, 2), dtype=torch.float32, device=ctx.torch_device)
    p = probe.desc
    _expect(rf, n_tx * p.n_elem * p.n_t, torch.float32, "rf")
    _expect(iq, 2 * g.n_x * g.n_z, torch.float32, "iq")
    _check(load().us_beamform_static(ctx.handle, probe.handle, ctypes.byref(g), tx, n_tx, _ptr(rf), _ptr(iq),
                                     _stream(stream)), "us_beamform_static")
    return iq


def us_beamform_acq_vjp(ctx: Context, probe: Probe, grid, angles, tx_ids, rf, g_iq, out=None,
                        workspace=None, stream=None):
    """d Re<g_iq, I> / d (steering angle of each transmit, c_ref, pitch) as a
    float64 device tensor [n_tx + 2]."""
    torch = _torch()
    tx, n_tx = _tx_array(angles, tx_ids)
    g = _grid(grid)
    if out is None:
        out = torch.empty(n_tx + 2, dtype=torch.float64, device=ctx.torch_device)
    p = probe.desc
    _expect(rf, n_tx * p.n_elem * p.n_t, torch.float32, "rf")
    _expect(g_iq, 2 * g.n_x * g.n_z, torch.float32, "g_iq")
    _expect(out, n_tx + 2, torch.float64, "out")
    if workspace is None:
        workspace = _workspace(load().us_beamform_acq_vjp_workspace_size(probe.handle, ctypes.byref(g), n_tx),
                               ctx.torch_device)
    _expect_ws(workspace)
    _check(load().us_beamform_acq_vjp(ctx.handle, probe.handle, ctypes.byref(g), tx, n_tx, _ptr(rf), _ptr(g_iq),
                                      _ptr(out), _ptr(workspace), workspace.numel(), _stream(stream)),
           "us_beamform_acq_vjp")
    return out


def us_bmode(ctx: Context, iq, dr_db: float, out=None, workspace=None, stream=None):
    torch = _torch()
    n_px = iq.numel() // 2
    _expect(iq, 2 * n_px, torch.float32, "iq")
    if out is None:
        out = torch.empty(iq.shape[:-1], dtype=torch.float32, device=ctx.torch_device)
    _expect(out, n_px, torch.float32, "bmode")
    if workspace is None:
        workspace = _workspace(load().us_bmode_workspace_size(n_px), ctx.torch_device)
    _expect_ws(workspace)
    _check(load().us_bmode(ctx.handle, _ptr(iq), n_px, float(dr_db), _ptr(out), _ptr(workspace),
                           workspace.numel(), _stream(stream)), "us_bmode")
    return out


def us_image_loss(ctx: Context, bmode, ref, lambda1: float = 0.0, lambda2: float = 1.0,
                  loss=None, g_bmode=None, want_grad: bool = True, workspace=None, stream=None):
    """Returns (loss as a 1-element float64 device tensor, dL/dB or None)."""
    torch = _torch()
    n_px = bmode.numel()
    if workspace is None:
        workspace = _workspace(load().us_image_loss_workspace_size(n_px), ctx.torch_device)
    _expect_ws(workspace)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=ctx.torch_device)
    if want_grad and g_bmode is None:
        g_bmode = torch.empty_like(bmode)
    _expect(bmode, n_px, torch.float32, "bmode")
    _expect(ref, n_px, torch.float32, "ref")
    _expect(loss, 1, torch.float64, "loss")
    if want_grad:
        _expect(g_bmode, n_px, torch.float32, "g_bmode")
    _check(load().us_image_loss(ctx.handle, _ptr(bmode), _ptr(ref), n_px, float(lambda1),
                                float(lambda2), _ptr(loss), _ptr(g_bmode if want_grad else None),
                                _ptr(workspace), workspace.numel(), _stream(stream)), "us_image_loss")
    return loss, (g_bmode if want_grad else None)


def us_bmode_vjp(ctx: Context, iq, g_bmode, dr_db: float, g_iq=None, workspace=None, stream=None):
    torch = _torch()
    n_px = iq.numel() // 2
    if g_iq is None:
        g_iq = torch.empty_like(iq)
    _expect(iq, 2 * n_px, torch.float32, "iq")
    _expect(g_bmode, n_px, torch.float32, "g_bmode")
    _expect(g_iq, 2 * n_px, torch.float32, "g_iq")
    if workspace is None:
        workspace = _workspace(load().us_bmode_workspace_size(n_px), ctx.torch_device)
    _expect_ws(workspace)
    _check(load().us_bmode_vjp(ctx.handle, _ptr(iq), _ptr(g_bmode), n_px, float(dr_db), _ptr(g_iq),
                               _ptr(workspace), workspace.numel(), _stream(stream)), "us_bmode_vjp")
    return g_iq


def us_beamform_vjp(ctx: Context, probe: Probe, grid, angles, tx_ids, g_iq, g_rf=None,
                    workspace=None, stream=None):
    torch = _torch()
    tx, n_tx = _tx_array(angles, tx_ids)
    g = _grid(grid)
    p = probe.desc
    if g_rf is None:
        g_rf = torch.empty((n_tx, p.n_elem, p.n_t), dtype=torch.float32, device=ctx.torch_device)
    _expect(g_iq, 2 * g.n_x * g.n_z, torch.float32, "g_iq")
    _expect(g_rf, n_tx * p.n_elem * p.n_t, torch.float32, "g_rf")
    if workspace is None:
        workspace = _workspace(load().us_beamform_vjp_workspace_size(probe.handle, n_tx),
                               ctx.torch_device)
    _expect_ws(workspace)
    _check(load().us_beamform_vjp(ctx.handle, probe.handle, ctypes.byref(g), tx, n_tx, _ptr(g_iq),
                                  _ptr(g_rf), _ptr(workspace), workspace.numel(), _stream(stream)),
           "us_beamform_vjp")
    return g_rf


def us_simulate_rf_vjp_workspace_size(scene: Scene, probe: Probe, n_tx: int, ray_count: int,
                                      max_bounces: int) -> int:
    return int(load().us_simulate_rf_vjp_workspace_size(scene.handle, probe.handle, n_tx,
                                                        ray_count, max_bounces))


def us_simulate_rf_vjp(ctx: Context, scene: Scene, probe: Probe, angles, tx_ids, seed: int,
                       rays_per_elem: int, max_bounces: int, g_rf, g_theta=None,
                       ray_begin: int = 0, ray_count: Optional[int] = None, workspace=None,
                       stream=None, g_acq=None):
    """g_theta += (d rf / d theta)^T g_rf; with g_acq (float64 [n_tx + 3]) also
    the acquisition parameters (steering angles, c_ref, pitch, f0), accumulated."""
    torch = _torch()
    p = probe.desc
    tx, n_tx = _tx_array(angles, tx_ids)
    if ray_count is None:
        ray_count = int(p.n_elem) * int(rays_per_elem) - ray_begin
    if g_theta is None:
        g_theta = torch.zeros(scene.n_params, dtype=torch.float64, device=ctx.torch_device)
    _expect(g_rf, n_tx * p.n_elem * p.n_t, torch.float32, "g_rf")
    _expect(g_theta, scene.n_params, torch.float64, "g_theta")
    if workspace is None:
        workspace = _workspace(us_simulate_rf_vjp_workspace_size(scene, probe, n_tx, ray_count,
                                                                 max_bounces), ctx.torch_device)
    _expect_ws(workspace)
    if g_acq is None:
        _check(load().us_simulate_rf_vjp(ctx.handle, scene.handle, probe.handle, tx, n_tx, int(seed),
                                         int(rays_per_elem), int(ray_begin), int(ray_count),
                                         int(max_bounces), _ptr(g_rf), _ptr(g_theta), _ptr(workspace),
                                         workspace.numel(), _stream(stream)), "us_simulate_rf_vjp")
    else:
        _expect(g_acq, n_tx + 3, torch.float64, "g_acq")
        _check(load().us_simulate_rf_vjp_acq(ctx.handle, scene.handle, probe.handle, tx, n_tx, int(seed),
                                             int(rays_per_elem), int(ray_begin), int(ray_count),
                                             int(max_bounces), _ptr(g_rf), _ptr(g_theta), _ptr(g_acq),
                                             _ptr(workspace), workspace.numel(), _stream(stream)),
               "us_simulate_rf_vjp_acq")
    return g_theta


def us_frame_vjp_workspace_size(scene: Scene, probe: Probe, grid, n_tx: int, ray_count: int,
                                max_bounces: int) -> int:
    g = _grid(grid)
    return int(load().us_frame_vjp_workspace_size(scene.handle, probe.handle, ctypes.byref(g), n_tx, ray_count,
                                                  max_bounces))


def us_frame_vjp(ctx: Context, scene: Scene, probe: Probe, grid, angles, tx_ids, seed: int,
                 rays_per_elem: int, max_bounces: int, iq, g_bmode, dr_db: float, g_theta=None,
                 ray_begin: int = 0, ray_count: Optional[int] = None, workspace=None, stream=None):
    """g_theta += (d bmode / d theta)^T g_bmode in one call: the B-mode, DAS,
    analytic-signal, pulse and transport adjoints (iq: the image the B-mode
    frame was formed from)."""
    torch = _torch()
    p = probe.desc
    tx, n_tx = _tx_array(angles, tx_ids)
    g = _grid(grid)
    n_px = g.n_x * g.n_z
    if ray_count is None:
        ray_count = int(p.n_elem) * int(rays_per_elem) - ray_begin
    if g_theta is None:
        g_theta = torch.zeros(scene.n_params, dtype=torch.float64, device=ctx.torch_device)
    _expect(iq, 2 * n_px, torch.float32, "iq")
    _expect(g_bmode, n_px, torch.float32, "g_bmode")
    _expect(g_theta, scene.n_params, torch.float64, "g_theta")
    if workspace is None:
        workspace = _workspace(us_frame_vjp_workspace_size(scene, probe, grid, n_tx, ray_count, max_bounces),
                               ctx.torch_device)
    _expect_ws(workspace)
    _check(load().us_frame_vjp(ctx.handle, scene.handle, probe.handle, ctypes.byref(g), tx, n_tx, int(seed),
                               int(rays_per_elem), int(ray_begin), int(ray_count), int(max_bounces), _ptr(iq),
                               _ptr(g_bmode), float(dr_db), _ptr(g_theta), _ptr(workspace), workspace.numel(),
                               _stream(stream)), "us_frame_vjp")
    return g_theta


class Recorded:
    """One recorded forward: its workspace (the step records the backward
    reads) and the arguments a recorded backward repeats."""

    def __init__(self, scene, probe, angles, tx_ids, seed, rays_per_elem, max_bounces, ray_begin, ray_count,
                 workspace):
        self.scene, self.probe = scene, probe
        self.angles, self.tx_ids = angles, tx_ids
        self.seed, self.rays_per_elem, self.max_bounces = int(seed), int(rays_per_elem), int(max_bounces)
        self.ray_begin, self.ray_count = int(ray_begin), int(ray_count)
        self.workspace = workspace

    def args(self):
        tx, n_tx = _tx_array(self.angles, self.tx_ids)
        return tx, n_tx, (self.seed, self.rays_per_elem, self.ray_begin, self.ray_count, self.max_bounces)


def us_recorded_workspace_size(scene: Scene, probe: Probe, n_tx: int, ray_count: int, max_bounces: int) -> int:
    return int(load().us_recorded_workspace_size(scene.handle, probe.handle, n_tx, ray_count, max_bounces))


def us_simulate_rf_recorded(ctx: Context, scene: Scene, probe: Probe, angles, tx_ids, seed: int,
                            rays_per_elem: int, max_bounces: int, ray_begin: int = 0,
                            ray_count: Optional[int] = None, rf=None, counters=None, workspace=None,
                            stream=None):
    """The RF of us_simulate_rf (and its event counters, added to counters
    when given), keeping the path records for a recorded backward; returns
    (rf, Recorded)."""
    torch = _torch()
    p = probe.desc
    tx, n_tx = _tx_array(angles, tx_ids)
    if ray_count is None:
        ray_count = int(p.n_elem) * int(rays_per_elem) - ray_begin
    if rf is None:
        rf = torch.empty((n_tx, p.n_elem, p.n_t), dtype=torch.float32, device=ctx.torch_device)
    _expect(rf, n_tx * p.n_elem * p.n_t, torch.float32, "rf")
    if counters is not None:
        _expect(counters, 5, torch.int64, "counters")
    if workspace is None:
        need = us_recorded_workspace_size(scene, probe, n_tx, ray_count, max_bounces)
        if need == 0:
            raise USError(US_EINVAL, "us_simulate_rf_recorded: at most 64 transmits and at least one ray")
        workspace = _workspace(need, ctx.torch_device)
    _expect_ws(workspace)
    _check(load().us_simulate_rf_recorded(ctx.handle, scene.handle, probe.handle, tx, n_tx, int(seed),
                                          int(rays_per_elem), int(ray_begin), int(ray_count), int(max_bounces),
                                          _ptr(rf), _ptr(counters), _ptr(workspace), workspace.numel(),
                                          _stream(stream)),
           "us_simulate_rf_recorded")
    return rf, Recorded(scene, probe, angles, tx_ids, seed, rays_per_elem, max_bounces, ray_begin, ray_count,
                        workspace)


def us_simulate_rf_vjp_recorded(ctx: Context, rec: Recorded, g_rf, g_theta=None, stream=None):
    """us_simulate_rf_vjp from the records of a recorded forward."""
    torch = _torch()
    p = rec.probe.desc
    tx, n_tx, (seed, rpe, rb, rc, nb) = rec.args()
    if g_theta is None:
        g_theta = torch.zeros(rec.scene.n_params, dtype=torch.float64, device=ctx.torch_device)
    _expect(g_rf, n_tx * p.n_elem * p.n_t, torch.float32, "g_rf")
    _expect(g_theta, rec.scene.n_params, torch.float64, "g_theta")
    _check(load().us_simulate_rf_vjp_recorded(ctx.handle, rec.scene.handle, rec.probe.handle, tx, n_tx, seed, rpe,
                                              rb, rc, nb, _ptr(g_rf), _ptr(g_theta), _ptr(rec.workspace),
                                              rec.workspace.numel(), _stream(stream)),
           "us_simulate_rf_vjp_recorded")
    return g_theta


def us_frame_vjp_recorded_workspace_size(probe: Probe, grid, n_tx: int) -> int:
    g = _grid(grid)
    return int(load().us_frame_vjp_recorded_workspace_size(probe.handle, ctypes.byref(g), n_tx))


def us_frame_vjp_recorded(ctx: Context, rec: Recorded, grid, iq, g_bmode, dr_db: float, g_theta=None,
                          workspace=None, stream=None):
    """us_frame_vjp from the records of a recorded forward."""
    torch = _torch()
    tx, n_tx, (seed, rpe, rb, rc, nb) = rec.args()
    g = _grid(grid)
    n_px = g.n_x * g.n_z
    if g_theta is None:
        g_theta = torch.zeros(rec.scene.n_params, dtype=torch.float64, device=ctx.torch_device)
    _expect(iq, 2 * n_px, torch.float32, "iq")
    _expect(g_bmode, n_px, torch.float32, "g_bmode")
    _expect(g_theta, rec.scene.n_params, torch.float64, "g_theta")
    if workspace is None:
        workspace = _workspace(us_frame_vjp_recorded_workspace_size(rec.probe, grid, n_tx), ctx.torch_device)
    _expect_ws(workspace)
    _check(load().us_frame_vjp_recorded(ctx.handle, rec.scene.handle, rec.probe.handle, ctypes.byref(g), tx, n_tx,
                                        seed, rpe, rb, rc, nb, _ptr(iq), _ptr(g_bmode), float(dr_db),
                                        _ptr(g_theta), _ptr(workspace), workspace.numel(), _ptr(rec.workspace),
                                        rec.workspace.numel(), _stream(stream)), "us_frame_vjp_recorded")
    return g_theta


def us_param_map(ctx: Context, u, lo, hi, theta=None, stream=None):
    """theta = lo + clip(u, 0, 1) (hi - lo) on float64 device tensors."""
    torch = _torch()
    n = u.numel()
    if theta is None:
        theta = torch.empty(n, dtype=torch.float64, device=ctx.torch_device)
    for t, name in ((u, "u"), (lo, "lo"), (hi, "hi"), (theta, "theta")):
        _expect(t, n, torch.float64, name)
    _check(load().us_param_map(ctx.handle, _ptr(u), _ptr(lo), _ptr(hi), n, _ptr(theta),
                               _stream(stream)), "us_param_map")
    return theta


def us_adam_step(ctx: Context, u, m, v, g_theta, lo, hi, lr, step: int, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8, max_norm: float = 0.0, stream=None):
    """One Adam step on u (float64 device tensors, updated in place with m, v)."""
    torch = _torch()
    n = u.numel()
    for t, name in ((u, "u"), (m, "m"), (v, "v"), (g_theta, "g_theta"), (lo, "lo"), (hi, "hi"), (lr, "lr")):
        _expect(t, n, torch.float64, name)
    _check(load().us_adam_step(ctx.handle, _ptr(u), _ptr(m), _ptr(v), _ptr(g_theta), _ptr(lo),
                               _ptr(hi), _ptr(lr), u.numel(), int(step), float(beta1),
                               float(beta2), float(eps), float(max_norm), _stream(stream)),
           "us_adam_step")


def us_profile_enable(ctx: Context, enable: bool = True):
    _check(load().us_profile_enable(ctx.handle, 1 if enable else 0), "us_profile_enable")


def us_profile_read(ctx: Context, max_kernels: int = 64):
    """{kernel name: (total ms, launches)} since the last read."""
    names = ctypes.create_string_buffer(32 * max_kernels)
    ms = (ctypes.c_double * max_kernels)()
    cnt = (ctypes.c_int64 * max_kernels)()
    n = ctypes.c_int32()
    _check(load().us_profile_read(ctx.handle, max_kernels, names, ms, cnt, ctypes.byref(n)),
           "us_profile_read")
    out = {}
    for i in range(n.value):
        name = names.raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
        out[name] = (ms[i], cnt[i])
    return out
