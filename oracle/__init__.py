"""FP64 CPU oracle for the differentiable Monte-Carlo ultrasound pipeline.

TEST INFRASTRUCTURE ONLY. Only tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package. It shares no code with the GPU
library and imports nothing from it; inputs arrive as plain objects (scene,
probe, grid, transmit list) with the attributes documented in `trace`.

Pieces:
  transport.cpp  - FP64 ray transport (paper Sec. 2.3) with forward-mode dual
                   numbers for parameter gradients (Sec. 3.2, Eq. chain_rule)
  chain.py       - splat, pulse filter (Eq. axial_sig), analytic signal,
                   delay-and-sum (Eq. das) and its adjoint (Eq. das_adjoint),
                   envelope / log compression and their adjoints, numpy FP64
  optim.py       - the inverse loop: clip parameterisation (Eq. clip01,
                   scale_phys, clip_grad), Adam (Eq. adam), the weighted
                   L1 + L2 image loss, one micro-batched iteration

Parity status: every function here is pinned by a `-m "not gpu"` test against
a closed form, an invariant, a library routine, brute force or finite
differences (tests/test_oracle_*.py), except the absolute scale of diffuse
backscatter, which is a modelling choice ("parity unpinned"; only its
consistency with a second estimator is pinned).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "transport.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C++ transport with g++ (plain -O2, OpenMP over rays)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(ctypes.Structure):
    _fields_ = [("n_regions", ctypes.c_int), ("n_planes", ctypes.c_int),
                ("n_spheres", ctypes.c_int),
                ("plane_regions", ctypes.c_void_p), ("plane_kd", ctypes.c_void_p),
                ("sphere_regions", ctypes.c_void_p), ("sphere_kd", ctypes.c_void_p),
                ("start_region", ctypes.c_int),
                ("n_meshes", ctypes.c_int), ("n_basis", ctypes.c_int),
                ("mesh_regions", ctypes.c_void_p), ("mesh_kd", ctypes.c_void_p),
                ("n_vertices", ctypes.c_int64), ("n_triangles", ctypes.c_int64),
                ("vrest", ctypes.c_void_p), ("vnormal", ctypes.c_void_p), ("vbasis", ctypes.c_void_p),
                ("vmesh", ctypes.c_void_p), ("tris", ctypes.c_void_p), ("tmesh", ctypes.c_void_p),
                ("mesh_bruteforce", ctypes.c_int),
                ("n_cylinders", ctypes.c_int), ("cylinder_regions", ctypes.c_void_p),
                ("cylinder_kd", ctypes.c_void_p)]


class _Probe(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int), ("pitch", ctypes.c_double),
                ("elem_width", ctypes.c_double), ("elem_height", ctypes.c_double),
                ("f0", ctypes.c_double), ("n_cycles", ctypes.c_double), ("fs", ctypes.c_double),
                ("n_t", ctypes.c_int), ("c_ref", ctypes.c_double),
                ("alpha_main", ctypes.c_double), ("alpha_cut", ctypes.c_double)]


class _Run(ctypes.Structure):
    _fields_ = [("n_tx", ctypes.c_int), ("angles", ctypes.c_void_p), ("tx_ids", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("rays_per_elem", ctypes.c_int),
                ("ray_begin", ctypes.c_int64), ("ray_count", ctypes.c_int64),
                ("max_bounces", ctypes.c_int), ("nee_mode", ctypes.c_int),
                ("n_threads", ctypes.c_int), ("prob_mode", ctypes.c_int),
                ("prob_buf", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.oracle_trace.restype = vp
        lib.oracle_trace.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]
        lib.oracle_result_count.restype = ctypes.c_int64
        lib.oracle_result_count.argtypes = [vp]
        lib.oracle_result_segments.restype = ctypes.c_int64
        lib.oracle_result_segments.argtypes = [vp]
        lib.oracle_result_copy.argtypes = [vp] * 7
        lib.oracle_result_free.argtypes = [vp]
        lib.oracle_splat.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, vp]
        lib.oracle_philox.argtypes = [vp, vp, vp]
        lib.oracle_uniform.restype = ctypes.c_double
        lib.oracle_uniform.argtypes = [ctypes.c_uint64]
        lib.oracle_interface.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, vp, vp, vp]
        lib.oracle_cosine_dir.argtypes = [vp, ctypes.c_double, ctypes.c_double, vp]
        lib.oracle_directivity.restype = ctypes.c_double
        lib.oracle_directivity.argtypes = [vp, ctypes.c_double]
        lib.oracle_glossy.argtypes = [vp, vp] + [ctypes.c_double] * 7 + [vp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _probe_struct(probe) -> _Probe:
    return _Probe(int(probe.n_elem), float(probe.pitch), float(probe.elem_width),
                  float(probe.elem_height), float(probe.f0), float(probe.n_cycles),
                  float(probe.fs), int(probe.n_t), float(probe.c_ref),
                  float(probe.alpha_main), float(probe.alpha_cut))


class TraceResult:
    """Contributions (tx index, element, time, amplitude, ray id) of one trace call."""

    def __init__(self, tx, elem, t, a, ray, segments, g_theta=None, hashes=None):
        self.tx, self.elem, self.t, self.a, self.ray = tx, elem, t, a, ray
        self.segments = segments
        self.g_theta = g_theta
        self.hashes = hashes

    def splat(self, n_tx: int, n_elem: int, n_t: int, fs: float) -> np.ndarray:
        h = np.zeros((n_tx, n_elem, n_t), dtype=np.float64)
        n = self.t.shape[0]
        if n:
            _load().oracle_splat(n, _ptr(self.tx), _ptr(self.elem), _ptr(self.t), _ptr(self.a),
                                 n_elem, n_t, fs, _ptr(h))
        return h


def trace(scene, probe, angles, tx_ids, seed: int, rays_per_elem: int, max_bounces: int,
          ray_begin: int = 0, ray_count: Optional[int] = None, theta: Optional[np.ndarray] = None,
          nee_mode: int = 0, g_h: Optional[np.ndarray] = None,
          grad_params: Optional[Sequence[int]] = None, want_hashes: bool = False,
          n_threads: int = 0, probs: Optional[np.ndarray] = None,
          record_probs: bool = False, mesh_bruteforce: bool = False) -> TraceResult:
    """FP64 transport of rays [ray_begin, ray_begin + ray_count) of every transmit.

    scene: attributes regions (R,3), planes (P,), plane_regions (P,2), plane_kd (P,),
           spheres (S,4), sphere_regions (S,2), sphere_kd (S,), start_region, theta().
    g_h:   optional dL/dh [n_tx][n_elem][n_t]; then the gradient with respect to
           theta[grad_params] (at most 64 per call) is returned in g_theta.
    record_probs / probs: record the branch probabilities of this call
           (returned as .probs), or reuse given ones; finite differences of the
           estimator with its sampling density held fixed need this.
    scene.meshes (optional): closed triangle meshes with attributes vertices,
           triangles, normals, basis, region_in, region_out, kd.
    scene.cylinders (optional): (C, 3) axes x, z and radii of cylinders along
           y, with cylinder_regions (C, 2) inside / outside and cylinder_kd.
    theta layout: (c, Z, alpha) per region, plane depths, (x, y, z, r) per
           sphere, (x, z, R) per cylinder, GGX roughness per plane, sphere,
           cylinder and mesh, then the mesh displacement coefficients
           [mesh][basis].
    mesh_bruteforce: test every triangle instead of walking the hierarchy.
    """
    lib = _load()
    th = np.ascontiguousarray(scene.theta() if theta is None else theta, dtype=np.float64)
    pr = np.ascontiguousarray(scene.plane_regions, dtype=np.int32).reshape(-1)
    pk = np.ascontiguousarray(scene.plane_kd, dtype=np.float64)
    sr = np.ascontiguousarray(scene.sphere_regions, dtype=np.int32).reshape(-1)
    sk = np.ascontiguousarray(scene.sphere_kd, dtype=np.float64)
    meshes = list(getattr(scene, "meshes", []) or [])
    cyl = np.ascontiguousarray(getattr(scene, "cylinders", np.zeros((0, 3))), dtype=np.float64).reshape(-1, 3)
    cr = np.ascontiguousarray(getattr(scene, "cylinder_regions", np.zeros((0, 2))), dtype=np.int32).reshape(-1)
    ck = np.ascontiguousarray(getattr(scene, "cylinder_kd", np.zeros(0)), dtype=np.float64).reshape(-1)
    n_c = cyl.shape[0]
    if cr.shape[0] != 2 * n_c or ck.shape[0] != n_c:
        raise ValueError("cylinder arrays disagree")
    keep = [pr, pk, sr, sk, cr, ck]
    if meshes:
        vs, ns, bs, vm, ts, tm, off = [], [], [], [], [], [], 0
        for k, mm in enumerate(meshes):
            vs.append(mm.vertices); ns.append(mm.normals); bs.append(mm.basis)
            vm.append(np.full(len(mm.vertices), k, np.int32))
            ts.append(np.asarray(mm.triangles) + off); tm.append(np.full(len(mm.triangles), k, np.int32))
            off += len(mm.vertices)
        arr = [np.ascontiguousarray(np.concatenate(x), dtype=dt) for x, dt in
               ((vs, np.float64), (ns, np.float64), (bs, np.float64), (vm, np.int32), (ts, np.int32), (tm, np.int32))]
        mreg = np.ascontiguousarray([[mm.region_in, mm.region_out] for mm in meshes], dtype=np.int32)
        mkd = np.ascontiguousarray([mm.kd for mm in meshes], dtype=np.float64)
        keep += arr + [mreg, mkd]
        nb = int(arr[2].shape[1])
        mesh_fields = (len(meshes), nb, _ptr(mreg), _ptr(mkd), int(arr[0].shape[0]), int(arr[4].shape[0]),
                       _ptr(arr[0]), _ptr(arr[1]), _ptr(arr[2]), _ptr(arr[3]), _ptr(arr[4]), _ptr(arr[5]))
    else:
        mesh_fields = (0, 0, None, None, 0, 0, None, None, None, None, None, None)
    n_m = len(meshes)
    n_b = int(meshes[0].basis.shape[1]) if meshes else 0
    n_exp = (3 * scene.regions.shape[0] + 2 * scene.planes.shape[0] + 5 * scene.spheres.shape[0]
             + 4 * n_c + n_m + n_m * n_b)
    if th.shape != (n_exp,):
        raise ValueError(f"theta has {th.shape} entries, the scene needs {n_exp}")
    sd = _Scene(int(scene.regions.shape[0]), int(scene.planes.shape[0]),
                int(scene.spheres.shape[0]), _ptr(pr), _ptr(pk), _ptr(sr), _ptr(sk),
                int(scene.start_region), *mesh_fields, 1 if mesh_bruteforce else 0,
                n_c, _ptr(cr) if n_c else None, _ptr(ck) if n_c else None)
    pd = _probe_struct(probe)
    ang = np.ascontiguousarray(angles, dtype=np.float64)
    ids = np.ascontiguousarray(tx_ids, dtype=np.uint32)
    n_tx = ang.shape[0]
    total = int(probe.n_elem) * int(rays_per_elem)
    if ray_count is None:
        ray_count = total - ray_begin
    assert 0 <= ray_begin and ray_begin + ray_count <= total
    prob_mode, pbuf = 0, None
    if probs is not None:
        pbuf = np.ascontiguousarray(probs, dtype=np.float64)
        assert pbuf.shape == (n_tx, ray_count, max_bounces)
        prob_mode = 2
    elif record_probs:
        pbuf = np.full((n_tx, ray_count, max(1, max_bounces)), np.nan)
        prob_mode = 1
    rd = _Run(n_tx, _ptr(ang), _ptr(ids), int(seed), int(rays_per_elem), int(ray_begin),
              int(ray_count), int(max_bounces), int(nee_mode), int(n_threads), prob_mode,
              _ptr(pbuf) if pbuf is not None else None)
    gh = None
    sel = np.zeros(1, dtype=np.int32)
    if g_h is not None:
        gh = np.ascontiguousarray(g_h, dtype=np.float64)
        assert gh.shape == (n_tx, int(probe.n_elem), int(probe.n_t))
        sel = np.ascontiguousarray(grad_params if grad_params is not None
                                   else np.arange(th.shape[0]), dtype=np.int32)
        assert sel.shape[0] <= 64
    hashes = np.zeros((n_tx, ray_count), dtype=np.uint64) if want_hashes else None
    handle = lib.oracle_trace(ctypes.byref(sd), ctypes.byref(pd), ctypes.byref(rd), _ptr(th),
                              _ptr(gh) if gh is not None else None, _ptr(sel),
                              int(sel.shape[0]) if gh is not None else 0,
                              _ptr(hashes) if hashes is not None else None)
    if not handle:
        raise ValueError("oracle_trace rejected its arguments")
    try:
        n = lib.oracle_result_count(handle)
        tx = np.empty(n, np.int32); el = np.empty(n, np.int32)
        t = np.empty(n, np.float64); a = np.empty(n, np.float64); ray = np.empty(n, np.int64)
        g = np.zeros(sel.shape[0], np.float64) if gh is not None else None
        lib.oracle_result_copy(handle, _ptr(tx), _ptr(el), _ptr(t), _ptr(a), _ptr(ray),
                               _ptr(g) if g is not None else None)
        segs = lib.oracle_result_segments(handle)
    finally:
        lib.oracle_result_free(handle)
    g_theta = None
    if g is not None:
        g_theta = np.zeros(th.shape[0], np.float64)
        g_theta[sel] += g
    res = TraceResult(tx, el, t, a, ray, segs, g_theta, hashes)
    res.probs = pbuf if prob_mode == 1 else None
    return res


def philox4x64_10(counter: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.array(counter, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().oracle_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(x: int) -> float:
    return _load().oracle_uniform(int(x))


def interface(w, n, c1, Z1, c2, Z2):
    """(A_r, A_t, R_E, tir), reflected and transmitted directions at one interface."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    coef = np.zeros(4); wr = np.zeros(3); wt = np.zeros(3)
    _load().oracle_interface(_ptr(w), _ptr(n), c1, Z1, c2, Z2, _ptr(coef), _ptr(wr), _ptr(wt))
    return coef, wr, wt


def cosine_dir(n, u1, u2):
    n = np.ascontiguousarray(n, dtype=np.float64)
    out = np.zeros(3)
    _load().oracle_cosine_dir(_ptr(n), float(u1), float(u2), _ptr(out))
    return out


def glossy(w, n, c1, Z1, c2, Z2, rho, u1, u2):
    """Rough (GGX) reflection of w at normal n: (direction, estimator factor, ok)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    out = np.zeros(5)
    _load().oracle_glossy(_ptr(w), _ptr(n), c1, Z1, c2, Z2, float(rho), float(u1), float(u2), _ptr(out))
    return out[:3], out[3], bool(out[4])


def directivity(probe, cos_a: float) -> float:
    pd = _probe_struct(probe)
    return _load().oracle_directivity(ctypes.byref(pd), float(cos_a))


from .chain import *  # noqa: E402,F401,F403
from . import optim  # noqa: E402,F401
