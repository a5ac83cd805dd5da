"""Seeded synthetic workloads: scene, probe, transmit and pixel-grid descriptions.

This module only *describes* inputs. It holds none of the method's arithmetic
(no transport, no Fresnel, no pulse, no beamforming); both the HIP path and the
FP64 oracle take their inputs from here, so it must stay free of either's code.

Units everywhere: metres, seconds, hertz, m/s for sound speed, MRayl for
acoustic impedance, dB/cm/MHz for attenuation, radians for angles.

Parameter vector theta (flat float64), in this order:
  regions  : (c, Z, alpha) for each region
  planes   : depth z for each horizontal interface plane
  spheres  : (cx, cy, cz, r) for each sphere
The layout is what the C-ABI reports from scene upload as well.

Workloads (Sec. 3 of the paper sets the problem; the sizes below are the
synthetic phantoms the build is measured on):
  two_layer()      : water over tissue, flat interface at 30 mm, 64 elements,
                     one 0 deg plane wave, 2^14 rays per element, 4 bounces.
  layered_phantom(): three drawn layers at 10/25/45 mm under a water slab,
                     five drawn diffuse spherical inclusions, 128 elements,
                     11 plane waves over [-10, 10] deg, 2^20 rays per transmit,
                     8 bounces, 4096 samples, 256 x 512 pixels.
  layered_phantom_target(): the same scene with 34 of its parameters moved by
                     a seeded +-5 %, used as the reference image for the
                     forward+backward workload.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# stream tag used for drawing scene parameters (the ray streams use tag 0)
SCENE_STREAM_TAG = 1
TARGET_STREAM_TAG = 2


@dataclasses.dataclass
class Probe:
    """Linear array at z = 0 facing +z (Sec. 2.3.1: aperture, N_e elements, pitch p)."""
    n_elem: int
    pitch: float
    elem_width: float
    elem_height: float
    f0: float
    n_cycles: float
    fs: float
    n_t: int
    c_ref: float
    alpha_main: float = math.radians(20.0)   # receive main-lobe angle (Eq. cutoff)
    alpha_cut: float = math.radians(60.0)    # receive cutoff angle (Eq. cutoff)


@dataclasses.dataclass
class Scene:
    """Regions of homogeneous media bounded by planes z = d and spheres."""
    regions: np.ndarray          # (R, 3) float64: c [m/s], Z [MRayl], alpha [dB/cm/MHz]
    planes: np.ndarray           # (Pl,) float64 depth [m]
    plane_regions: np.ndarray    # (Pl, 2) int32: region above (smaller z), region below
    plane_kd: np.ndarray         # (Pl,) float64 diffuse fraction of reflected energy
    spheres: np.ndarray          # (S, 4) float64: cx, cy, cz, r [m]
    sphere_regions: np.ndarray   # (S, 2) int32: region inside, region outside
    sphere_kd: np.ndarray        # (S,) float64
    start_region: int = 0        # region just below the array face
    meshes: list = dataclasses.field(default_factory=list)   # closed triangle meshes (Mesh)
    mesh_q: Optional[np.ndarray] = None   # (n_meshes, n_basis) displacement coefficients [m]
    plane_rough: Optional[np.ndarray] = None    # (Pl,) GGX roughness (Eq. GGX_PDF); None: 0
    sphere_rough: Optional[np.ndarray] = None   # (S,) GGX roughness; None: 0
    # cylinders along y (the elevation axis): axis at (x, z), radius R
    cylinders: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))   # (C, 3) x, z, R [m]
    cylinder_regions: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 2), np.int32))
    cylinder_kd: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    cylinder_rough: Optional[np.ndarray] = None  # (C,) GGX roughness; None: 0

    @property
    def n_cylinders(self) -> int:
        return int(np.asarray(self.cylinders).reshape(-1, 3).shape[0])

    def roughness(self) -> np.ndarray:
        """Roughness of every plane, sphere, cylinder, then mesh (theta's order)."""
        def arr(x, n):
            return np.zeros(n) if x is None else np.asarray(x, np.float64).reshape(-1)
        rm = np.array([getattr(m, "rough", 0.0) for m in self.meshes], dtype=np.float64)
        return np.concatenate([arr(self.plane_rough, self.n_planes), arr(self.sphere_rough, self.n_spheres),
                               arr(self.cylinder_rough, self.n_cylinders), rm])

    @property
    def n_meshes(self) -> int:
        return len(self.meshes)

    @property
    def n_basis(self) -> int:
        return int(self.meshes[0].basis.shape[1]) if self.meshes else 0

    def q(self) -> np.ndarray:
        if self.mesh_q is not None:
            return np.asarray(self.mesh_q, dtype=np.float64).reshape(self.n_meshes, self.n_basis)
        return np.zeros((self.n_meshes, self.n_basis))

    @property
    def n_regions(self) -> int:
        return int(self.regions.shape[0])

    @property
    def n_planes(self) -> int:
        return int(self.planes.shape[0])

    @property
    def n_spheres(self) -> int:
        return int(self.spheres.shape[0])

    @property
    def n_surfaces(self) -> int:
        return self.n_planes + self.n_spheres + self.n_cylinders + self.n_meshes

    @property
    def rough_offset(self) -> int:
        return 3 * self.n_regions + self.n_planes + 4 * self.n_spheres + 3 * self.n_cylinders

    @property
    def n_params(self) -> int:
        return self.rough_offset + self.n_surfaces + self.n_meshes * self.n_basis

    def theta(self) -> np.ndarray:
        """[(c, Z, alpha) per region, plane depths, (x, y, z, r) per sphere,
        (x, z, R) per cylinder, roughness per plane, sphere, cylinder and
        mesh, mesh basis coefficients]."""
        return np.concatenate([self.regions.reshape(-1), self.planes.reshape(-1),
                               self.spheres.reshape(-1), np.asarray(self.cylinders, np.float64).reshape(-1),
                               self.roughness(), self.q().reshape(-1)]).astype(np.float64)

    def with_theta(self, theta: np.ndarray) -> "Scene":
        theta = np.asarray(theta, dtype=np.float64)
        assert theta.shape == (self.n_params,)
        r, p, s, c, m = self.n_regions, self.n_planes, self.n_spheres, self.n_cylinders, self.n_meshes
        os_ = 3 * r + p
        oc = os_ + 4 * s
        o = self.rough_offset
        rough = theta[o:o + p + s + c + m]
        meshes = [dataclasses.replace(mm, rough=float(rough[p + s + c + k])) for k, mm in enumerate(self.meshes)]
        return dataclasses.replace(
            self,
            regions=theta[:3 * r].reshape(r, 3).copy(),
            planes=theta[3 * r:os_].copy(),
            spheres=theta[os_:oc].reshape(s, 4).copy(),
            cylinders=theta[oc:o].reshape(c, 3).copy(),
            plane_rough=rough[:p].copy(), sphere_rough=rough[p:p + s].copy(),
            cylinder_rough=rough[p + s:p + s + c].copy(), meshes=meshes,
            mesh_q=theta[o + p + s + c + m:].reshape(m, self.n_basis).copy() if self.meshes else None)

    def idx_mesh(self, m: int, j: int) -> int:
        return self.rough_offset + self.n_surfaces + m * self.n_basis + j

    def idx_rough(self, kind: str, k: int) -> int:
        """Roughness of plane / sphere / cylinder / mesh k."""
        base = {"plane": 0, "sphere": self.n_planes, "cylinder": self.n_planes + self.n_spheres,
                "mesh": self.n_planes + self.n_spheres + self.n_cylinders}[kind]
        return self.rough_offset + base + k

    def idx_cylinder(self, k: int, which: str) -> int:
        return 3 * self.n_regions + self.n_planes + 4 * self.n_spheres + 3 * k + {"x": 0, "z": 1, "R": 2}[which]

    # index helpers for the flat parameter vector
    def idx_region(self, k: int, which: str) -> int:
        return 3 * k + {"c": 0, "Z": 1, "alpha": 2}[which]

    def idx_plane(self, k: int) -> int:
        return 3 * self.n_regions + k

    def idx_sphere(self, k: int, which: str) -> int:
        return 3 * self.n_regions + self.n_planes + 4 * k + {"x": 0, "y": 1, "z": 2, "r": 3}[which]


@dataclasses.dataclass
class Grid:
    """Pixel centres x_a = x0 + a*dx, z_b = z0 + b*dz; images are [n_x][n_z]."""
    n_x: int
    n_z: int
    x0: float
    dx: float
    z0: float
    dz: float

    @staticmethod
    def span(n_x: int, n_z: int, x_min: float, x_max: float, z_min: float, z_max: float) -> "Grid":
        dx = (x_max - x_min) / n_x
        dz = (z_max - z_min) / n_z
        return Grid(n_x, n_z, x_min + 0.5 * dx, dx, z_min + 0.5 * dz, dz)

    @property
    def n_px(self) -> int:
        return self.n_x * self.n_z


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    probe: Probe
    angles: np.ndarray            # (n_tx,) steering angles [rad]
    tx_ids: np.ndarray            # (n_tx,) uint32 ids used in the ray counters
    grid: Grid
    seed: int
    rays_per_elem: int
    max_bounces: int
    dr_db: float = 60.0

    @property
    def n_tx(self) -> int:
        return int(self.angles.shape[0])

    @property
    def rays_per_tx(self) -> int:
        return self.probe.n_elem * self.rays_per_elem

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _water():
    return [1480.0, 1.48, 0.0]


def two_layer(rays_per_elem: int = 1 << 14) -> Workload:
    """Water (1480 m/s, 1.48 MRayl) over tissue (1540 m/s, 1.63 MRayl, 0.5 dB/cm/MHz)."""
    scene = Scene(
        regions=np.array([_water(), [1540.0, 1.63, 0.5]], dtype=np.float64),
        planes=np.array([30e-3]),
        plane_regions=np.array([[0, 1]], dtype=np.int32),
        plane_kd=np.array([0.0]),
        spheres=np.zeros((0, 4)),
        sphere_regions=np.zeros((0, 2), dtype=np.int32),
        sphere_kd=np.zeros((0,)),
    )
    probe = Probe(n_elem=64, pitch=0.3e-3, elem_width=0.3e-3, elem_height=5e-3, f0=5e6,
                  n_cycles=2.0, fs=40e6, n_t=2048, c_ref=1480.0)
    grid = Grid.span(128, 256, -19.2e-3, 19.2e-3, 0.0, 40e-3)
    return Workload("two_layer", scene, probe, np.array([0.0]), np.array([0], dtype=np.uint32),
                    grid, seed=0, rays_per_elem=rays_per_elem, max_bounces=4)


def _layered_scene(seed: int) -> Scene:
    rng = np.random.Generator(np.random.Philox(key=[seed, SCENE_STREAM_TAG]))
    depths = [10e-3, 25e-3, 45e-3]
    layer_span = [(10e-3, 25e-3), (25e-3, 45e-3), (45e-3, 58e-3)]

    def draw_medium():
        return [rng.uniform(1450.0, 1600.0), rng.uniform(1.3, 1.8), rng.uniform(0.3, 1.0)]

    regions = [_water()] + [draw_medium() for _ in range(3)]
    spheres, sph_regions = [], []
    while len(spheres) < 5:
        r = rng.uniform(2e-3, 6e-3)
        layer = int(rng.integers(0, 3))
        lo, hi = layer_span[layer]
        lo, hi = lo + r + 0.5e-3, hi - r - 0.5e-3
        if hi <= lo:
            continue
        cx, cz = rng.uniform(-15e-3, 15e-3), rng.uniform(lo, hi)
        if any(math.hypot(cx - s[0], cz - s[2]) < r + s[3] + 0.5e-3 for s in spheres):
            continue
        spheres.append([cx, 0.0, cz, r])
        sph_regions.append([4 + len(sph_regions), 1 + layer])
        regions.append(draw_medium())
    return Scene(
        regions=np.array(regions, dtype=np.float64),
        planes=np.array(depths),
        plane_regions=np.array([[0, 1], [1, 2], [2, 3]], dtype=np.int32),
        plane_kd=np.zeros(3),
        spheres=np.array(spheres, dtype=np.float64),
        sphere_regions=np.array(sph_regions, dtype=np.int32),
        sphere_kd=np.full(5, 0.2),
    )


def layered_probe() -> Probe:
    return Probe(n_elem=128, pitch=0.3e-3, elem_width=0.3e-3, elem_height=5e-3, f0=5e6,
                 n_cycles=2.0, fs=40e6, n_t=4096, c_ref=1540.0)


def layered_phantom(seed: int = 1, rays_per_tx: int = 1 << 20, n_tx: int = 11) -> Workload:
    probe = layered_probe()
    angles = np.radians(np.linspace(-10.0, 10.0, n_tx))
    grid = Grid.span(256, 512, -19.2e-3, 19.2e-3, 0.0, 60e-3)
    return Workload("layered_phantom", _layered_scene(seed), probe, angles,
                    np.arange(n_tx, dtype=np.uint32), grid, seed=0,
                    rays_per_elem=rays_per_tx // probe.n_elem, max_bounces=8)


def cylinder_phantom(radius: float = 5e-3, depth: float = 15e-3, Z: float = 1.7, rough: float = 0.15,
                     kd: float = 0.1, rays_per_tx: int = 1 << 20, n_tx: int = 5) -> Workload:
    """The hollow-cylinder scene of the paper's forward check and its
    simulated-reference inversion: a cylindrical interface of radius 5 mm
    along the elevation axis, its axis 15 mm below the array (reading), water
    outside and a tissue-like medium of impedance Z inside (1540 m/s,
    0.5 dB/cm/MHz), GGX roughness 0.15 and a Lambertian share 0.1; the
    128-element probe of the layered phantom with its delays at the water
    speed, 5 plane waves over [-10, 10] degrees, 128 x 256 pixels over
    +-12.8 mm x [0, 30] mm."""
    scene = Scene(
        regions=np.array([_water(), [1540.0, Z, 0.5]], dtype=np.float64),
        planes=np.zeros(0), plane_regions=np.zeros((0, 2), dtype=np.int32), plane_kd=np.zeros(0),
        spheres=np.zeros((0, 4)), sphere_regions=np.zeros((0, 2), dtype=np.int32), sphere_kd=np.zeros(0),
        cylinders=np.array([[0.0, depth, radius]]), cylinder_regions=np.array([[1, 0]], dtype=np.int32),
        cylinder_kd=np.array([kd]), cylinder_rough=np.array([rough]))
    probe = dataclasses.replace(layered_probe(), c_ref=1480.0)   # delays at the water speed
    angles = np.radians(np.linspace(-10.0, 10.0, n_tx))
    grid = Grid.span(128, 256, -12.8e-3, 12.8e-3, 0.0, 30e-3)
    return Workload("cylinder_phantom", scene, probe, angles, np.arange(n_tx, dtype=np.uint32), grid,
                    seed=0, rays_per_elem=rays_per_tx // probe.n_elem, max_bounces=8)


ROUGH_STREAM_TAG = 4


def rough_layered_phantom(seed: int = 1, rays_per_tx: int = 1 << 20, n_tx: int = 11) -> Workload:
    """The layered phantom with rough interfaces (Eq. GGX_PDF): plane
    roughness U[0.02, 0.15], sphere roughness U[0.1, 0.4], seeded."""
    wl = layered_phantom(seed, rays_per_tx, n_tx)
    rng = np.random.Generator(np.random.Philox(key=[seed, ROUGH_STREAM_TAG]))
    sc = wl.scene
    scene = dataclasses.replace(sc, plane_rough=rng.uniform(0.02, 0.15, sc.n_planes),
                                sphere_rough=rng.uniform(0.1, 0.4, sc.n_spheres))
    return wl.replace(name="rough_layered_phantom", scene=scene)


def perturbed_indices(scene: Scene) -> List[int]:
    """The 34 perturbed parameters: (c, Z, alpha) of every non-water region, then
    every sphere's depth and radius."""
    idx = [scene.idx_region(k, w) for k in range(1, scene.n_regions) for w in ("c", "Z", "alpha")]
    idx += [scene.idx_sphere(k, "z") for k in range(scene.n_spheres)]
    idx += [scene.idx_sphere(k, "r") for k in range(scene.n_spheres)]
    return idx


def layered_phantom_target(wl: Workload, seed: int = 1) -> Scene:
    """theta_target_j = theta_j * (1 + 0.05 (2u_j - 1)) on the perturbed set; redrawn
    if a sphere would leave its layer or touch another sphere."""
    rng = np.random.Generator(np.random.Philox(key=[seed, TARGET_STREAM_TAG]))
    sc = wl.scene
    theta0 = sc.theta()
    idx = perturbed_indices(sc)
    bounds = {1: (10e-3, 25e-3), 2: (25e-3, 45e-3), 3: (45e-3, 58e-3)}
    while True:
        theta = theta0.copy()
        theta[idx] *= 1.0 + 0.05 * (2.0 * rng.random(len(idx)) - 1.0)
        cand = sc.with_theta(theta)
        ok = True
        for k in range(cand.n_spheres):
            cx, _, cz, r = cand.spheres[k]
            lo, hi = bounds[int(cand.sphere_regions[k, 1])]
            if cz - r < lo + 0.25e-3 or cz + r > hi - 0.25e-3:
                ok = False
            for j in range(k):
                d = math.hypot(cx - cand.spheres[j, 0], cz - cand.spheres[j, 2])
                if d < r + cand.spheres[j, 3] + 0.25e-3:
                    ok = False
        if ok:
            return cand


def tiny(workload: Workload, rays_per_elem: int, n_elem: Optional[int] = None,
         n_t: Optional[int] = None, grid: Optional[Grid] = None) -> Workload:
    """A reduced copy of a workload (fewer rays/elements/samples) for fast parity runs."""
    probe = workload.probe
    if n_elem is not None:
        probe = dataclasses.replace(probe, n_elem=n_elem)
    if n_t is not None:
        probe = dataclasses.replace(probe, n_t=n_t)
    return workload.replace(probe=probe, rays_per_elem=rays_per_elem,
                            grid=grid if grid is not None else workload.grid)


def with_grid(wl: Workload, n_x: int, n_z: int) -> Workload:
    """Same field of view, another pixel count."""
    g = wl.grid
    x_min, x_max = g.x0 - 0.5 * g.dx, g.x0 + (g.n_x - 0.5) * g.dx
    z_min, z_max = g.z0 - 0.5 * g.dz, g.z0 + (g.n_z - 0.5) * g.dz
    return wl.replace(grid=Grid.span(n_x, n_z, x_min, x_max, z_min, z_max))


@dataclasses.dataclass
class ServingRequestSpec:
    workload: Workload
    want_grad: bool
    target: Optional[Scene]      # scene of the reference image for gradient requests
    total_rays: int


def serving_requests(n: int = 512, seed: int = 4, generators=None, min_log2_rays: int = 14,
                     max_log2_rays: int = 24) -> List[ServingRequestSpec]:
    """Serving stream: scenes drawn 40/40/20 from the generators (default: the
    two-layer, layered-phantom and mesh anatomy generators), ray counts
    2^U{min..max} per frame, grids from {128x256, 256x512, 512x1024}, 30 % of
    the requests ask for the gradient of the B-mode MSE against the image of a
    seeded +-5 % perturbation of their scene. Scene descriptions are shared
    between requests of the same draw, so a server keeps them resident."""
    rng = np.random.Generator(np.random.Philox(key=[seed, 5]))
    if generators is None:
        base = [two_layer(), layered_phantom(seed=1), anatomy_phantom()]
    else:
        base = generators
    weights = np.array([0.4, 0.4, 0.2])[:len(base)]
    weights = weights / weights.sum()
    targets = {}
    grids = [(128, 256), (256, 512), (512, 1024)]
    out = []
    for i in range(n):
        k = int(rng.choice(len(base), p=weights))
        wl = base[k]
        total = 1 << int(rng.integers(min_log2_rays, max_log2_rays + 1))
        rpe = max(1, total // (wl.probe.n_elem * wl.n_tx))
        gx, gz = grids[int(rng.integers(0, len(grids)))]
        want_grad = bool(rng.random() < 0.3)
        target = None
        if want_grad:
            if k not in targets:
                if wl.scene.meshes:
                    targets[k] = anatomy_phantom_target(wl, seed=seed + k)
                elif wl.scene.n_spheres:
                    targets[k] = layered_phantom_target(wl, seed=seed + k)
                else:   # perturb every region's (c, Z, alpha) and the plane depths
                    r2 = np.random.Generator(np.random.Philox(key=[seed + k, TARGET_STREAM_TAG]))
                    th = wl.scene.theta()
                    th = th * (1.0 + 0.05 * (2.0 * r2.random(th.shape[0]) - 1.0))
                    targets[k] = wl.scene.with_theta(th)
            target = targets[k]
        out.append(ServingRequestSpec(with_grid(wl.replace(rays_per_elem=rpe), gx, gz), want_grad,
                                      target, rpe * wl.probe.n_elem * wl.n_tx))
    return out


# ----------------------------------------------------------------------------
# Triangle meshes: closed, outward-oriented, each with a displacement basis.
# A vertex moves as v = v_rest + sum_j q_j phi_j(v_rest) n_rest, where q (one
# coefficient per basis function and mesh, in metres) is part of theta.
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Mesh:
    vertices: np.ndarray      # (V, 3) float64 rest positions [m]
    triangles: np.ndarray     # (T, 3) int32, counter-clockwise seen from outside
    normals: np.ndarray       # (V, 3) float64 unit displacement directions
    basis: np.ndarray         # (V, nb) float64 basis weights phi_j(v)
    region_in: int
    region_out: int
    kd: float
    rough: float = 0.0        # GGX roughness (Eq. GGX_PDF)


def _orient_outward(v, f, inside_point):
    c = v[f].mean(axis=1)
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    flip = np.einsum("ij,ij->i", n, c - inside_point) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return f


def _vertex_normals(v, f):
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])   # area-weighted
    vn = np.zeros_like(v)
    for k in range(3):
        np.add.at(vn, f[:, k], n)
    return vn / np.linalg.norm(vn, axis=1, keepdims=True)


def icosphere(level: int):
    """Unit icosphere: 20 * 4^level faces."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t],
         [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]]
    f = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4],
         [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    v = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = np.array(f, dtype=np.int64)
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]
        nf = []
        for a, b, c in faces.tolist():
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        faces = np.array(nf, dtype=np.int64)
    V = np.array(v)
    return V, _orient_outward(V, faces, np.zeros(3)).astype(np.int32)


def _fibonacci_sphere(n):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


def blob_mesh(center, radius, level, rng, noise=0.08, n_basis=16, region_in=1, region_out=0,
              kd=0.2, basis_width=0.35) -> Mesh:
    """Icosphere displaced radially by smooth seeded noise (a few Gaussian bumps)."""
    u, f = icosphere(level)
    bumps = _fibonacci_sphere(8) @ np.linalg.qr(rng.standard_normal((3, 3)))[0]
    amp = noise * (2 * rng.random(8) - 1)
    r = 1.0 + sum(a * np.exp(-np.sum((u - b) ** 2, 1) / (2 * 0.4 ** 2)) for a, b in zip(amp, bumps))
    v = np.asarray(center) + radius * r[:, None] * u
    centres = _fibonacci_sphere(n_basis)
    basis = np.exp(-((u[:, None, :] - centres[None, :, :]) ** 2).sum(-1) / (2 * basis_width ** 2))
    return Mesh(v, f, _vertex_normals(v, f), basis, region_in, region_out, kd)


def tube_mesh(center, radius, half_length, n_around, n_along, n_basis=16, region_in=1, region_out=0,
              kd=0.2) -> Mesh:
    """Closed tube along y (a vessel crossing the image plane) with flat caps."""
    ang = 2 * np.pi * np.arange(n_around) / n_around
    ys = np.linspace(-half_length, half_length, n_along + 1)
    cx, cy, cz = center
    ring = np.stack([np.cos(ang), np.sin(ang)], 1)
    v = [[cx + radius * c, cy + y, cz + radius * s] for y in ys for c, s in ring]
    f = []
    for i in range(n_along):
        for j in range(n_around):
            a, b = i * n_around + j, i * n_around + (j + 1) % n_around
            c, d = a + n_around, b + n_around
            f += [[a, b, d], [a, d, c]]
    base = len(v)
    v += [[cx, cy - half_length, cz], [cx, cy + half_length, cz]]
    top = n_along * n_around
    for j in range(n_around):
        f.append([base, (j + 1) % n_around, j])
        f.append([base + 1, top + j, top + (j + 1) % n_around])
    V = np.array(v, dtype=np.float64)
    F = _orient_outward(V, np.array(f), np.asarray(center, dtype=np.float64))
    rel = V - np.asarray(center)
    ay, az = np.meshgrid(np.linspace(-half_length, half_length, 4), np.arange(4) * np.pi / 2, indexing="ij")
    angle = np.arctan2(rel[:, 2], rel[:, 0])
    basis = np.stack([np.exp(-(rel[:, 1] - y0) ** 2 / (2 * (half_length / 3) ** 2)
                             - (1 - np.cos(angle - a0)) / (2 * 0.5 ** 2))
                      for y0, a0 in zip(ay.ravel(), az.ravel())], 1)[:, :n_basis]
    return Mesh(V, F.astype(np.int32), _vertex_normals(V, F), basis, region_in, region_out, kd)


def mesh_arrays(scene: Scene) -> dict:
    """The scene's meshes concatenated: rest vertices, displacement normals,
    basis weights, per-vertex and per-triangle mesh ids, global triangles."""
    if not scene.meshes:
        z = np.zeros
        return dict(vertices=z((0, 3)), normals=z((0, 3)), basis=z((0, 0)), vmesh=z(0, np.int32),
                    triangles=z((0, 3), np.int32), tmesh=z(0, np.int32),
                    regions=z((0, 2), np.int32), kd=z(0))
    vs, ns, bs, vm, ts, tm = [], [], [], [], [], []
    off = 0
    for k, m in enumerate(scene.meshes):
        vs.append(m.vertices); ns.append(m.normals); bs.append(m.basis)
        vm.append(np.full(len(m.vertices), k, np.int32))
        ts.append(m.triangles + off); tm.append(np.full(len(m.triangles), k, np.int32))
        off += len(m.vertices)
    return dict(vertices=np.concatenate(vs), normals=np.concatenate(ns), basis=np.concatenate(bs),
                vmesh=np.concatenate(vm), triangles=np.concatenate(ts).astype(np.int32),
                tmesh=np.concatenate(tm),
                regions=np.array([[m.region_in, m.region_out] for m in scene.meshes], np.int32),
                kd=np.array([m.kd for m in scene.meshes]))


def anatomy_probe() -> Probe:
    return Probe(n_elem=192, pitch=0.2e-3, elem_width=0.2e-3, elem_height=5e-3, f0=7.5e6,
                 n_cycles=2.0, fs=60e6, n_t=8192, c_ref=1540.0)


def anatomy_scene(seed: int = 3, level_organ: int = 6, level_lesion: int = 5,
                  tube_around: int = 128, tube_along: int = 190) -> Scene:
    """Nested closed meshes: an organ (noise-displaced icosphere, radius 14 mm,
    centre 40 mm deep) holding a lesion (icosphere, 4 mm) and a vessel (capped
    tube across the image plane, 1.5 mm), and a second vessel (2.5 mm) below
    the organ in the background tissue. Defaults give 200,192 triangles."""
    rng = np.random.Generator(np.random.Philox(key=[seed, SCENE_STREAM_TAG]))

    def medium(c, z, a):
        return [rng.uniform(*c), rng.uniform(*z), rng.uniform(*a)]

    regions = [[1540.0, 1.63, 0.5],                                   # background tissue
               medium((1560, 1600), (1.60, 1.75), (0.5, 0.9)),        # organ
               medium((1450, 1520), (1.35, 1.50), (0.3, 0.6)),        # lesion
               medium((1560, 1590), (1.58, 1.65), (0.1, 0.2)),        # vessel in the organ
               medium((1560, 1590), (1.58, 1.65), (0.1, 0.2))]        # vessel in the background
    meshes = [
        blob_mesh([0.0, 0.0, 40e-3], 14e-3, level_organ, rng, noise=0.06, region_in=1, region_out=0),
        blob_mesh([-5e-3, 0.0, 44e-3], 4e-3, level_lesion, rng, noise=0.08, region_in=2, region_out=1),
        tube_mesh([6e-3, 0.0, 35e-3], 1.5e-3, 6e-3, tube_around, tube_along, region_in=3, region_out=1),
        tube_mesh([-12e-3, 0.0, 64e-3], 2.5e-3, 8e-3, tube_around, tube_along, region_in=4, region_out=0),
    ]
    return Scene(regions=np.array(regions, dtype=np.float64), planes=np.zeros(0),
                 plane_regions=np.zeros((0, 2), np.int32), plane_kd=np.zeros(0),
                 spheres=np.zeros((0, 4)), sphere_regions=np.zeros((0, 2), np.int32),
                 sphere_kd=np.zeros(0), meshes=meshes)


def anatomy_phantom(seed: int = 3, rays_per_elem: int = 4161, **mesh_kw) -> Workload:
    """Triangle-mesh anatomy: 192 elements x 0.2 mm, 7.5 MHz, 60 MHz, 21 plane
    waves over [-10, 10] deg, 4161 rays per element and transmit (16,777,152 per
    frame), 12 interactions, 8192 samples, 512 x 1024 pixels over 38.4 x 76.8 mm."""
    probe = anatomy_probe()
    angles = np.radians(np.linspace(-10.0, 10.0, 21))
    grid = Grid.span(512, 1024, -19.2e-3, 19.2e-3, 0.0, 76.8e-3)
    return Workload("anatomy_phantom", anatomy_scene(seed, **mesh_kw), probe, angles,
                    np.arange(21, dtype=np.uint32), grid, seed=0, rays_per_elem=rays_per_elem,
                    max_bounces=12)


def anatomy_phantom_target(wl: Workload, seed: int = 3, dq: float = 0.3e-3) -> Scene:
    """Target scene of the mesh workload: every region's (c, Z, alpha) times
    (1 + 0.05 (2u - 1)) and every displacement coefficient moved by
    dq (2u - 1) metres (u uniform from the target stream)."""
    rng = np.random.Generator(np.random.Philox(key=[seed, TARGET_STREAM_TAG]))
    sc = wl.scene
    theta = sc.theta().copy()
    nr = 3 * sc.n_regions
    theta[:nr] *= 1.0 + 0.05 * (2.0 * rng.random(nr) - 1.0)
    if sc.meshes:
        q0 = sc.idx_mesh(0, 0)
        theta[q0:] += dq * (2.0 * rng.random(theta.shape[0] - q0) - 1.0)
    return sc.with_theta(theta)