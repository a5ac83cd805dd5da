"""Pins of the oracle's triangle-mesh path: the hierarchy walk against a
linear scan, a closed box mesh against the (already pinned) analytic planes it
coincides with, and mesh-displacement gradients against finite differences
and against the plane-depth gradient. CPU only."""
import numpy as np
import pytest

import oracle
from paper_2604_15017_amd import workloads as W


def _mesh_scene(meshes, regions):
    return W.Scene(regions=np.array(regions, dtype=np.float64), planes=np.zeros(0),
                   plane_regions=np.zeros((0, 2), np.int32), plane_kd=np.zeros(0),
                   spheres=np.zeros((0, 4)), sphere_regions=np.zeros((0, 2), np.int32),
                   sphere_kd=np.zeros(0), meshes=meshes)


def _small_anatomy(rays_per_elem=16, kd=0.2):
    rng = np.random.default_rng(0)
    meshes = [W.blob_mesh([0, 0, 25e-3], 8e-3, 3, rng, region_in=1, region_out=0, kd=kd),
              W.tube_mesh([3e-3, 0, 26e-3], 1.5e-3, 4e-3, 24, 10, region_in=2, region_out=1, kd=kd)]
    sc = _mesh_scene(meshes, [[1540, 1.63, 0.5], [1580, 1.75, 0.7], [1500, 1.45, 0.4]])
    return W.anatomy_phantom(level_organ=1, level_lesion=1, tube_around=8, tube_along=2).replace(
        scene=sc, rays_per_elem=rays_per_elem, angles=np.radians([-6.0, 4.0]),
        tx_ids=np.arange(2, dtype=np.uint32), max_bounces=6)


def _key(tr):
    o = np.lexsort((tr.t, tr.elem, tr.tx, tr.ray))
    return tr.ray[o], tr.elem[o], tr.t[o], tr.a[o]


def test_hierarchy_equals_linear_scan():
    wl = _small_anatomy()
    a = oracle.trace(wl.scene, wl.probe, wl.angles, wl.tx_ids, 0, wl.rays_per_elem, wl.max_bounces,
                     want_hashes=True)
    b = oracle.trace(wl.scene, wl.probe, wl.angles, wl.tx_ids, 0, wl.rays_per_elem, wl.max_bounces,
                     want_hashes=True, mesh_bruteforce=True)
    assert len(a.t) > 1000 and a.segments == b.segments
    assert np.array_equal(a.hashes, b.hashes)
    for x, y in zip(_key(a), _key(b)):
        assert np.array_equal(x, y)


def box_mesh(z0, z1, half=0.5, region_in=1, region_out=0):
    """Closed axis-aligned box; only the top face (z = z0) moves with the one
    basis function, along -z (outward)."""
    v = np.array([[x, y, z] for z in (z0, z1) for y in (-half, half) for x in (-half, half)], dtype=np.float64)
    f = np.array([[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1],
                  [2, 3, 7], [2, 7, 6], [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]])
    f = W._orient_outward(v, f, np.array([0.0, 0.0, 0.5 * (z0 + z1)])).astype(np.int32)
    normals = np.tile([0.0, 0.0, -1.0], (8, 1))
    basis = (np.abs(v[:, 2] - z0) < 1e-12).astype(np.float64)[:, None]
    return W.Mesh(v, f, normals, basis, region_in, region_out, 0.0)


def test_box_mesh_equals_two_planes():
    z0, z1 = 12e-3, 31e-3
    regions = [[1480.0, 1.48, 0.0], [1560.0, 1.7, 0.6]]
    planes = W.Scene(regions=np.array(regions), planes=np.array([z0, z1]),
                     plane_regions=np.array([[0, 1], [1, 0]], np.int32), plane_kd=np.zeros(2),
                     spheres=np.zeros((0, 4)), sphere_regions=np.zeros((0, 2), np.int32),
                     sphere_kd=np.zeros(0))
    box = _mesh_scene([box_mesh(z0, z1)], regions)
    wl = W.layered_phantom().replace(rays_per_elem=64, angles=np.radians([-8.0, 3.0]),
                                     tx_ids=np.arange(2, dtype=np.uint32), max_bounces=5)
    a = oracle.trace(planes, wl.probe, wl.angles, wl.tx_ids, 1, 64, 5)
    b = oracle.trace(box, wl.probe, wl.angles, wl.tx_ids, 1, 64, 5)
    assert a.segments == b.segments and len(a.t) == len(b.t) > 100
    ka, kb = _key(a), _key(b)
    assert np.array_equal(ka[0], kb[0]) and np.array_equal(ka[1], kb[1])
    assert np.allclose(ka[2], kb[2], rtol=1e-13, atol=0) and np.allclose(ka[3], kb[3], rtol=1e-11, atol=0)
    # gradients: moving the top face outward by q is moving plane 0 by -q
    p = wl.probe
    rng = np.random.default_rng(2)
    g_h = rng.standard_normal((2, p.n_elem, p.n_t))
    ga = oracle.trace(planes, p, wl.angles, wl.tx_ids, 1, 64, 5, g_h=g_h).g_theta
    gb = oracle.trace(box, p, wl.angles, wl.tx_ids, 1, 64, 5, g_h=g_h).g_theta
    assert np.allclose(gb[:6], ga[:6], rtol=1e-9, atol=1e-12 * np.abs(ga).max())
    assert gb[box.idx_mesh(0, 0)] == pytest.approx(-ga[planes.idx_plane(0)], rel=1e-9)
    # one roughness for both faces of the box: the sum of the two planes' roughness gradients
    g_rho = ga[planes.idx_rough("plane", 0)] + ga[planes.idx_rough("plane", 1)]
    assert abs(g_rho) > 1e-6 * np.abs(ga).max()
    assert gb[box.idx_rough("mesh", 0)] == pytest.approx(g_rho, rel=1e-9)


def test_mesh_displacement_gradient_matches_finite_differences():
    wl = _small_anatomy(rays_per_elem=24)
    p, sc = wl.probe, wl.scene
    theta = sc.theta()
    k = np.exp(-0.5 * (np.arange(-30, 31) / 10.0) ** 2)
    rng = np.random.default_rng(5)
    g_h = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1,
                              rng.standard_normal((wl.n_tx, p.n_elem, p.n_t)))
    probs = oracle.trace(sc, p, wl.angles, wl.tx_ids, 0, wl.rays_per_elem, wl.max_bounces,
                         theta=theta, record_probs=True).probs
    idx = [sc.idx_mesh(m, j) for m in range(2) for j in range(16)] + [3, 4, 5, 6, 7, 8]
    ad = oracle.trace(sc, p, wl.angles, wl.tx_ids, 0, wl.rays_per_elem, wl.max_bounces, theta=theta,
                      g_h=g_h, grad_params=idx).g_theta

    def L(th):
        tr = oracle.trace(sc, p, wl.angles, wl.tx_ids, 0, wl.rays_per_elem, wl.max_bounces,
                          theta=th, probs=probs)
        return float(np.sum(g_h * tr.splat(wl.n_tx, p.n_elem, p.n_t, p.fs)))

    unit = np.where(theta != 0, np.abs(theta), 1e-3)
    scale = max(abs(ad[j]) * unit[j] for j in idx)
    n_sig = 0
    for j in idx:
        h = 1e-7 * unit[j] if theta[j] != 0 else 1e-10
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h; tm[j] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        assert abs(fd - ad[j]) * unit[j] <= 1e-3 * abs(ad[j]) * unit[j] + 1e-7 * scale, (j, fd, ad[j])
        n_sig += abs(ad[j]) * unit[j] > 1e-3 * scale
    assert n_sig >= 12
