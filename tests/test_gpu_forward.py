"""GPU parity of the forward path through the C-ABI against the FP64 oracle.

Tolerances: RF relative L2 <= 1e-4; B-mode <= 0.05 dB wherever either image
is above the -60 dB floor; paths whose discrete decisions differ (per-ray
decision hashes) <= 1e-5 of all rays; segment counts identical."""
import numpy as np
import pytest

import oracle
from paper_2604_15017_amd import workloads as W

pytestmark = pytest.mark.gpu

RF_TOL = 1e-4
DB_TOL = 0.05


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_2604_15017_amd import _lib
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return _lib


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def db_err(a, b, dr=60.0):
    live = (a > -dr) | (b > -dr)
    return float(np.abs(a - b)[live].max()) if live.any() else 0.0


def gpu_trace(L, ctx, wl, audit=False, ray_begin=0, ray_count=None, workspace=None):
    import torch
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    if ray_count is None:
        ray_count = wl.rays_per_tx - ray_begin
    counters = torch.zeros(5, dtype=torch.int64, device="cuda")
    hashes = torch.zeros((wl.n_tx, ray_count), dtype=torch.int64, device="cuda") if audit else None
    rf = L.us_simulate_rf(ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                          wl.max_bounces, ray_begin=ray_begin, ray_count=ray_count,
                          counters=counters, ray_hash=hashes, workspace=workspace)
    torch.cuda.synchronize()
    out = dict(rf=rf.cpu().numpy().astype(np.float64), counters=counters.cpu().numpy())
    if audit:
        out["hashes"] = hashes.cpu().numpy().view(np.uint64)
    return out


def check_transport(L, ctx, wl, **kw):
    g = gpu_trace(L, ctx, wl, audit=True, **kw)
    rf, h, tr = oracle.simulate_rf(wl, want_hashes=True, **kw)
    rel = rel_l2(g["rf"], rf)
    flips = int(np.count_nonzero(g["hashes"] != tr.hashes))
    frac = flips / tr.hashes.size
    print(f"{wl.name}: rf rel-L2 {rel:.3e}, flipped paths {flips}/{tr.hashes.size}, "
          f"segments gpu {g['counters'][0] + g['counters'][1]} oracle {tr.segments}", flush=True)
    assert frac <= 1e-5
    assert rel <= RF_TOL
    if flips == 0:
        assert g["counters"][0] + g["counters"][1] == tr.segments
        assert g["counters"][2] == tr.t.shape[0]
    return g, rf


def test_two_layer_full_size(L, ctx):
    check_transport(L, ctx, W.two_layer())


def test_layered_phantom_reduced_rays(L, ctx):
    wl = W.layered_phantom()
    check_transport(L, ctx, wl.replace(rays_per_elem=128))


def test_rough_layered_phantom(L, ctx):
    """Rough planes and spheres (Eq. GGX_PDF): glossy reflections, the paths
    they end, and their direct deposits."""
    check_transport(L, ctx, W.rough_layered_phantom().replace(rays_per_elem=128))


def test_rough_layered_phantom_full_size(L, ctx):
    check_transport(L, ctx, W.rough_layered_phantom())


def test_cylinder_phantom_full_size(L, ctx):
    """The hollow cylinder (radius, axis, roughness, Lambertian share): 5 x 2^20 rays."""
    check_transport(L, ctx, W.cylinder_phantom())


def test_cylinder_walls_in_the_bmode_image(L, ctx):
    """The paper's forward check: in the B-mode image of the hollow cylinder
    (R = 5 mm, axis 15 mm deep) the brightest pixel of the central columns is
    the near wall at z_c - R, and the far wall, seen through the cylinder's
    medium with the delays of the water speed, at z_c - R + 2 R c_water / c_in;
    the measured diameter (c_in / c_water times the wall distance) is 2 R to
    within a pixel."""
    import torch
    wl = W.cylinder_phantom()
    sc, g = wl.scene, wl.grid
    _, zc, R = sc.cylinders[0]
    c_w, c_in = sc.regions[0, 0], sc.regions[1, 0]
    scene, probe = L.Scene(ctx, sc), L.Probe(ctx, wl.probe)
    rf = L.us_simulate_rf(ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces)
    iq = L.us_beamform(ctx, probe, wl.grid, wl.angles, wl.tx_ids, rf)
    B = L.us_bmode(ctx, iq, wl.dr_db)
    torch.cuda.synchronize()
    B = B.cpu().numpy()
    x = g.x0 + g.dx * np.arange(g.n_x)
    z = g.z0 + g.dz * np.arange(g.n_z)
    col = B[np.abs(x) < 0.5e-3].max(axis=0)          # central columns, per depth
    z_near = z[np.argmax(np.where(z < zc, col, -np.inf))]
    z_far = z[np.argmax(np.where(z > zc, col, -np.inf))]
    print(f"near wall {z_near * 1e3:.3f} mm (expected {(zc - R) * 1e3:.3f}), far wall {z_far * 1e3:.3f} mm "
          f"(expected {(zc - R + 2 * R * c_w / c_in) * 1e3:.3f}), peaks {col.max():.1f} dB", flush=True)
    assert abs(z_near - (zc - R)) <= 1.5 * g.dz
    assert abs(z_far - (zc - R + 2 * R * c_w / c_in)) <= 2.5 * g.dz
    assert abs((z_far - z_near) * c_in / c_w - 2 * R) <= 3 * g.dz


def test_layered_phantom_full_size(L, ctx):
    """The benchmark workload itself: 11 transmits x 2^20 rays, 8 bounces."""
    check_transport(L, ctx, W.layered_phantom())


def test_ragged_ray_range_and_subsets_add_up(L, ctx):
    wl = W.layered_phantom().replace(rays_per_elem=64, angles=np.radians([-7.0, 3.0]),
                                     tx_ids=np.array([4, 9], dtype=np.uint32))
    n = wl.rays_per_tx
    # a ragged range that is not a multiple of the block or wave size
    check_transport(L, ctx, wl, ray_begin=37, ray_count=n - 37 - 1001)
    a = gpu_trace(L, ctx, wl, ray_begin=0, ray_count=3001)["rf"]
    b = gpu_trace(L, ctx, wl, ray_begin=3001, ray_count=n - 3001)["rf"]
    full = gpu_trace(L, ctx, wl)["rf"]
    assert rel_l2(a + b, full) <= 1e-6


def test_empty_ray_range_and_zero_bounces(L, ctx):
    wl = W.layered_phantom().replace(rays_per_elem=16, angles=np.radians([0.0]),
                                     tx_ids=np.array([0], dtype=np.uint32))
    g = gpu_trace(L, ctx, wl, ray_begin=5, ray_count=0)
    assert not g["rf"].any() and g["counters"].sum() == 0
    wl0 = wl.replace(max_bounces=0)
    g0 = gpu_trace(L, ctx, wl0)
    rf0, _, tr0 = oracle.simulate_rf(wl0)
    assert not g0["rf"].any() and not rf0.any()
    assert g0["counters"][0] == tr0.segments


def test_small_workspace_forces_chunks(L, ctx):
    import torch
    wl = W.layered_phantom().replace(rays_per_elem=96, angles=np.radians([-10.0, 0.0, 10.0]),
                                     tx_ids=np.arange(3, dtype=np.uint32))
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    need = L.us_simulate_rf_workspace_size(scene, probe, wl.n_tx, wl.rays_per_tx, wl.max_bounces)
    hist = wl.n_tx * wl.probe.n_elem * wl.probe.n_t * 8 + 4096   # fixed-point histogram + counters
    small = hist + (need - hist) // 7                             # queues for ~1/7 of the rays
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    g_small = gpu_trace(L, ctx, wl, workspace=ws)["rf"]
    g_full = gpu_trace(L, ctx, wl)["rf"]
    # the same integer additions grouped by chunk: the same bits
    assert np.array_equal(g_small, g_full)
    rf, _, _ = oracle.simulate_rf(wl)
    assert rel_l2(g_small, rf) <= RF_TOL


def test_deposits_beyond_the_record_buffer(L, ctx):
    """Twelve weakly reflecting, half-diffuse layers of equal sound speed: each
    ray crosses them all and sends a secondary ray at every crossing, about 10
    deposits per ray, more than the binned splat records (2 per ray); the rest
    take the direct path and the RF still matches the oracle."""
    n = 12
    regions = np.array([[1540.0, 1.5 + 0.05 * (i % 2), 0.3] for i in range(n + 1)])
    sc = W.Scene(regions=regions, planes=np.linspace(2e-3, 24e-3, n),
                 plane_regions=np.array([[i, i + 1] for i in range(n)], np.int32),
                 plane_kd=np.full(n, 0.5), spheres=np.zeros((0, 4)),
                 sphere_regions=np.zeros((0, 2), np.int32), sphere_kd=np.zeros(0))
    wl = W.two_layer().replace(scene=sc, rays_per_elem=64, max_bounces=12)
    g, rf = check_transport(L, ctx, wl)
    assert g["counters"][2] > 4 * wl.n_tx * wl.rays_per_tx   # more deposits than records


def test_wide_transmit_groups_splat_directly(L, ctx):
    """65 transmits of a 130-element array: the first launch group has 64 x 130
    rows, beyond what the binned splat sorts in LDS, and deposits directly;
    the second (one transmit) is binned."""
    import dataclasses
    wl = W.two_layer()
    probe = dataclasses.replace(wl.probe, n_elem=130)
    sc = dataclasses.replace(wl.scene, plane_kd=np.full_like(wl.scene.plane_kd, 0.3))
    wl = wl.replace(scene=sc, probe=probe, rays_per_elem=4, angles=np.radians(np.linspace(-10, 10, 65)),
                    tx_ids=np.arange(65, dtype=np.uint32))
    check_transport(L, ctx, wl)


def test_invalid_arguments_are_rejected(L, ctx):
    import torch
    wl = W.two_layer(rays_per_elem=64)
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    with pytest.raises(L.USError) as e:
        L.us_simulate_rf(ctx, scene, probe, wl.angles, wl.tx_ids, 0, 64, 4, ray_begin=0,
                         ray_count=wl.rays_per_tx + 1)
    assert e.value.code == L.US_EINVAL
    with pytest.raises(L.USError) as e:
        L.us_simulate_rf(ctx, scene, probe, [np.pi / 2], [0], 0, 64, 4)
    assert e.value.code == L.US_EINVAL
    with pytest.raises(L.USError) as e:
        L.us_simulate_rf(ctx, scene, probe, wl.angles, wl.tx_ids, 0, 64, 4,
                         workspace=torch.empty(1024, dtype=torch.uint8, device="cuda"))
    assert e.value.code == L.US_ETOOBIG
    bad = W.Scene(regions=np.array([[1480.0, 1.48, 0.0]]), planes=np.array([0.01]),
                  plane_regions=np.array([[0, 3]], np.int32), plane_kd=np.zeros(1),
                  spheres=np.zeros((0, 4)), sphere_regions=np.zeros((0, 2), np.int32),
                  sphere_kd=np.zeros(0))
    with pytest.raises(L.USError):
        L.Scene(ctx, bad)


def test_handles_destroyed_after_their_context(L, ctx):
    """A garbage collector may finalize a context before its probe and scene
    (objects in a reference cycle, such as the locals a caught exception's
    traceback keeps). Destroying them afterwards must neither read the freed
    context nor leave a HIP error that a later call on another context would
    report as its own."""
    wl = W.two_layer(rays_per_elem=4)
    lib = L.load()
    for _ in range(3):
        c2 = L.Context(0)
        probe, scene = L.Probe(c2, wl.probe), L.Scene(c2, wl.scene)
        assert lib.us_destroy(c2.handle) == L.US_OK
        c2.handle = None
        assert lib.us_probe_destroy(probe.handle) == L.US_OK
        probe.handle = None
        assert lib.us_scene_destroy(scene.handle) == L.US_OK
        scene.handle = None
    g = gpu_trace(L, ctx, wl)   # checks the runtime's last error after its launches
    assert np.isfinite(g["rf"]).all() and g["counters"][0] > 0


# ------------------------------------------------------------------ image chain
def _gpu_image(L, ctx, wl, rf_np):
    import torch
    probe = L.Probe(ctx, wl.probe)
    rf = torch.tensor(rf_np, dtype=torch.float32, device="cuda")
    iq = L.us_beamform(ctx, probe, wl.grid, wl.angles, wl.tx_ids, rf)
    bm = L.us_bmode(ctx, iq, wl.dr_db)
    torch.cuda.synchronize()
    iq = iq.cpu().numpy().astype(np.float64)
    return iq[..., 0] + 1j * iq[..., 1], bm.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("which", ["two_layer", "layered"])
def test_beamform_and_bmode_on_oracle_rf(L, ctx, which):
    """Each stage fed the oracle's own input, so a failure points at the stage."""
    wl = W.two_layer() if which == "two_layer" else W.layered_phantom().replace(rays_per_elem=128)
    rf, _, _ = oracle.simulate_rf(wl)
    A = oracle.analytic(rf)
    I = oracle.das(A, wl.probe, wl.grid, wl.angles)
    B = oracle.bmode(I, wl.dr_db)
    Ig, Bg = _gpu_image(L, ctx, wl, rf)
    rel = rel_l2(Ig, I)
    err = db_err(Bg, B)
    print(f"{which}: iq rel-L2 {rel:.3e}, B-mode max dB error {err:.3e}", flush=True)
    assert rel <= 1e-5
    assert err <= DB_TOL


@pytest.mark.parametrize("n_t", [64, 128, 256, 512, 1024, 2048, 8192])
def test_analytic_signal_at_every_transform_size(L, ctx, n_t):
    """The analytic signal splits n_t = 2^6..2^13 into two or three register
    passes of radix 8-32; each split is checked through us_beamform on seeded
    random channels (3 transmits, 2 rows of pixels near the bottom of the
    record so that late samples are read) against the oracle."""
    import dataclasses
    wl = W.two_layer()
    p = dataclasses.replace(wl.probe, n_t=n_t)
    depth = 0.45 * n_t / p.fs * p.c_ref   # pixels reach the last quarter of the record
    g = W.Grid.span(32, 24, -4e-3, 4e-3, 0.2 * depth, depth)
    wl = wl.replace(probe=p, grid=g, angles=np.radians([-6.0, 0.0, 5.0]),
                    tx_ids=np.arange(3, dtype=np.uint32))
    rng = np.random.default_rng(n_t)
    rf = rng.standard_normal((3, p.n_elem, n_t)).astype(np.float32)
    I = oracle.das(oracle.analytic(rf.astype(np.float64)), p, g, wl.angles)
    Ig, _ = _gpu_image(L, ctx, wl, rf)
    rel = rel_l2(Ig, I)
    print(f"n_t {n_t}: iq rel-L2 {rel:.3e}", flush=True)
    assert rel <= 1e-5


def test_tiled_and_gather_beamformers_on_a_large_grid(L, ctx):
    """The 512 x 1024 anatomy grid (192 elements, 21 transmits) is beamformed
    by the LDS-tiled kernel; a ragged 61 x 133 window of it, beamformed alone,
    is small enough for the per-pixel gather kernel. Both match the oracle on
    that window (to 1e-5, as for the full pipeline), and each other."""
    import torch
    wl = W.anatomy_phantom(level_organ=1, level_lesion=1, tube_around=8, tube_along=2)
    p, g = wl.probe, wl.grid
    rng = np.random.default_rng(9)
    k = np.exp(-0.5 * (np.arange(-12, 13) / 4.0) ** 2)
    rf = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1,
                             rng.standard_normal((wl.n_tx, p.n_elem, p.n_t))).astype(np.float32)
    probe = L.Probe(ctx, p)
    rf_t = torch.tensor(rf, device="cuda")
    big = L.us_beamform(ctx, probe, g, wl.angles, wl.tx_ids, rf_t)
    a0, b0 = 203, 301
    sub = W.Grid(61, 133, g.x0 + a0 * g.dx, g.dx, g.z0 + b0 * g.dz, g.dz)
    small = L.us_beamform(ctx, probe, sub, wl.angles, wl.tx_ids, rf_t)
    torch.cuda.synchronize()
    big = big.cpu().numpy().astype(np.float64)
    small = small.cpu().numpy().astype(np.float64)
    win = big[a0:a0 + sub.n_x, b0:b0 + sub.n_z]
    I = oracle.das(oracle.analytic(rf.astype(np.float64)), p, sub, wl.angles)
    r_tiled = rel_l2(win[..., 0] + 1j * win[..., 1], I)
    r_gather = rel_l2(small[..., 0] + 1j * small[..., 1], I)
    print(f"tiled {r_tiled:.3e}, gather {r_gather:.3e}, between {rel_l2(win, small):.3e}", flush=True)
    assert r_tiled <= 1e-5 and r_gather <= 1e-5
    assert rel_l2(win, small) <= 1e-6


def _window_widths(p, g, angles, tile=16):
    """Sample-window lengths of every (tile, element, transmit) of a tiled
    beamformer with the conservative bound of the tile's corners (the
    transmit term's extremes plus the receive distance's, one sample of slack
    on each side), computed here from the geometry alone."""
    spm = p.fs / p.c_ref
    out = []
    for a0 in range(0, g.n_x, tile):
        for b0 in range(0, g.n_z, tile):
            xa, xb = g.x0 + a0 * g.dx, g.x0 + (min(a0 + tile, g.n_x) - 1) * g.dx
            za, zb = g.z0 + b0 * g.dz, g.z0 + (min(b0 + tile, g.n_z) - 1) * g.dz
            xe = (np.arange(p.n_elem) - 0.5 * (p.n_elem - 1)) * p.pitch
            near = np.where(xe < xa, xa - xe, np.where(xe > xb, xe - xb, 0.0))
            far = np.maximum(np.abs(xe - xa), np.abs(xe - xb))
            for th in angles:
                l = [xa * np.sin(th) + za * np.cos(th), xb * np.sin(th) + za * np.cos(th),
                     xa * np.sin(th) + zb * np.cos(th), xb * np.sin(th) + zb * np.cos(th)]
                lo = np.floor((min(l) + np.hypot(near, za)) * spm) - 1
                hi = np.floor((max(l) + np.hypot(far, zb)) * spm) + 2
                out.append(hi - lo + 1)
    return np.concatenate(out)


def test_tiled_beamformer_wide_windows_and_ragged_groups(L, ctx):
    """127 elements x 5 transmits (635 pairs: the last group of 16 is partial)
    on a 128 x 160 grid of 0.12 mm rows, so that about 40 % of the tile
    windows exceed the 144 samples held in LDS and are read from HBM while the
    rest come from LDS; seeded random channels against the oracle's fp64
    delay-and-sum."""
    import dataclasses
    wl = W.two_layer()
    p = dataclasses.replace(wl.probe, n_elem=127)
    g = W.Grid.span(128, 160, -12e-3, 12e-3, 2e-3, 2e-3 + 160 * 0.12e-3)
    angles = np.radians([-8.0, -4.0, 0.0, 4.0, 8.0])
    wl = wl.replace(probe=p, grid=g, angles=angles, tx_ids=np.arange(5, dtype=np.uint32))
    widths = _window_widths(p, g, angles)
    assert (widths > 144).any() and (widths <= 144).any(), (widths.min(), widths.max())
    assert (p.n_elem * len(angles)) % 16 != 0 and (g.n_x // 16) * (g.n_z // 16) >= 64
    rng = np.random.default_rng(21)
    k = np.exp(-0.5 * (np.arange(-12, 13) / 4.0) ** 2)
    rf = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1,
                             rng.standard_normal((5, p.n_elem, p.n_t))).astype(np.float32)
    I = oracle.das(oracle.analytic(rf.astype(np.float64)), p, g, angles)
    Ig, _ = _gpu_image(L, ctx, wl, rf)
    rel = rel_l2(Ig, I)
    print(f"wide windows {np.mean(widths > 144):.2f} of tile pairs: iq rel-L2 {rel:.3e}", flush=True)
    assert rel <= 1e-5


def test_beamform_more_transmits_than_one_launch(L, ctx):
    """70 transmits: the library beamforms them in two launches (64, then 6,
    the second adding into the image) with the two-slice tiled kernel
    (64 tiles); seeded random channels against the oracle."""
    import dataclasses
    wl = W.two_layer()
    p = dataclasses.replace(wl.probe, n_elem=48)
    g = W.Grid.span(128, 128, -6e-3, 6e-3, 4e-3, 4e-3 + 128 * 0.12e-3)
    angles = np.radians(np.linspace(-12.0, 12.0, 70))
    wl = wl.replace(probe=p, grid=g, angles=angles, tx_ids=np.arange(70, dtype=np.uint32))
    rng = np.random.default_rng(5)
    k = np.exp(-0.5 * (np.arange(-12, 13) / 4.0) ** 2)
    rf = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1,
                             rng.standard_normal((70, p.n_elem, p.n_t))).astype(np.float32)
    I = oracle.das(oracle.analytic(rf.astype(np.float64)), p, g, angles)
    Ig, _ = _gpu_image(L, ctx, wl, rf)
    rel = rel_l2(Ig, I)
    print(f"70 transmits: iq rel-L2 {rel:.3e}", flush=True)
    assert rel <= 1e-5


@pytest.mark.parametrize("case", ["two_layer_3tx", "layered_full_grid"])
def test_beamform_acquisition_gradients_against_oracle(L, ctx, case):
    """d Re<g, I> / d (steering angle of each transmit, c_ref, pitch) from the
    library against the oracle's on the same RF and image gradient (the oracle
    forms the analytic signal in fp64, the library in fp32): within the
    gradient tolerance, 1e-3 relative per parameter."""
    import torch
    if case == "two_layer_3tx":
        wl = W.two_layer().replace(angles=np.radians([-6.0, 0.0, 5.0]), tx_ids=np.arange(3, dtype=np.uint32))
    else:
        wl = W.layered_phantom()
    p, g, angles = wl.probe, wl.grid, wl.angles
    rng = np.random.default_rng(31)
    k = np.exp(-0.5 * (np.arange(-12, 13) / 4.0) ** 2)
    rf = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1,
                             rng.standard_normal((len(angles), p.n_elem, p.n_t))).astype(np.float32)
    g_I = (rng.standard_normal((g.n_x, g.n_z)) + 1j * rng.standard_normal((g.n_x, g.n_z))).astype(np.complex64)
    ref = oracle.das_acq_vjp(oracle.analytic(rf.astype(np.float64)), g_I.astype(np.complex128), p, g, angles)
    ref = np.array([*ref[0], ref[1], ref[2]])
    probe = L.Probe(ctx, p)
    giq = torch.tensor(np.stack([g_I.real, g_I.imag], -1), dtype=torch.float32, device="cuda")
    got = L.us_beamform_acq_vjp(ctx, probe, g, angles, wl.tx_ids, torch.tensor(rf, device="cuda"), giq)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"{case}: acquisition gradients worst relative error {rel.max():.2e} "
          f"(angles {rel[:-2].max():.2e}, c_ref {rel[-2]:.2e}, pitch {rel[-1]:.2e})", flush=True)
    assert np.all(rel <= 1e-3)


def test_end_to_end_bmode_full_size(L, ctx):
    wl = W.two_layer()
    out = oracle.render(wl)
    g = gpu_trace(L, ctx, wl)
    _, Bg = _gpu_image(L, ctx, wl, g["rf"])
    assert db_err(Bg, out["B"]) <= DB_TOL


def test_bmode_vjp_against_oracle(L, ctx):
    import torch
    rng = np.random.default_rng(0)
    wl = W.layered_phantom().replace(rays_per_elem=64)
    out = oracle.render(wl)
    I = out["I"]
    g_B = rng.standard_normal(I.shape)
    ref = oracle.bmode_vjp(I, g_B, 60.0)
    iq = torch.tensor(np.stack([I.real, I.imag], -1), dtype=torch.float32, device="cuda")
    gb = torch.tensor(g_B, dtype=torch.float32, device="cuda")
    g = L.us_bmode_vjp(ctx, iq, gb, 60.0)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    gc = g[..., 0] + 1j * g[..., 1]
    assert rel_l2(gc, ref) <= 1e-4


@pytest.mark.parametrize("case", ["layered_3tx", "two_layer_40tx_ragged", "fine_grid_gather", "odd_channel_count"])
def test_beamform_vjp_against_oracle(L, ctx, case):
    """Transposed DAS + analytic VJP. The first two cases take the column
    kernel (pixels of a column more than two samples apart), the second with
    40 transmits on a ragged grid starting 2 mm below the array; the third,
    with 0.03 mm pixels (under one sample apart), the per-sample gather; the
    fourth has 63 elements x 3 transmits, an odd number of channels, so the
    analytic adjoint's last block transforms one channel alone."""
    import dataclasses
    import torch
    rng = np.random.default_rng(1)
    if case == "odd_channel_count":
        base = W.two_layer()
        wl = base.replace(probe=dataclasses.replace(base.probe, n_elem=63), angles=np.radians([-5.0, 0.0, 6.0]),
                          tx_ids=np.arange(3, dtype=np.uint32))
    elif case == "layered_3tx":
        wl = W.layered_phantom().replace(angles=np.radians([-10.0, 2.0, 10.0]),
                                         tx_ids=np.arange(3, dtype=np.uint32))
    elif case == "two_layer_40tx_ragged":
        wl = W.two_layer().replace(angles=np.radians(np.linspace(-12.0, 12.0, 40)),
                                   tx_ids=np.arange(40, dtype=np.uint32),
                                   grid=W.Grid(101, 173, -15e-3, 0.3e-3, 2.0e-3, 0.2e-3))
    else:
        wl = W.layered_phantom().replace(angles=np.radians([-7.0, 4.0]), tx_ids=np.arange(2, dtype=np.uint32),
                                         grid=W.Grid(61, 301, -6e-3, 0.2e-3, 18e-3, 0.03e-3))
    gI = rng.standard_normal((wl.grid.n_x, wl.grid.n_z)) + 1j * rng.standard_normal((wl.grid.n_x, wl.grid.n_z))
    ref = oracle.analytic_vjp(oracle.das_vjp(gI, wl.probe, wl.grid, wl.angles, wl.probe.n_t))
    probe = L.Probe(ctx, wl.probe)
    giq = torch.tensor(np.stack([gI.real, gI.imag], -1), dtype=torch.float32, device="cuda")
    g = L.us_beamform_vjp(ctx, probe, wl.grid, wl.angles, wl.tx_ids, giq)
    torch.cuda.synchronize()
    assert rel_l2(g.cpu().numpy().astype(np.float64), ref) <= 1e-5
