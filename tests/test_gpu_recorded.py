"""The recorded frame (us_simulate_rf_recorded, then us_simulate_rf_vjp_recorded
or us_frame_vjp_recorded from its step records) against the plain calls on
the same frame: the RF and the gradients bit for bit, since the recorded
forward forms every path and deposit with the same arithmetic and both sides
sum in integers. The plain calls are pinned to the oracle by the forward,
backward and mesh parity tests."""
import numpy as np
import pytest

from paper_2604_15017_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_2604_15017_amd import _lib
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return _lib


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


def smooth_field(shape, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(shape)
    k = np.exp(-0.5 * (np.arange(-30, 31) / 10.0) ** 2)
    return np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1, g).astype(np.float32)


def rf_and_grad(L, ctx, wl, label, ray_begin=0, ray_count=None, nonzero=True):
    import torch
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    args = (wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces)
    c = torch.zeros(5, dtype=torch.int64, device=ctx.torch_device)
    c_r = torch.zeros_like(c)
    rf = L.us_simulate_rf(ctx, scene, probe, *args, ray_begin=ray_begin, ray_count=ray_count, counters=c)
    rf_r, rec = L.us_simulate_rf_recorded(ctx, scene, probe, *args, ray_begin=ray_begin, ray_count=ray_count,
                                          counters=c_r)
    g_rf = torch.tensor(smooth_field(tuple(rf.shape), 5), device=ctx.torch_device)
    g = L.us_simulate_rf_vjp(ctx, scene, probe, *args, g_rf, ray_begin=ray_begin, ray_count=ray_count)
    g_r = L.us_simulate_rf_vjp_recorded(ctx, rec, g_rf)
    g_r2 = L.us_simulate_rf_vjp_recorded(ctx, rec, g_rf)   # the records stay valid
    torch.cuda.synchronize()
    a, b = rf.cpu().numpy(), rf_r.cpu().numpy()
    ga, gb, gc = g.cpu().numpy(), g_r.cpu().numpy(), g_r2.cpu().numpy()
    print(f"{label}: rf |max| {np.abs(a).max():.3e}, {int(np.count_nonzero(a != b))} samples differ; "
          f"|g| max {np.abs(ga).max():.3e}, {int(np.count_nonzero(ga != gb))} gradient entries differ", flush=True)
    print(f"  counters {c.tolist()} (plain), {c_r.tolist()} (recorded)", flush=True)
    if nonzero:
        assert np.abs(a).max() > 0 and np.abs(ga).max() > 0
    assert torch.equal(c, c_r) and int(c[0]) > 0
    assert np.array_equal(a, b)
    assert np.array_equal(ga, gb) and np.array_equal(gb, gc)
    return scene, probe, rec


def test_layered_phantom(L, ctx):
    rf_and_grad(L, ctx, W.layered_phantom(rays_per_tx=1 << 15), "layered, 11 x 2^15 rays")


def test_rough_layered_phantom_ray_range(L, ctx):
    wl = W.rough_layered_phantom(rays_per_tx=1 << 14)
    rf_and_grad(L, ctx, wl, "rough layered, ray range", ray_begin=1000, ray_count=9001)


def test_cylinder_phantom(L, ctx):
    rf_and_grad(L, ctx, W.cylinder_phantom(rays_per_tx=1 << 14), "cylinder, 5 x 2^14 rays")


def test_anatomy_phantom_ray_sample(L, ctx):
    rf_and_grad(L, ctx, W.anatomy_phantom(), "anatomy, 21 x 20000 rays", ray_begin=390_000, ray_count=20_000)


@pytest.mark.parametrize("bounces", [0, 1])
def test_few_interactions(L, ctx, bounces):
    # no interaction: every ray leaves downwards and the RF is zero on both sides
    wl = W.tiny(W.two_layer(rays_per_elem=1 << 8), rays_per_elem=1 << 8).replace(max_bounces=bounces)
    rf_and_grad(L, ctx, wl, f"two-layer, {bounces} interactions", nonzero=bounces > 0)


def test_frame_vjp_recorded_full_anatomy_frame(L, ctx):
    """The benchmark's forward+backward frame: recorded forward and one-call
    backward against the plain ones, bit for bit."""
    import torch
    wl = W.anatomy_phantom()
    target = W.anatomy_phantom_target(wl)
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    args = (wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces)
    rf_t = L.us_simulate_rf(ctx, L.Scene(ctx, target), probe, *args)
    b_ref = L.us_bmode(ctx, L.us_beamform(ctx, probe, wl.grid, wl.angles, wl.tx_ids, rf_t), wl.dr_db)
    c = torch.zeros(5, dtype=torch.int64, device=ctx.torch_device)
    c_r = torch.zeros_like(c)
    rf = L.us_simulate_rf(ctx, scene, probe, *args, counters=c)
    iq = L.us_beamform(ctx, probe, wl.grid, wl.angles, wl.tx_ids, rf)
    _, g_b = L.us_image_loss(ctx, L.us_bmode(ctx, iq, wl.dr_db), b_ref, 0.0, 1.0)
    g = L.us_frame_vjp(ctx, scene, probe, wl.grid, *args, iq, g_b, wl.dr_db)
    rf_r, rec = L.us_simulate_rf_recorded(ctx, scene, probe, *args, counters=c_r)
    g_r = L.us_frame_vjp_recorded(ctx, rec, wl.grid, iq, g_b, wl.dr_db)
    torch.cuda.synchronize()
    a, b = rf.cpu().numpy(), rf_r.cpu().numpy()
    ga, gb = g.cpu().numpy(), g_r.cpu().numpy()
    print(f"anatomy frame: {int(np.count_nonzero(a != b))} RF samples and {int(np.count_nonzero(ga != gb))} of "
          f"{ga.size} gradient entries differ, |g| max {np.abs(ga).max():.3e}; counters {c.tolist()}", flush=True)
    assert np.array_equal(a, b) and np.array_equal(ga, gb) and np.abs(ga).max() > 0
    assert torch.equal(c, c_r)


def test_recorded_backward_checks_its_records(L, ctx):
    import torch
    wl = W.tiny(W.two_layer(rays_per_elem=1 << 8), rays_per_elem=1 << 8)
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    args = (wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces)
    rf, rec = L.us_simulate_rf_recorded(ctx, scene, probe, *args)
    g_rf = torch.ones_like(rf)
    L.us_simulate_rf_vjp_recorded(ctx, rec, g_rf)
    # another seed, another ray range, another workspace: no records for them
    for change in (dict(seed=wl.seed + 1), dict(ray_count=rec.ray_count - 1)):
        bad = L.Recorded(
            scene, probe, rec.angles, rec.tx_ids, change.get("seed", rec.seed), rec.rays_per_elem,
            rec.max_bounces, rec.ray_begin, change.get("ray_count", rec.ray_count), rec.workspace)
        with pytest.raises(L.USError, match="no recorded forward"):
            L.us_simulate_rf_vjp_recorded(ctx, bad, g_rf)
    other = L.Recorded(scene, probe, rec.angles, rec.tx_ids, rec.seed, rec.rays_per_elem, rec.max_bounces,
                       rec.ray_begin, rec.ray_count, rec.workspace.clone())
    with pytest.raises(L.USError, match="no recorded forward"):
        L.us_simulate_rf_vjp_recorded(ctx, other, g_rf)
    # new parameters invalidate the records
    scene.set_params(torch.tensor(wl.scene.theta(), dtype=torch.float64, device=ctx.torch_device))
    with pytest.raises(L.USError, match="no recorded forward"):
        L.us_simulate_rf_vjp_recorded(ctx, rec, g_rf)
    # a workspace one byte short, and more transmits than one launch group
    need = L.us_recorded_workspace_size(scene, probe, wl.n_tx, wl.rays_per_tx, wl.max_bounces)
    short = torch.empty(need - 1, dtype=torch.uint8, device=ctx.torch_device)
    with pytest.raises(L.USError, match="workspace too small"):
        L.us_simulate_rf_recorded(ctx, scene, probe, *args, workspace=short)
    assert L.us_recorded_workspace_size(scene, probe, 65, wl.rays_per_tx, wl.max_bounces) == 0
