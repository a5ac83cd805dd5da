"""The one-call backward us_frame_vjp (dL/dB to the parameters, the
analytic-signal and pulse adjoints fused into one kernel per RF row) against
the chain of the three vector-Jacobian products it composes (us_bmode_vjp,
us_beamform_vjp, us_simulate_rf_vjp) on the same frame: bit for bit, since
both form the same sums in the same order. The chain itself is pinned to the
oracle by the backward parity tests."""
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


def frame(L, ctx, scene, probe, wl, ray_begin, ray_count):
    rf = L.us_simulate_rf(ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                          wl.max_bounces, ray_begin=ray_begin, ray_count=ray_count)
    iq = L.us_beamform(ctx, probe, wl.grid, wl.angles, wl.tx_ids, rf)
    return iq, L.us_bmode(ctx, iq, wl.dr_db)


def chain_vs_fused(L, ctx, wl, target, label, ray_begin=0, ray_count=None):
    import torch
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    _, b_ref = frame(L, ctx, L.Scene(ctx, target), probe, wl, ray_begin, ray_count)
    iq, b = frame(L, ctx, scene, probe, wl, ray_begin, ray_count)
    _, g_b = L.us_image_loss(ctx, b, b_ref, 0.0, 1.0)
    g_iq = L.us_bmode_vjp(ctx, iq, g_b, wl.dr_db)
    g_rf = L.us_beamform_vjp(ctx, probe, wl.grid, wl.angles, wl.tx_ids, g_iq)
    g_chain = L.us_simulate_rf_vjp(ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                                   wl.max_bounces, g_rf, ray_begin=ray_begin, ray_count=ray_count)
    g_fused = L.us_frame_vjp(ctx, scene, probe, wl.grid, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                             wl.max_bounces, iq, g_b, wl.dr_db, ray_begin=ray_begin, ray_count=ray_count)
    torch.cuda.synchronize()
    a, f = g_chain.cpu().numpy(), g_fused.cpu().numpy()
    diff = int(np.count_nonzero(a != f))
    print(f"{label}: {a.shape[0]} parameters, |g| max {np.abs(a).max():.3e}, {diff} differ", flush=True)
    assert np.isfinite(a).all() and np.abs(a).max() > 0
    assert np.array_equal(a, f)


def test_layered_phantom_column_adjoint(L, ctx):
    # 256 x 512 pixels: rows more than two samples apart, the column DAS adjoint
    wl = W.layered_phantom(rays_per_tx=1 << 15)
    chain_vs_fused(L, ctx, wl, W.layered_phantom_target(wl), "layered, 11 x 2^15 rays")


def test_layered_phantom_gather_adjoint_ragged_rows(L, ctx):
    # a finer, ragged grid (per-sample gather adjoint) and 3 transmits
    wl = W.with_grid(W.layered_phantom(rays_per_tx=1 << 14, n_tx=3), 77, 1333)
    chain_vs_fused(L, ctx, wl, W.layered_phantom_target(wl), "layered, 77 x 1333 grid")


@pytest.mark.parametrize("n_t", [64, 256, 8192])
def test_transform_sizes(L, ctx, n_t):
    # the shortest and longest rows the analytic map supports (the pulse's taps
    # reach past both ends of the shortest); the interface 30 % into the record
    # (at most 20 mm deep) and 1 % deeper in the target
    import dataclasses
    base = W.two_layer(rays_per_elem=1 << 9)
    depth = min(0.3 * n_t / base.probe.fs * base.scene.regions[0, 0] / 2, 20e-3)
    wl = W.tiny(base, rays_per_elem=1 << 9, n_t=n_t)
    wl = wl.replace(scene=dataclasses.replace(wl.scene, planes=np.array([depth])))
    target = dataclasses.replace(wl.scene, planes=np.array([1.01 * depth]))
    chain_vs_fused(L, ctx, wl, target, f"two-layer, n_t = {n_t}")


def test_odd_channel_count(L, ctx):
    # 63 elements and one transmit: the analytic adjoint takes the channels two
    # at a time and the last one alone, in the chain and in the fused kernel
    import dataclasses
    base = W.two_layer(rays_per_elem=1 << 9)
    wl = W.tiny(base, rays_per_elem=1 << 9, n_elem=63)
    depth = float(base.scene.planes[0])
    target = dataclasses.replace(wl.scene, planes=np.array([1.01 * depth]))
    chain_vs_fused(L, ctx, wl, target, "two-layer, 63 channels")


def test_anatomy_phantom_ray_sample(L, ctx):
    wl = W.anatomy_phantom()
    chain_vs_fused(L, ctx, wl, W.anatomy_phantom_target(wl), "anatomy, 21 x 20000 rays",
                   ray_begin=390_000, ray_count=20_000)


def test_autograd_frame_matches_the_chain(L, ctx):
    import torch
    from paper_2604_15017_amd.autograd import Renderer, mse
    wl = W.layered_phantom(rays_per_tx=1 << 14, n_tx=4)
    r = Renderer(wl, ctx)
    b_ref = r.render(torch.tensor(W.layered_phantom_target(wl).theta(), device=ctx.torch_device)).detach()
    th1 = r.theta0.clone().requires_grad_(True)
    mse(r.render(th1), b_ref, r).backward()
    th2 = r.theta0.clone().requires_grad_(True)
    mse(r.render_frame(th2), b_ref, r).backward()
    torch.cuda.synchronize()
    assert torch.equal(th1.grad, th2.grad)


def test_autograd_recorded_frame(L, ctx):
    """render_frame(recorded=True): the gradient of the plain frame bit for bit;
    after another recorded forward with other parameters its records are gone
    and the backward traces the paths again, with the same gradient."""
    import torch
    from paper_2604_15017_amd.autograd import Renderer, mse
    wl = W.layered_phantom(rays_per_tx=1 << 14, n_tx=4)
    r = Renderer(wl, ctx)
    b_ref = r.render(torch.tensor(W.layered_phantom_target(wl).theta(), device=ctx.torch_device)).detach()
    th1 = r.theta0.clone().requires_grad_(True)
    mse(r.render_frame(th1), b_ref, r).backward()
    th2 = r.theta0.clone().requires_grad_(True)
    mse(r.render_frame(th2, recorded=True), b_ref, r).backward()
    th3 = r.theta0.clone().requires_grad_(True)
    loss3 = mse(r.render_frame(th3, recorded=True), b_ref, r)
    other = r.theta0.clone() * (1.0 + 1e-3)
    r.render_frame(other, recorded=True)   # overwrites the records with other parameters
    loss3.backward()
    torch.cuda.synchronize()
    assert torch.equal(th1.grad, th2.grad) and torch.equal(th1.grad, th3.grad)


def test_workspace_sets_the_chunks(L, ctx):
    """A workspace sized for fewer rays than the frame's makes the replay run
    in shorter chunks, with the same gradient bit for bit; one holding the
    image buffers but no replay chunk is refused."""
    import torch
    wl = W.tiny(W.two_layer(rays_per_elem=1 << 8), rays_per_elem=1 << 8)
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    iq, b = frame(L, ctx, scene, probe, wl, 0, None)
    g_b = torch.ones_like(b)
    args = (ctx, scene, probe, wl.grid, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces, iq, g_b,
            wl.dr_db)
    g_full = L.us_frame_vjp(*args)
    short = L.us_frame_vjp_workspace_size(scene, probe, wl.grid, wl.n_tx, wl.rays_per_tx // 7, wl.max_bounces)
    assert short < L.us_frame_vjp_workspace_size(scene, probe, wl.grid, wl.n_tx, wl.rays_per_tx, wl.max_bounces)
    g_short = L.us_frame_vjp(*args, workspace=torch.empty(short, dtype=torch.uint8, device=ctx.torch_device))
    torch.cuda.synchronize()
    assert torch.equal(g_full, g_short) and g_full.abs().max() > 0
    image_only = L.us_frame_vjp_recorded_workspace_size(probe, wl.grid, wl.n_tx)
    ws = torch.empty(image_only, dtype=torch.uint8, device=ctx.torch_device)
    with pytest.raises(L.USError, match="workspace too small"):
        L.us_frame_vjp(*args, workspace=ws)
