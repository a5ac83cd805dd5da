"""Identical calls give bitwise identical results, whatever the scheduling of
the threads: the deposit histogram is fixed point and filled with integer
atomics, and every adjoint sum (parameters, mesh vertices, acquisition
parameters, the loss, the B-mode normalisation term) is kept in integer
windows whose total does not depend on the order of the additions. Splitting
a call into chunks through a small workspace changes the grouping of the
same additions, so it gives the same bits too."""
import numpy as np
import pytest

from paper_2604_15017_amd import workloads as W

from test_gpu_mesh import small_anatomy

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
    rng = np.random.Generator(np.random.Philox(key=[seed, 5]))
    x = rng.standard_normal(shape)
    k = np.exp(-0.5 * (np.arange(-8, 9) / 3.0) ** 2)
    return np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), -1, x)


def forward(L, ctx, scene, probe, wl, workspace=None):
    import torch
    counters = torch.zeros(5, dtype=torch.int64, device="cuda")
    rf = L.us_simulate_rf(ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                          counters=counters, workspace=workspace)
    torch.cuda.synchronize()
    return rf.cpu().numpy(), counters.cpu().numpy()


def vjp(L, ctx, scene, probe, wl, g_rf, workspace=None):
    import torch
    g_acq = torch.zeros(wl.n_tx + 3, dtype=torch.float64, device="cuda")
    g = L.us_simulate_rf_vjp(ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                             wl.max_bounces, g_rf, workspace=workspace, g_acq=g_acq)
    torch.cuda.synchronize()
    return g.cpu().numpy(), g_acq.cpu().numpy()


@pytest.mark.parametrize("name", ["layered", "mesh"])
def test_forward_and_vjp_bitwise_repeatable(L, ctx, name):
    """Layered phantom (binned splat, LDS sums) and blob + tube meshes (direct
    integer atomics, per-vertex sums): two calls, and a call split into
    chunks, give the same RF and the same gradients bit for bit."""
    import torch
    if name == "layered":
        wl = W.layered_phantom().replace(rays_per_elem=96, angles=np.radians([-8.0, 0.0, 6.0]),
                                         tx_ids=np.array([0, 5, 9], dtype=np.uint32))
    else:
        wl = small_anatomy(rays_per_elem=96)
    p = wl.probe
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    rf1, c1 = forward(L, ctx, scene, probe, wl)
    rf2, c2 = forward(L, ctx, scene, probe, wl)
    assert np.abs(rf1).max() > 0
    assert np.array_equal(rf1, rf2) and np.array_equal(c1, c2)
    small = L._workspace(L.us_simulate_rf_workspace_size(scene, probe, wl.n_tx, 700, wl.max_bounces), "cuda")
    rf3, c3 = forward(L, ctx, scene, probe, wl, workspace=small)
    assert np.array_equal(rf1, rf3) and np.array_equal(c1, c3)

    g_rf = torch.tensor(smooth_field((wl.n_tx, p.n_elem, p.n_t), 21).astype(np.float32), device="cuda")
    g1, a1 = vjp(L, ctx, scene, probe, wl, g_rf)
    g2, a2 = vjp(L, ctx, scene, probe, wl, g_rf)
    assert np.abs(g1).max() > 0 and np.abs(a1).max() > 0
    assert np.array_equal(g1, g2) and np.array_equal(a1, a2)
    small = L._workspace(L.us_simulate_rf_vjp_workspace_size(scene, probe, wl.n_tx, 500, wl.max_bounces), "cuda")
    g3, a3 = vjp(L, ctx, scene, probe, wl, g_rf, workspace=small)
    assert np.array_equal(g1, g3) and np.array_equal(a1, a3)


def test_image_chain_bitwise_repeatable(L, ctx):
    """Loss, B-mode VJP (with its normalisation sum) and the transposed DAS on
    the layered grid: two calls, same bits."""
    import torch
    wl = W.layered_phantom()
    p, g = wl.probe, wl.grid
    rf = torch.tensor(smooth_field((wl.n_tx, p.n_elem, p.n_t), 3).astype(np.float32), device="cuda")
    probe = L.Probe(ctx, p)
    iq = L.us_beamform(ctx, probe, g, wl.angles, wl.tx_ids, rf)
    b = L.us_bmode(ctx, iq, wl.dr_db)
    ref = (b + torch.tensor(smooth_field((g.n_x, g.n_z), 4).astype(np.float32), device="cuda")).contiguous()
    outs = []
    for _ in range(2):
        loss, g_b = L.us_image_loss(ctx, b, ref, 0.5, 1.0)
        g_iq = L.us_bmode_vjp(ctx, iq, g_b, wl.dr_db)
        g_rf = L.us_beamform_vjp(ctx, probe, g, wl.angles, wl.tx_ids, g_iq)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in (loss, g_b, g_iq, g_rf)])
    for x, y in zip(*outs):
        assert np.array_equal(x, y)
    assert outs[0][0][0] > 0


def test_full_frame_bitwise_repeatable(L, ctx):
    """The layered phantom's whole forward frame (11 x 2^20 rays): two calls
    give the same RF bit for bit (the determinism check of the measurement
    protocol asks for 1e-6 relative L2 at most)."""
    wl = W.layered_phantom()
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    rf1, c1 = forward(L, ctx, scene, probe, wl)
    rf2, c2 = forward(L, ctx, scene, probe, wl)
    assert np.array_equal(rf1, rf2) and np.array_equal(c1, c2)
