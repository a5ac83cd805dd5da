"""us_beamform_static (the allocation-free entry point, static scratch) against
us_beamform (caller workspace) through the C-ABI: the same kernels, so the
images agree bit for bit, on two calls in a row, the second with a smaller
input; a request beyond the 64 MiB scratch is refused before any launch."""
import numpy as np
import pytest

from paper_2604_15017_amd import workloads as W

pytestmark = pytest.mark.gpu


def _field(shape, seed):
    rng = np.random.Generator(np.random.Philox(key=[seed, 9]))
    return rng.standard_normal(shape).astype(np.float32)


def test_static_beamform_equals_workspace_beamform():
    import torch
    from paper_2604_15017_amd import _lib as L
    assert torch.cuda.is_available()
    ctx = L.Context(0)
    big = W.layered_phantom()                                    # 11 x 128 x 4096: 46 MB of analytic signal
    small = W.two_layer().replace(angles=np.radians([-5.0, 5.0]), tx_ids=np.arange(2, dtype=np.uint32))
    for wl, seed in ((big, 1), (small, 2)):
        p = wl.probe
        probe = L.Probe(ctx, p)
        rf = torch.tensor(_field((wl.n_tx, p.n_elem, p.n_t), seed), device="cuda")
        ref = L.us_beamform(ctx, probe, wl.grid, wl.angles, wl.tx_ids, rf)
        got = L.us_beamform_static(ctx, probe, wl.grid, wl.angles, wl.tx_ids, rf)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.abs(r).max() > 0
        assert np.array_equal(r, g), (wl.name, float(np.abs(r - g).max()))
    # beyond the scratch: 21 x 192 x 8192 complex samples (264 MB)
    wa = W.anatomy_phantom()
    pa = wa.probe
    probe = L.Probe(ctx, pa)
    rf = torch.zeros((wa.n_tx, pa.n_elem, pa.n_t), dtype=torch.float32, device="cuda")
    with pytest.raises(L.USError, match="static scratch"):
        L.us_beamform_static(ctx, probe, wa.grid, wa.angles, wa.tx_ids, rf)
