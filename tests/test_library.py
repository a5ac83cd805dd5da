"""Host-side checks of the C-ABI library (no GPU needed): it loads, and it
exports every entry point the header declares."""
import ctypes
import os

import pytest

from paper_2604_15017_amd import _lib as L


def test_header_declares_the_boundary():
    names = L.header_symbols()
    for required in ["us_create", "us_destroy", "us_last_error", "us_probe_upload",
                     "us_scene_upload", "us_scene_set_params", "us_simulate_rf", "us_beamform",
                     "us_bmode", "us_bmode_vjp", "us_beamform_vjp", "us_simulate_rf_vjp"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libusrt.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in L.header_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L._SIGNATURES) == set(L.header_symbols())


def test_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libusrt.so not built")
    with pytest.raises(Exception):
        L.Context(0)


def test_binding_rejects_tensors_the_library_would_overrun():
    """The binding checks each caller tensor's dtype, element count, layout
    and device before handing its raw pointer to the library."""
    import torch
    from paper_2604_15017_amd import _lib
    with pytest.raises(ValueError, match="elements"):
        _lib._expect(torch.zeros(5, dtype=torch.float64), 6, torch.float64, "out")
    with pytest.raises(ValueError, match="float32"):
        _lib._expect(torch.zeros(6, dtype=torch.float64), 6, torch.float32, "rf")
    with pytest.raises(ValueError, match="contiguous"):
        _lib._expect(torch.zeros(4, 6, dtype=torch.float32).t(), 24, torch.float32, "rf")
    with pytest.raises(ValueError, match="GPU"):
        _lib._expect(torch.zeros(6, dtype=torch.float32), 6, torch.float32, "rf")
    with pytest.raises(ValueError, match="missing"):
        _lib._expect(None, 6, torch.float32, "g_iq")


def test_binding_rejects_mismatched_transmits_and_workspaces():
    """Every steering angle needs its transmit id (each id selects the Philox
    stream of its transmit), and a workspace is a uint8 device buffer whose
    element count the library takes as its size in bytes."""
    import torch
    from paper_2604_15017_amd import _lib
    arr, n = _lib._tx_array([0.0, 0.1], [3, 4])
    assert n == 2 and arr[1].id == 4 and abs(arr[1].angle - 0.1) < 1e-15
    with pytest.raises(ValueError, match="tx_ids"):
        _lib._tx_array([0.0, 0.1, 0.2], [0, 1])
    with pytest.raises(ValueError, match="uint8"):
        _lib._expect_ws(torch.zeros(16, dtype=torch.float32))
    with pytest.raises(ValueError, match="GPU"):
        _lib._expect_ws(torch.zeros(16, dtype=torch.uint8))
    with pytest.raises(ValueError, match="missing"):
        _lib._expect_ws(None)
