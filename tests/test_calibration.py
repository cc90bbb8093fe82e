"""The vector-ALU rate and clock probe behind the sweep's ALU roofline (libpa_calib.so): it is
built, exports its calls, rejects bad arguments without touching the device, and on the GPU gives
a clock and a per-CU issue rate the hardware can have."""
import ctypes

import pytest

from paper_1006_0252_amd import valu_calibration as vc


def test_probe_library_exports_and_rejects_bad_arguments():
    L = vc.lib()
    for n in ("pa_calib_valu", "pa_calib_instructions_per_iteration", "pa_calib_wall_clock_khz"):
        assert hasattr(L, n)
    assert L.pa_calib_instructions_per_iteration(0) == 16
    assert L.pa_calib_instructions_per_iteration(len(vc.KINDS)) == -1
    assert L.pa_calib_valu(len(vc.KINDS), 1, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == 1
    assert L.pa_calib_valu(0, 0, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == 1
    assert L.pa_calib_valu(0, 1, 1, None, ctypes.c_void_p(8), None) == 1


@pytest.mark.gpu
def test_probe_measures_a_plausible_clock_and_issue_rate():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[case] VALU probe", flush=True)
    res = vc.measure(kinds=[0, 5], iters=4000, repeats=1)
    for kind, r in res.items():
        # one wave64 instruction per SIMD every four cycles is 64 lanes per cycle per CU
        assert 0.5e9 < r["clock_hz"] < 3.5e9, kind
        assert 16.0 < r["per_cu_per_clock"] < 130.0, kind
