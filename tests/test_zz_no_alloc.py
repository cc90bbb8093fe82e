"""pa_mlp_grad_static, the loss gradient for callers that cannot allocate: its work matrix lives in
a fixed device array of the library.  Through the C ABI it must give exactly the gradient and
loss of pa_mlp_grad (the same kernels on caller memory) on two calls in a row, the second with a
smaller batch (the array keeps the first call's contents), and reject batches beyond its size
before any device work."""
import ctypes
import sys

import numpy as np
import pytest

from tests import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1006_0252_amd import learned, pa  # noqa: E402

DEV = "cuda:0"


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def test_static_gradient_equals_caller_work_gradient():
    s = torch.cuda.current_stream(DEV).cuda_stream
    theta = torch.from_numpy(inputs.mlp_theta(51, scale=1.5)).to(DEV)
    w = torch.zeros(learned.N_PARAMS, dtype=torch.int16, device=DEV)
    pa.check(pa.lib().pa_bf16_round(theta.data_ptr(), w.data_ptr(), learned.N_PARAMS, s), "pa_bf16_round")
    for B in (pa.PA_MLP_STATIC_MAX_B - 96, 700):  # several 1024-sample chunks, then fewer than the first call
        note(f"static gradient B={B}")
        X = torch.from_numpy(inputs.mlp_features(52 + B, B, zero_var_every=43)).to(DEV)
        t = torch.from_numpy(inputs.mlp_targets(53 + B, B, bad_every=31)).to(DEV)
        nb = ctypes.c_int64()
        pa.check(pa.lib().pa_mlp_work_bytes(B, ctypes.byref(nb)), "pa_mlp_work_bytes")
        work = torch.zeros(int(nb.value), dtype=torch.uint8, device=DEV)
        g_ref = torch.full((learned.N_PARAMS,), np.nan, dtype=torch.float32, device=DEV)
        l_ref = torch.full((1,), np.nan, dtype=torch.float32, device=DEV)
        pa.check(pa.lib().pa_mlp_grad(w.data_ptr(), X.data_ptr(), t.data_ptr(), B, work.data_ptr(), g_ref.data_ptr(),
                                      l_ref.data_ptr(), s), "pa_mlp_grad")
        g = torch.full((learned.N_PARAMS,), np.nan, dtype=torch.float32, device=DEV)
        loss = torch.full((1,), np.nan, dtype=torch.float32, device=DEV)
        pa.check(pa.lib().pa_mlp_grad_static(w.data_ptr(), X.data_ptr(), t.data_ptr(), B, g.data_ptr(),
                                             loss.data_ptr(), s), "pa_mlp_grad_static")
        torch.cuda.synchronize()
        assert torch.isfinite(g_ref).all() and torch.isfinite(l_ref).all()
        assert torch.equal(g, g_ref), f"gradient differs at B={B}"
        assert torch.equal(loss, l_ref), f"loss differs at B={B}"
    # beyond the array: refused on the host, nothing launched
    B = pa.PA_MLP_STATIC_MAX_B + 1
    assert pa.lib().pa_mlp_grad_static(w.data_ptr(), X.data_ptr(), t.data_ptr(), B, g.data_ptr(), loss.data_ptr(),
                                       s) == pa.PA_ERR_SIZE
    assert pa.lib().pa_mlp_grad_static(w.data_ptr(), X.data_ptr(), t.data_ptr(), 0, g.data_ptr(), None,
                                       s) == pa.PA_ERR_ARG
