"""The forward transform that allocates nothing (mifft_execute_forward_static,
workspace in the library's static device array) against the same transform
with a caller workspace (mifft_execute_forward_ws): bit-equal results on two
calls in a row, the second with a smaller grid, and the oracle's bar."""
import ctypes

import numpy as np
import pytest

import oracle
from conftest import TOL, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _plan(L, shape, prec):
    from paper_1506_07933_amd._lib import MIFFT_C2C, MIFFT_FP32, MIFFT_FP64
    p = ctypes.c_void_p()
    rc = L.mifft_plan_create(ctypes.byref(p), shape[0], shape[1], shape[2], MIFFT_C2C,
                             MIFFT_FP64 if prec == "fp64" else MIFFT_FP32, 0)
    assert rc == 0, L.mifft_last_error()
    return p


@pytest.mark.parametrize("order", ["large_then_small"])
def test_static_scratch_forward_matches_workspace_forward(order):
    from paper_1506_07933_amd import synth
    from paper_1506_07933_amd._lib import lib as L
    cases = [((256, 256, 256), "fp64", np.complex128),   # workspace 256 MiB: the whole array
             ((96, 256, 256), "fp32", np.complex64)]     # 48 MiB, a smaller call after it
    for shape, prec, dt in cases:
        print("  case", shape, prec, flush=True)
        p = _plan(L, shape, prec)
        try:
            ws_bytes = L.mifft_workspace_bytes(p)
            assert 0 < ws_bytes <= 256 << 20
            x = synth.uniform_complex(shape, dt, seed=5)
            xd = torch.from_numpy(x).to(DEV)
            y_static = torch.empty_like(xd)
            y_ws = torch.empty_like(xd)
            ws = torch.empty(ws_bytes, dtype=torch.uint8, device=DEV)
            s = torch.cuda.current_stream().cuda_stream
            assert L.mifft_execute_forward_static(p, xd.data_ptr(), y_static.data_ptr(), s) == 0, \
                L.mifft_last_error()
            assert L.mifft_execute_forward_ws(p, xd.data_ptr(), y_ws.data_ptr(), ws.data_ptr(), s) == 0
            torch.cuda.synchronize()
            assert torch.equal(y_static, y_ws), "static-scratch result differs from the workspace call"
            if shape[0] <= 96:
                e = rel_l2(y_static.cpu().numpy(), oracle.fft3d_c2c(x.astype(np.complex128), -1))
                print("  %s %s rel_l2 vs oracle %.3e" % (shape, prec, e), flush=True)
                assert e <= TOL[prec]
        finally:
            assert L.mifft_plan_destroy(p) == 0
