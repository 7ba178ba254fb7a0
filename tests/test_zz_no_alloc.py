"""expenc_forward_static (the forward with the library's static scratch, for
callers that cannot allocate) against expenc_forward with a caller workspace,
through the C ABI: two calls in a row on one device, the second on a smaller
operator (so it runs on scratch that still holds the first call's contents),
in the FP32 and fp16 split forms; the small one also against the FP64 oracle.
The 1.5 mm FP32 forward needs more partial-sum space than the default split
gives inside the scratch, so the call lowers its split (summation order only
differs).  An operator whose forward cannot fit is rejected before any launch."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import encoding
from tests.gpu_common import Case, rel

pytestmark = pytest.mark.gpu


def _static_forward(case, x, prec):
    import torch
    import paper_2211_07532_amd as ee
    from paper_2211_07532_amd import _binding as b
    op = case.op
    y = torch.empty((1, op.nsamples, op.ncoils), dtype=torch.complex64, device=case.dev)
    st = b.lib().expenc_forward_static(ctypes.byref(op._c), 1, ee.expenc._prec(prec), ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(y.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    b.check(st, "expenc_forward_static")
    return y[0]


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_static_forward_matches_workspace_forward(prec):
    import paper_2211_07532_amd as ee
    bar = 1e-6 if prec == "fp32" else 1e-5
    big = Case(synth.MM15, sh=True)
    small = Case(synth.TINY, sh=True)
    for case in (big, small):
        x = case.to_dev(case.x_noisy)
        print(f"[case] static forward {prec} {case.w.name}", flush=True)
        got = _static_forward(case, x, prec).cpu().numpy()
        ref = ee.forward(x, case.op, precision=prec).cpu().numpy()
        e = rel(got, ref)
        print(f"  static vs workspace forward: {e:.2e}", flush=True)
        assert np.all(np.isfinite(got)) and e <= bar
    y_or = encoding.forward(small.x_noisy, *small.oracle_args())
    e = rel(got, y_or)
    print(f"  small operator vs FP64 oracle: {e:.2e}", flush=True)
    assert e <= (1e-5 if prec == "fp32" else 1e-4)


def test_static_forward_rejects_operators_that_do_not_fit():
    import torch
    from paper_2211_07532_amd import _binding as b
    op = b.ExpencOp()
    op.nx = op.ny = 200
    op.ncoils, op.nbasis, op.nsamples = 32, 16, 40000
    op.coef = op.time = op.smaps = 0x1000  # never dereferenced: the plan is rejected first
    op.basis_kind = b.BASIS_SH
    op.fov_x = op.fov_y = 0.22
    x = torch.zeros(200 * 200, dtype=torch.complex64, device="cuda")
    st = b.lib().expenc_forward_static(ctypes.byref(op), 1, b.FP32, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(x.data_ptr()), None)
    assert st == b.EXPENC_EWORKSPACE
    assert b"static scratch" in b.lib().expenc_last_error()
