"""offt_exec_noalloc, the transform that allocates nothing (its twiddle tables
in a file-scope device array), called through the C ABI and compared with
offt_exec_fwd / offt_exec_bwd of a plan of the same heuristic: bit for bit,
on two calls in a row, the second with a smaller grid (which rewrites the
shared array), forward and normalised backward, both precisions."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1501_07350_amd as offt
import synth
from paper_1501_07350_amd import _lib

pytestmark = pytest.mark.gpu


def noalloc(shape, dtype, batch, direction, normalize, x, out):
    code = 0 if dtype == torch.complex128 else 1
    rc = _lib.load().offt_exec_noalloc(*shape, code, batch, direction, normalize, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream)))
    _lib.check(rc, "offt_exec_noalloc")
    return out


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_noalloc_matches_planned_exec_on_two_calls(dtype):
    for shape, batch in (((64, 48, 80), 2), ((16, 12, 10), 1)):
        x = synth.complex_grid((batch,) + shape, dtype, device="cuda")
        plan = offt.Plan(shape, dtype=dtype, batch=batch, normalize_inverse=True)
        want_f = plan.forward(x)
        want_b = plan.backward(want_f)
        got_f = noalloc(shape, dtype, batch, offt.FORWARD, 0, x, torch.empty_like(x))
        got_b = noalloc(shape, dtype, batch, offt.BACKWARD, 1, got_f, torch.empty_like(x))
        torch.cuda.synchronize()
        assert torch.equal(got_f, want_f), shape
        assert torch.equal(got_b, want_b), shape
        ref = oracle.fft3_batch(x.cpu().numpy().astype(np.complex128))
        assert oracle.rel_l2(got_f.cpu().numpy(), ref) <= oracle.tolerance(int(np.prod(shape)),
                                                                           dtype == torch.complex64)
        plan.close()


def test_noalloc_rejects_bad_arguments():
    x = torch.zeros((4, 4, 4), dtype=torch.complex64, device="cuda")
    lib = _lib.load()
    for args in ((4, 4, 7, 1, 1, offt.FORWARD, 0), (4, 4, 2048, 1, 1, offt.FORWARD, 0),
                 (4, 4, 4, 1, 1, 0, 0), (4, 4, 4, 1, 1, offt.FORWARD, 2), (4, 4, 4, 1, 0, offt.FORWARD, 0)):
        rc = lib.offt_exec_noalloc(*args, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), None)
        assert rc in (_lib.ERR_INVALID_ARG, _lib.ERR_UNSUPPORTED_SIZE), args
