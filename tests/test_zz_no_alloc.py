"""The allocation-free P^{-1} entry point (nys_apply_static) against
nys_apply, through the C ABI: two calls in a row, the second on a smaller
preconditioner and fewer columns, each bit-identical to the workspace entry
point's result (same kernels, same summation order)."""
import ctypes as C

import pytest
import torch

import workloads as W
from gpu_util import banner, dev, host, need_gpu

pytestmark = pytest.mark.gpu


def _pc(P, n, ell, seed):
    op = P.Operator(P.OP_BLUR, n, n, psf=W.gaussian_psf(9, 1.5))
    om = dev(W.omega(ell, n, n, seed), "f32")
    return P.nys_factor(om, P.nys_sketch(op, om), ell, u_dtype=torch.float32)


def _static(P, pc, v, inverse):
    out = torch.empty_like(v)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = P.lib().nys_apply_static(pc.handle, 1 if inverse else 0, P.F32, C.c_void_p(v.data_ptr()),
                                 C.c_void_p(out.data_ptr()), v.shape[0], st)
    if r != 0:
        raise P.NysError(r, P.lib().nys_last_error().decode())
    return out


def test_static_apply_matches_workspace_apply():
    P = need_gpu()
    P.lib().nys_apply_static.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                         C.c_int64, C.c_void_p]
    P.lib().nys_apply_static.restype = C.c_int
    # first call: the largest shape the array holds (8 columns, ell = 100)
    for (n, ell, ncols, inverse, seed) in [(256, 100, 8, True, 60), (64, 16, 3, False, 61)]:
        banner(f"no-alloc apply n={n} ell={ell} ncols={ncols} inverse={inverse}")
        pc = _pc(P, n, ell, seed)
        v = dev(W.gaussian((ncols, n, n), seed + 1), "f32")
        got = _static(P, pc, v, inverse)
        want = P.nys_apply(pc, v, inverse=inverse)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, want), float((got - want).abs().max())
    # beyond the array's capacity: refused before any work
    pc = _pc(P, 32, 8, 62)
    v = dev(W.gaussian((9, 32, 32), 63), "f32")
    with pytest.raises(P.NysError) as e:
        _static(P, pc, v, True)
    assert e.value.status == 1
