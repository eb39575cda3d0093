"""Failure reporting through the C ABI, forced from the host: every kernel
exits normally and only the status says what went wrong.

- NaN in the measurements: the solve's device status word (TV prior: the
  finite check of the iterate; l1 prior: the semismooth Newton decision of
  Thm. 1's iteration) -> NYS_ENOTFINITE;
- one Newton trial point for a prox that needs several -> NYS_ENOCONV;
- a workspace below the queried size, mismatched shapes or dtypes -> EINVAL
  before anything is enqueued.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import banner, dev, need_gpu
from oracle import solver as sv

pytestmark = pytest.mark.gpu

ENOTFINITE, ENOCONV, EINVAL = 4, 5, 1


def _deblur(P, n=32, dt="f64"):
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=2, n=n)
    op = P.Operator(P.OP_BLUR, n, n, psf=prob.h)
    return prob, op, dev(prob.y, dt)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_nan_in_measurements_tv_is_not_finite(dt):
    P = need_gpu()
    banner(f"status: NaN in y, TV, {dt}")
    prob, op, yd = _deblur(P, dt=dt)
    yd[3, 5] = float("nan")
    rd = P.reg_desc("tv", prob.n, prob.n, n_inner=5)
    with pytest.raises(P.NysError) as e:
        P.solve(op, yd, rd, prob.lam, None, 4, alpha=0.5)
    assert e.value.status == ENOTFINITE
    # the device is still usable: the same solve on clean data succeeds
    _, _, info = P.solve(op, dev(prob.y, dt), rd, prob.lam, None, 4, alpha=0.5)
    assert info["status"] == 0


def test_nan_in_measurements_l1_newton_is_not_finite():
    P = need_gpu()
    banner("status: NaN in y, l1 prox with a preconditioner")
    wl = W.workload("sr512_haar_bf16")
    prob, _ = sv.problem_from_workload(wl, seed=3, n=32)
    n, ell = 32, 8
    op = P.Operator(P.OP_BLURDOWN, n, n, psf=prob.h, factor=2, wavelet_levels=3)
    om = dev(W.omega(ell, n, n, 20), "f32")
    pc = P.nys_factor(om, P.nys_sketch(op, om), ell, u_dtype=torch.float32)
    yd = dev(prob.y, "f32")
    yd[2, 2] = float("nan")
    rd = P.reg_desc("l1", n, n)
    # least squares: the Huber derivative would clip the NaN residual away
    with pytest.raises(P.NysError) as e:
        P.solve(op, yd, rd, prob.lam, pc, 3, alpha=0.01, loss=P.LOSS_LS)
    assert e.value.status == ENOTFINITE
    # a clean solve on the same preconditioner afterwards converges as usual
    _, _, info = P.solve(op, dev(prob.y, "f32"), rd, prob.lam, pc, 3, alpha=0.01,
                         loss=P.LOSS_LS)
    assert info["status"] == 0


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_newton_trial_cap_is_reported(dt):
    P = need_gpu()
    banner(f"status: max_newton = 1, {dt}")
    n, ell = 32, 8
    h = W.gaussian_psf(7, 1.2)
    op = P.Operator(P.OP_BLURDOWN, n, n, psf=h, factor=2, wavelet_levels=3)
    om = dev(W.omega(ell, n, n, 16), dt)
    pc = P.nys_factor(om, P.nys_sketch(op, om), ell,
                      u_dtype=torch.float64 if dt == "f64" else torch.float32)
    s = dev(W.gaussian((n, n), 17) * 0.1, dt)
    # cold start: F(0) = -diag(e) U^T (soft(s) - s) != 0, so one trial point
    # cannot end the iteration
    with pytest.raises(P.NysError) as e:
        P.prox_weighted(P.reg_desc("l1", n, n, max_newton=1), 0.05, pc, s)
    assert e.value.status == ENOCONV
    x = P.prox_weighted(P.reg_desc("l1", n, n), 0.05, pc, s)
    assert torch.isfinite(x).all()


def test_workspace_and_shape_errors_are_einval():
    P = need_gpu()
    banner("status: workspace / shape errors")
    lib = P.lib()
    prob, op, yd = _deblur(P, dt="f32")
    n = prob.n
    x = torch.empty((n, n), dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    # the blur needs no workspace; the Haar composition does
    opw = P.Operator(P.OP_BLUR, n, n, psf=prob.h, wavelet_levels=2)
    need = C.c_size_t()
    assert lib.nys_op_workspace_size(opw.handle, P.F32, 1, C.byref(need)) == 0
    assert need.value > 0
    small = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = lib.op_forward(opw.handle, P.F32, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 1,
                       C.c_void_p(small.data_ptr()), need.value - 256, st)
    assert r == EINVAL and b"workspace" in lib.nys_last_error()
    # a preconditioner of another size, and a dtype that is not its U's
    om = dev(W.omega(4, 16, 16, 3), "f32")
    op16 = P.Operator(P.OP_BLUR, 16, 16, psf=prob.h)
    pc16 = P.nys_factor(om, P.nys_sketch(op16, om), 4, u_dtype=torch.float32)
    rd = P.reg_desc("tv", n, n)
    with pytest.raises(P.NysError) as e:
        P.solve(op, yd, rd, prob.lam, pc16, 2, alpha=0.5)
    assert e.value.status == EINVAL
    with pytest.raises(P.NysError) as e:
        P.nys_apply(pc16, torch.zeros((16, 16), dtype=torch.float64, device="cuda"))
    assert e.value.status == EINVAL
    torch.cuda.synchronize()
