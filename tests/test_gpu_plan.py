"""The captured fixed-count solve (nys_solve_plan_*): its replays give the
results of `solve` with the same arguments bit for bit (the same kernels in
the same order, the momentum weights and cost slots read through a device
counter), and those results match the FP64 oracle of WAPG (Alg. 3)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import nystrom as onys
from oracle import solver as sv
from gpu_util import TOL, banner, check, dev, host, need_gpu, rel

pytestmark = pytest.mark.gpu
EINVAL = 1


def _pc_for(P, prob, n, ell, dt, seed):
    om = W.omega(ell, n, n, seed)
    omd = dev(om, dt)
    Yd = dev(sv.sketch(prob, host(omd)), dt)
    ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    pc = P.nys_factor(omd, Yd, ell, u_dtype=torch.float64 if dt == "f64" else torch.float32)
    return opc, pc


def _replays_match_solve(P, op, yd, rd, lam, pc, iters, alpha):
    """Two plan runs with an eager solve between them, each against solve."""
    plan = P.SolvePlan(op, yd, rd, lam, pc, iters, alpha=alpha)
    x0, c0, info = P.solve(op, yd, rd, lam, pc, iters, alpha=alpha)
    assert info["status"] == 0
    for rep in range(2):
        x, c = plan.run()
        torch.cuda.synchronize()
        assert plan.status() == 0
        assert torch.equal(x, x0), f"replay {rep}: x differs from solve"
        assert torch.equal(c, c0), f"replay {rep}: costs differ from solve"
        if rep == 0:   # eager work on the same stream between the replays
            P.solve(op, yd, rd, lam, pc, 3, alpha=alpha)
    return host(x0), host(c0)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_plan_tv_deblur_with_preconditioner(dt):
    """40^2 deblurring, TV, ell = 10, 37 iterations: two 16-iteration chunks
    and a remainder of 5."""
    P = need_gpu()
    banner(f"solve plan TV deblur {dt}")
    n, ell, iters = 40, 10, 37
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=2, n=n)
    op = P.Operator(P.OP_BLUR, n, n, psf=prob.h)
    yd = dev(prob.y, dt)
    prob.y = host(yd)
    opc, pc = _pc_for(P, prob, n, ell, dt, 20)
    alpha = 0.9 / sv.lipschitz(prob, opc, W.gaussian((n, n), 21), 200)
    rd = P.reg_desc("tv", n, n, n_inner=10)
    x, c = _replays_match_solve(P, op, yd, rd, prob.lam, pc, iters, alpha)
    xr, cr = sv.wapg(prob, opc, alpha, iters, inner=10)
    check(x, xr, TOL[dt], what="x")
    check(c, cr, TOL[dt], what="costs")


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("warm", [True, False])
def test_solve_prox_warm_and_cold_start(dt, warm):
    """The solver keeps the warm start's coefficients d . U^T L^T Q from the
    previous prox (and clears them with Q at the start); with warm_start off
    every prox starts from Q = 0.  Both against the oracle's WAPG with the
    same start, and the plan's replays against solve."""
    P = need_gpu()
    banner(f"solve TV deblur warm={warm} {dt}")
    n, ell, iters = 40, 10, 21
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=3, n=n)
    op = P.Operator(P.OP_BLUR, n, n, psf=prob.h)
    yd = dev(prob.y, dt)
    prob.y = host(yd)
    opc, pc = _pc_for(P, prob, n, ell, dt, 22)
    alpha = 0.9 / sv.lipschitz(prob, opc, W.gaussian((n, n), 23), 200)
    rd = P.reg_desc("tv", n, n, n_inner=6)
    x0, c0, info = P.solve(op, yd, rd, prob.lam, pc, iters, alpha=alpha, warm_start=warm)
    assert info["status"] == 0
    plan = P.SolvePlan(op, yd, rd, prob.lam, pc, iters, alpha=alpha, warm_start=warm)
    x, c = plan.run()
    torch.cuda.synchronize()
    assert torch.equal(x, x0) and torch.equal(c, c0)
    xr, cr = sv.wapg(prob, opc, alpha, iters, inner=6, warm_start=warm)
    check(host(x0), xr, TOL[dt], what="x")
    check(host(c0), cr, TOL[dt], what="costs")


def test_plan_ct_hs1_f32():
    """32^2 parallel-beam CT (36 views, 48 bins), HS1, ell = 10, 20 iterations."""
    P = need_gpu()
    banner("solve plan CT HS1 f32")
    wl = W.workload("ct512_hs1_f32")
    prob, _ = sv.problem_from_workload(wl, seed=4, n=32, views=36, bins=48)
    n, ell, iters = 32, 10, 20
    op = P.Operator(P.OP_PARALLEL_BEAM, n, n, views=36, bins=48)
    yd = dev(prob.y, "f32")
    prob.y = host(yd)
    opc, pc = _pc_for(P, prob, n, ell, "f32", 20)
    alpha = 0.9 / sv.lipschitz(prob, opc, W.gaussian((n, n), 21), 200)
    rd = P.reg_desc("hs1", n, n, n_inner=10)
    x, c = _replays_match_solve(P, op, yd, rd, prob.lam, pc, iters, alpha)
    xr, cr = sv.wapg(prob, opc, alpha, iters, inner=10)
    check(x, xr, TOL["f32"], what="x")
    check(c, cr, TOL["f32"], what="costs")


def test_plan_plain_with_power_method():
    """No preconditioner, the step from the power method at creation, 5
    iterations (one chunk shorter than 16)."""
    P = need_gpu()
    banner("solve plan plain APG, power method")
    n = 32
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=3, n=n)
    op = P.Operator(P.OP_BLUR, n, n, psf=prob.h)
    yd = dev(prob.y, "f32")
    v0 = dev(W.gaussian((n, n), 9), "f32")
    rd = P.reg_desc("tv", n, n, n_inner=8)
    plan = P.SolvePlan(op, yd, rd, prob.lam, None, 5, power_v0=v0, power_iters=50)
    x0, c0, info = P.solve(op, yd, rd, prob.lam, None, 5, power_v0=v0, power_iters=50)
    assert plan.info["alpha"] == info["alpha"]
    x, c = plan.run()
    torch.cuda.synchronize()
    assert torch.equal(x, x0) and torch.equal(c, c0)


@pytest.mark.parametrize("n,ell,iters", [(64, 8, 20), (512, 64, 6)])
def test_plan_l1_super_resolution_f32(n, ell, iters):
    """The super-resolution problem (blur + 2x decimation, Haar-3, Huber, FP32)
    with the P-weighted l1 prox: the captured semismooth Newton trials decide
    on the device.  The plan's iterates against the oracle's FP64 ones; at
    512^2, ell = 64 the launch configuration of the workload."""
    P = need_gpu()
    banner(f"solve plan l1 SR n={n} ell={ell} f32")
    wl = W.workload("sr512_haar_bf16")
    prob, _ = sv.problem_from_workload(wl, seed=3, n=n if n != 512 else None)
    assert prob.n == n
    op = P.Operator(P.OP_BLURDOWN, n, n, psf=prob.h, factor=2, wavelet_levels=3)
    yd = dev(prob.y, "f32")
    prob.y = host(yd)
    om = W.omega(ell, n, n, 20)
    Yref = sv.sketch(prob, om)
    ref = onys.nystrom(Yref.reshape(ell, -1), om.reshape(ell, -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    pc = P.nys_factor(dev(om, "f32"), dev(Yref, "f32"), ell, u_dtype=torch.float32)
    alpha = 0.9 / sv.lipschitz(prob, opc, W.gaussian((n, n), 21), 60)
    rd = P.reg_desc("l1", n, n)
    plan = P.SolvePlan(op, yd, rd, prob.lam, pc, iters, alpha=alpha, loss=P.LOSS_HUBER,
                       delta=prob.delta)
    xr, cr = sv.wapg(prob, opc, alpha, iters, ssn_tol=1e-10)
    for rep in range(2):
        x, c = plan.run()
        torch.cuda.synchronize()
        assert plan.status() == 0
        ex, ec = rel(host(x), xr), np.max(np.abs(host(c) - cr) / np.abs(cr))
        banner(f"plan l1 replay {rep}: x rel err {ex:.2e}, cost rel err {ec:.2e}")
        assert ex < 2e-6 and ec < 1e-7    # the bounds of the host-driven solve's test
        if rep == 0:
            P.solve(op, yd, rd, prob.lam, pc, 2, alpha=alpha, loss=P.LOSS_HUBER, delta=prob.delta)


def test_plan_refuses_the_weighted_box_projection():
    """The P-weighted projection onto a box takes its semismooth Newton
    decisions on the host: no plan for it."""
    P = need_gpu()
    banner("solve plan: box with P is EINVAL")
    n, ell = 32, 6
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=2, n=n)
    op = P.Operator(P.OP_BLUR, n, n, psf=prob.h)
    yd = dev(prob.y, "f32")
    _, pc = _pc_for(P, prob, n, ell, "f32", 5)
    rd = P.reg_desc("tv", n, n, box=(0.0, 1.0))
    with pytest.raises(P.NysError) as e:
        P.SolvePlan(op, yd, rd, prob.lam, pc, 4, alpha=0.5)
    assert e.value.status == EINVAL


def _sr_small(P, n=32, ell=8):
    wl = W.workload("sr512_haar_bf16")
    prob, _ = sv.problem_from_workload(wl, seed=3, n=n)
    op = P.Operator(P.OP_BLURDOWN, n, n, psf=prob.h, factor=2, wavelet_levels=3)
    om = dev(W.omega(ell, n, n, 20), "f32")
    pc = P.nys_factor(om, P.nys_sketch(op, om), ell, u_dtype=torch.float32)
    return prob, op, pc


def test_plan_l1_reports_unconverged_newton_on_the_device():
    """A Newton tolerance no trial can meet: every captured prox call runs out
    of its trials, goes on from its last accepted point, and the run's second
    status word says NYS_ENOCONV; the iterate stays finite."""
    P = need_gpu()
    banner("solve plan: l1 prox out of trials -> ENOCONV")
    prob, op, pc = _sr_small(P)
    rd = P.reg_desc("l1", prob.n, prob.n, newton_tol=1e-30)
    plan = P.SolvePlan(op, dev(prob.y, "f32"), rd, prob.lam, pc, 3, alpha=0.01,
                       loss=P.LOSS_LS)
    x, _ = plan.run()
    torch.cuda.synchronize()
    assert plan.status() == 5          # NYS_ENOCONV
    assert torch.isfinite(x).all()


def test_plan_reports_non_finite_iterates():
    """NaN in the measurements: the run's final check sets NYS_ENOTFINITE in
    the first status word (the captured Newton trials meet a non-finite ||F||
    and keep the warm start).  The clean plan is made first, so that the
    preconditioner's Newton factors are stored before the NaN plan is
    captured (its creation then runs no iteration on the host)."""
    P = need_gpu()
    banner("solve plan: NaN in y -> ENOTFINITE")
    prob, op, pc = _sr_small(P)
    rd = P.reg_desc("l1", prob.n, prob.n)
    good = P.SolvePlan(op, dev(prob.y, "f32"), rd, prob.lam, pc, 3, alpha=0.01, loss=P.LOSS_LS)
    x, _ = good.run()
    torch.cuda.synchronize()
    assert good.status() == 0 and torch.isfinite(x).all()
    yd = dev(prob.y, "f32")
    yd[2, 2] = float("nan")
    bad = P.SolvePlan(op, yd, rd, prob.lam, pc, 3, alpha=0.01, loss=P.LOSS_LS)
    bad.run()
    torch.cuda.synchronize()
    assert bad.status() == 4           # NYS_ENOTFINITE
    x, _ = good.run()                  # the preconditioner is still usable
    torch.cuda.synchronize()
    assert good.status() == 0 and torch.isfinite(x).all()
