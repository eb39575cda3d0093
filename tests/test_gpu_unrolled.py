"""GPU parity of the differentiable unrolled WAPG (C ABI unrolled_forward /
unrolled_backward behind torch.autograd.Function) against the FP64 oracle
(torch CPU reverse mode over the oracle's operators), and the A / A^T / P^{-1}
autograd wrappers against their adjoint identities."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import nystrom as onys
from oracle import solver as sv
from oracle import unrolled as ou
from gpu_util import TOL, banner, check, dev, host, need_gpu, rel

pytestmark = pytest.mark.gpu


def _case(P, dt, with_pc, n=24, V=12, B=35, ell=6, batch=2, aniso=False):
    wl = W.workload("ct256_tv_unrolled")
    probs = [sv.problem_from_workload(wl, seed=s, n=n, views=V, bins=B)[0] for s in range(batch)]
    prob = probs[0]
    op = P.Operator(P.OP_PARALLEL_BEAM, n, n, views=V, bins=B)
    y = np.stack([p.y for p in probs])
    yd = dev(y, dt)
    pc = opc = None
    if with_pc:
        om = W.omega(ell, n, n, 40)
        Yref = sv.sketch(prob, om)
        omd, Yd = dev(om, "f64"), dev(Yref, "f64")
        ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
        opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
        if dt == "f64":
            pc = P.nys_factor(omd, Yd, ell, u_dtype=torch.float64)
        else:
            pc = P.nys_factor(dev(om, "f32"), dev(Yref, "f32"), ell, u_dtype=torch.float32)
            # the oracle sees the rounded inputs of the FP32 factorisation
            r32 = onys.nystrom(host(dev(Yref, "f32")).reshape(ell, -1), host(dev(om, "f32")).reshape(ell, -1))
            opc = sv.Precond(r32["U"], r32["shat"], r32["nu"], "sqrt")
    L = sv.lipschitz(prob, opc, W.gaussian((n, n), 41), 200)
    alpha = 1.0 / (1.01 * L)
    lam = np.array([2e-3 * (1 + 0.5 * b) for b in range(batch)])
    kind = "tv_aniso" if aniso else "tv"
    rd = P.reg_desc(kind, n, n)
    return prob, op, yd, pc, opc, alpha, lam, rd


@pytest.mark.parametrize("dt,with_pc,aniso", [("f64", False, False), ("f64", True, False),
                                              ("f64", True, True), ("f32", True, False)])
def test_unrolled_forward_backward_match_oracle(dt, with_pc, aniso):
    P = need_gpu()
    banner(f"unrolled {dt} pc={with_pc} aniso={aniso}")
    K, nin = 3, 4
    prob, op, yd, pc, opc, alpha, lam, rd = _case(P, dt, with_pc, aniso=aniso)
    batch = yd.shape[0]
    y = yd.clone().requires_grad_(True)
    lt = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
    x = P.unrolled_wapg(op, y, lt, rd, pc, K, nin, alpha)
    w = W.gaussian(tuple(x.shape), 42)
    (x.double() * torch.from_numpy(w).cuda()).sum().backward()
    gy, gl = host(y.grad), lt.grad.cpu().numpy()
    tol_f = 1e-10 if dt == "f64" else 1e-5
    tol_g = 1e-9 if dt == "f64" else 1e-5
    for b in range(batch):
        yb = torch.from_numpy(host(yd)[b]).requires_grad_(True)
        lb = torch.tensor(lam[b], dtype=torch.float64, requires_grad=True)
        xr = ou.unrolled(prob, opc, alpha, K, nin, yb, lb, aniso=aniso)
        check(host(x)[b], xr.detach().numpy(), tol_f, what="x")
        (xr * torch.from_numpy(w[b])).sum().backward()
        check(gy[b], yb.grad.numpy(), tol_g, what="dL/dy")
        # dL/dlambda is one inner product summed over every unrolled step
        # (terms of both signs): measured 1.2e-5 relative in FP32
        tol_l = tol_g if dt == "f64" else 5e-5
        assert abs(gl[b] - float(lb.grad)) <= tol_l * abs(float(lb.grad))


def test_unrolled_full_size_gradient_by_finite_differences():
    """256^2 phantoms, 180 views x 367 bins, ell = 48, 20 unrolled iterations,
    batch of 8, as timed: the FP64 GPU gradient against central differences
    of the GPU forward (h = 1e-4 along unit directions), and FP32 against FP64."""
    P = need_gpu()
    banner("unrolled full size 256^2 180x367 ell=48 K=20 batch=8")
    n, V, B, ell, K, nin, batch = 256, 180, 367, 48, 20, 10, 8
    wl = W.workload("ct256_tv_unrolled")
    op = P.Operator(P.OP_PARALLEL_BEAM, n, n, views=V, bins=B)
    ys = []
    for s in range(batch):
        xt = torch.from_numpy(W.phantom_ellipses(n, s)).cuda()
        clean = P.op_forward(op, xt)
        noise = torch.from_numpy(W.gaussian(tuple(clean.shape), s)).cuda()
        ys.append(clean + wl.noise_rel_max * float(clean.abs().max()) * noise)
    y64 = torch.stack(ys).contiguous()
    om = torch.from_numpy(W.omega(ell, n, n, 43)).cuda()
    Y = P.nys_sketch(op, om)
    pc64 = P.nys_factor(om, Y, ell, u_dtype=torch.float64)
    pc32 = P.nys_factor(om.float(), Y.float(), ell, u_dtype=torch.float32)
    rd = P.reg_desc("tv", n, n)
    v0 = torch.from_numpy(W.gaussian((n, n), 49)).cuda()
    _, _, info = P.solve(op, y64[0].contiguous(), rd, 2e-4, pc64, 0, power_v0=v0, power_iters=60,
                         record_cost=False)
    alpha = info["alpha"]
    lam = torch.full((batch,), 2e-4, dtype=torch.float64)
    wv = torch.from_numpy(W.gaussian((batch, n, n), 44)).cuda()
    y = y64.clone().requires_grad_(True)
    lt = lam.clone().requires_grad_(True)
    x = P.unrolled_wapg(op, y, lt, rd, pc64, K, nin, alpha)
    (x * wv).sum().backward()
    dy = torch.from_numpy(W.gaussian(tuple(y64.shape), 45)).cuda()
    dy = dy / torch.linalg.norm(dy)
    h = 1e-4

    def f(yy, ll):
        with torch.no_grad():
            return float((P.unrolled_wapg(op, yy, ll, rd, pc64, K, nin, alpha) * wv).sum())

    fd_y = (f(y64 + h * dy, lam) - f(y64 - h * dy, lam)) / (2 * h)
    assert abs(float((y.grad * dy).sum()) - fd_y) <= 1e-6 * max(1.0, abs(fd_y))
    e0 = torch.zeros(batch, dtype=torch.float64)
    e0[0] = 1.0
    fd_l = (f(y64, lam * (1 + h * e0)) - f(y64, lam * (1 - h * e0))) / (2 * h * lam[0].item())
    assert abs(float(lt.grad[0]) - fd_l) <= 1e-5 * max(1.0, abs(fd_l))
    # FP32 path against FP64
    y32 = y64.float().requires_grad_(True)
    l32 = lam.clone().requires_grad_(True)
    x32 = P.unrolled_wapg(op, y32, l32, rd, pc32, K, nin, alpha)
    (x32 * wv.float()).sum().backward()
    check(host(x32), host(x), 1e-5, what="FP32 x vs FP64")
    check(host(y32.grad), host(y.grad), 1e-5, what="FP32 dL/dy vs FP64")


@pytest.mark.parametrize("kind", ["ct", "blurdown_haar"])
def test_operator_autograd_is_adjoint(kind):
    P = need_gpu()
    banner(f"operator autograd {kind}")
    if kind == "ct":
        op = P.Operator(P.OP_PARALLEL_BEAM, 32, 32, views=20, bins=45)
    else:
        op = P.Operator(P.OP_BLURDOWN, 32, 32, psf=W.gaussian_psf(5, 1.0), factor=2, wavelet_levels=3)
    x = dev(W.gaussian((2, 32, 32), 46)).requires_grad_(True)
    y = P.OpForwardFn.apply(x, op)
    r = dev(W.gaussian(tuple(y.shape), 47))
    (y * r).sum().backward()
    check(host(x.grad), host(P.op_adjoint(op, r)), 1e-12)
    yy = r.clone().requires_grad_(True)
    xx = P.OpAdjointFn.apply(yy, op)
    g = dev(W.gaussian(tuple(xx.shape), 48))
    (xx * g).sum().backward()
    check(host(yy.grad), host(P.op_forward(op, g)), 1e-12)
    # <A x, r> = <x, A^T r> in the GPU arithmetic
    lhs = float((P.op_forward(op, x.detach()) * r).sum())
    rhs = float((x.detach() * P.op_adjoint(op, r)).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_unrolled_full_size_gradient_matches_oracle():
    """The timed configuration (256^2 phantom, 180 views x 367 bins, ell = 48,
    20 outer x 10 dual iterations), one sinogram: the FP64 x_K and the
    gradients with respect to y and lambda against the oracle's reverse pass,
    both sides on the preconditioner of the oracle's own sketch."""
    P = need_gpu()
    banner("unrolled full size vs oracle 256^2 180x367 ell=48 K=20")
    n, V, B, ell, K, nin = 256, 180, 367, 48, 20, 10
    wl = W.workload("ct256_tv_unrolled")
    prob, _ = sv.problem_from_workload(wl, seed=0, n=n, views=V, bins=B)
    om = W.omega(ell, n, n, 43)
    Yref = sv.sketch(prob, om)
    ref = onys.nystrom(Yref.reshape(ell, -1), om.reshape(ell, -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    pc = P.nys_factor(dev(om), dev(Yref), ell, u_dtype=torch.float64)
    # a step below 1 / L (L from a few oracle power steps, approached from below)
    alpha = 1.0 / (1.5 * sv.lipschitz(prob, opc, W.gaussian((n, n), 49), 8))
    op = P.Operator(P.OP_PARALLEL_BEAM, n, n, views=V, bins=B)
    rd = P.reg_desc("tv", n, n)
    lam = float(prob.lam)
    w = W.gaussian((1, n, n), 44)
    y = dev(prob.y[None]).requires_grad_(True)
    lt = torch.tensor([lam], dtype=torch.float64, requires_grad=True)
    x = P.unrolled_wapg(op, y, lt, rd, pc, K, nin, alpha)
    (x * torch.from_numpy(w).cuda()).sum().backward()
    yb = torch.from_numpy(np.asarray(prob.y, np.float64)).requires_grad_(True)
    lb = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
    xr = ou.unrolled(prob, opc, alpha, K, nin, yb, lb)
    (xr * torch.from_numpy(w[0])).sum().backward()
    check(host(x)[0], xr.detach().numpy(), TOL["f64"], what="x_K")
    check(host(y.grad)[0], yb.grad.numpy(), 1e-9, what="dL/dy")
    gl, gr = float(lt.grad[0]), float(lb.grad)
    banner(f"dL/dlambda gpu {gl:.12e} oracle {gr:.12e}")
    # one scalar summed over 200 dual steps of 65536 pixels with cancellation
    # (measured 1.2e-9 relative in FP64)
    assert abs(gl - gr) <= 1e-8 * abs(gr)
