"""Oracle of the unrolled WAPG map: its forward equals Alg. 3 as written in
oracle.solver, and its reverse-mode gradient matches central finite
differences (h = 1e-4 along a unit direction, FP64) in y and in lambda.  The
map is piecewise smooth (ball projections); a unit-norm direction keeps the
h = 1e-4 perturbation from switching projection cases."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import nystrom as onys
from oracle import solver as sv
from oracle import unrolled as ou


def _ct_problem(n=12, V=8, B=17, seed=3):
    wl = W.workload("ct256_tv_unrolled")
    prob, _ = sv.problem_from_workload(wl, seed=seed, n=n, views=V, bins=B)
    return prob


def _precond(prob, ell=4, seed=5):
    om = W.omega(ell, prob.n, prob.n, seed)
    Y = sv.sketch(prob, om).reshape(ell, -1)
    r = onys.nystrom(Y, om.reshape(ell, -1))
    return sv.Precond(r["U"], r["shat"], r["nu"], "sqrt")


@pytest.mark.parametrize("with_pc", [False, True])
def test_unrolled_forward_equals_alg3(with_pc):
    prob = _ct_problem()
    pc = _precond(prob) if with_pc else None
    lam = 2e-3
    prob.lam = lam
    L = sv.lipschitz(prob, pc, W.gaussian((prob.n, prob.n), 9), 200)
    alpha = 1.0 / (1.01 * L)
    x_ref, _ = sv.wapg(prob, pc, alpha, 4, inner=5, record_cost=False)
    x = ou.unrolled(prob, pc, alpha, 4, 5, torch.from_numpy(prob.y), torch.tensor(lam, dtype=torch.float64))
    assert np.allclose(x.numpy(), x_ref, rtol=0, atol=1e-12 * np.abs(x_ref).max())


@pytest.mark.parametrize("with_pc,aniso", [(False, False), (True, False), (True, True)])
def test_unrolled_gradient_matches_finite_differences(with_pc, aniso):
    prob = _ct_problem()
    pc = _precond(prob) if with_pc else None
    L = sv.lipschitz(prob, pc, W.gaussian((prob.n, prob.n), 9), 200)
    alpha = 1.0 / (1.01 * L)
    w = torch.from_numpy(W.gaussian((prob.n, prob.n), 10))
    dy = torch.from_numpy(W.gaussian(prob.y.shape, 11))
    dy = dy / torch.linalg.norm(dy)          # unit direction: h = 1e-4 stays off the kinks
    y0 = torch.from_numpy(prob.y)
    lam0 = 2e-3

    def loss(y, lam):
        x = ou.unrolled(prob, pc, alpha, 3, 4, y, lam, aniso=aniso)
        return torch.sum(w * x)

    y = y0.clone().requires_grad_(True)
    lam = torch.tensor(lam0, dtype=torch.float64, requires_grad=True)
    loss(y, lam).backward()
    h = 1e-4
    f64 = lambda v: torch.tensor(v, dtype=torch.float64)
    with torch.no_grad():
        fd_y = (loss(y0 + h * dy, f64(lam0)) - loss(y0 - h * dy, f64(lam0))) / (2 * h)
        fd_l = (loss(y0, f64(lam0 + h * lam0)) - loss(y0, f64(lam0 - h * lam0))) / (2 * h * lam0)
    g_y = float(torch.sum(y.grad * dy))
    assert abs(g_y - float(fd_y)) <= 1e-6 * max(1.0, abs(float(fd_y)))
    assert abs(float(lam.grad) - float(fd_l)) <= 1e-5 * max(1.0, abs(float(fd_l)))
