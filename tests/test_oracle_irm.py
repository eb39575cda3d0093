"""Pins of the IRM + PCG oracle (Alg. 2) against what the mathematics fixes:
the half-quadratic identity behind the weights, CG against a dense solve,
exact preconditioning, the p = q = 2 reduction to one linear solve, and the
majorise-minimise descent of the smoothed objective with exact x-updates."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import workloads as W
from oracle import irm as oi
from oracle import operators as ops


@pytest.mark.parametrize("p", [0.5, 1.0, 1.5])
@pytest.mark.parametrize("r", [0.03, 0.7, 2.5])
def test_half_quadratic_identity_and_weight(p, r):
    """min_{beta>0} beta r^2 + 1/(b_p beta^a_p) = |r|^p at beta* = p/2 |r|^(p-2),
    so the x-update weight (2/p) beta* is |r|^(p-2)."""
    a, b = oi.half_quadratic_constants(p)
    f = lambda lb: np.exp(lb) * r * r + 1.0 / (b * np.exp(lb) ** a)
    res = minimize_scalar(f, bounds=(-40, 40), method="bounded",
                          options={"xatol": 1e-12})
    assert abs(res.fun - abs(r) ** p) < 1e-9 * max(1.0, abs(r) ** p)
    beta = p / 2.0 * abs(r) ** (p - 2.0)
    assert abs(np.exp(res.x) - beta) < 1e-5 * beta
    assert abs(oi.weights(np.array(r), p, 0.0) - 2.0 / p * beta) < 1e-12 * beta


def test_pcg_matches_dense_solve_and_exact_preconditioner():
    g = W.rng(5, 0)
    M = g.standard_normal((40, 40))
    S = M @ M.T + 0.1 * np.eye(40)
    b = g.standard_normal(40)
    x, it = oi.pcg(lambda v: S @ v, b, np.zeros(40), 1e-13, 500)
    assert np.allclose(x, np.linalg.solve(S, b), rtol=1e-9, atol=1e-10)
    assert it <= 200
    Sinv = np.linalg.inv(S)
    x1, it1 = oi.pcg(lambda v: S @ v, b, np.zeros(40), 1e-10, 50, pinv=lambda v: Sinv @ v)
    assert it1 == 1
    assert np.allclose(x1, np.linalg.solve(S, b), rtol=1e-9)


def _small_deblur(n, seed):
    h = W.gaussian_psf(5, 1.2)
    xt = W.phantom_blocks(n, seed)
    y = ops.blur(xt, h) + 0.01 * W.gaussian((n, n), seed)
    A = lambda v: ops.blur(v, h)
    At = lambda v: ops.blur_adjoint(v, h)
    return A, At, y


def _dense(op, n):
    E = np.eye(n * n).reshape(n * n, n, n)
    return np.stack([np.asarray(op(e)).reshape(-1) for e in E], axis=1)


def test_p_q_2_is_one_linear_solve():
    """With p = q = 2 every weight is 1 and one x-update solves the normal
    equations (A^T A + lambda L^T L) x = A^T y exactly."""
    n, lam = 12, 0.05
    A, At, y = _small_deblur(n, 31)
    r = oi.irm(A, At, y, lam, 2.0, 2.0, 1e-6, np.zeros((n, n)), 1, 0.0, 1e-13, 2000)
    Am = _dense(A, n)
    Lm = np.stack([ops.grad(e.reshape(n, n)).reshape(-1) for e in np.eye(n * n)], axis=1)
    H = Am.T @ Am + lam * Lm.T @ Lm
    xs = np.linalg.solve(H, Am.T @ y.reshape(-1))
    assert np.allclose(r.x.reshape(-1), xs, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("p,q", [(1.0, 1.0), (0.5, 1.0)])
def test_exact_updates_decrease_the_smoothed_objective(p, q):
    """The x-update minimises a majoriser of the smoothed objective (the
    half-quadratic form is concave in r^2), so with exact solves the
    objective never increases."""
    n, lam, eps = 16, 0.03, 1e-6
    A, At, y = _small_deblur(n, 32)
    vals = []
    x = np.zeros((n, n))
    vals.append(oi.lp_objective(x, A, y, lam, p, q, eps))
    for _ in range(6):
        x = oi.irm(A, At, y, lam, p, q, eps, x, 1, 0.0, 1e-12, 5000).x
        vals.append(oi.lp_objective(x, A, y, lam, p, q, eps))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(vals, vals[1:]))
    assert vals[-1] < 0.5 * vals[0]


def test_full_sketch_preconditioner_solves_in_few_iterations():
    """With a sketch as large as the problem the Nystrom approximation is
    Phi_k itself, so P^{-1} Phi_k has (up to the shift) one eigenvalue and
    PCG stops after at most two iterations; plain CG needs many more."""
    n, lam, eps = 8, 0.02, 1e-6
    A, At, y = _small_deblur(n, 33)
    om = W.omega(n * n, n, n, 34)
    x0 = W.gaussian((n, n), 35)
    r_pc = oi.irm(A, At, y, lam, 1.0, 1.0, eps, x0, 1, 0.0, 1e-8, 500, omega=om)
    r_cg = oi.irm(A, At, y, lam, 1.0, 1.0, eps, x0, 1, 0.0, 1e-8, 500)
    assert r_pc.cg_iters[0] <= 2
    assert r_cg.cg_iters[0] > 5 * r_pc.cg_iters[0]
    # both stop on the residual of the same system (dense check)
    wf = oi.weights(A(x0) - y, 1.0, eps)
    wg = oi.weights(ops.grad(x0), 1.0, eps)
    phi = lambda v: (At(wf * A(v)) + lam * ops.grad_adjoint(wg * ops.grad(v))).reshape(-1)
    H = np.stack([phi(e.reshape(n, n)) for e in np.eye(n * n)], axis=1)
    b = At(wf * y).reshape(-1)
    for r in (r_pc, r_cg):
        assert np.linalg.norm(b - H @ r.x.reshape(-1)) <= 1.01e-8 * np.linalg.norm(b)
