"""Pins of the oracle's weighted proximal maps and of WAPG."""
import numpy as np
import pytest

import workloads as W
from oracle import nystrom as nys
from oracle import operators as ops
from oracle import prox as px
from oracle import solver as sv


def _small_precond(N, K, seed, tail="sqrt"):
    Q, _ = np.linalg.qr(W.gaussian((N, K), seed))
    U = Q.T
    shat = np.linspace(3.0, 0.5, K)
    return sv.Precond(U, shat, 1e-9, tail)


# --- dual FISTA prox ------------------------------------------------------

@pytest.mark.parametrize("reg", ["tv", "hs1", "tv_aniso", "hs2", "hsinf"])
def test_dual_prox_gap_nonnegative_and_vanishing(reg):
    n = 12
    s = W.gaussian((n, n), 1)
    pc = _small_precond(n * n, 5, 2)
    lam_bar = 0.3
    gaps = []
    for it in (5, 50, 2000):
        x, Q = px.prox_mixed_dual(s, lam_bar, reg, pc.pinv, pc.pinv_norm, it)
        gaps.append(px.dual_gap(s, x, Q, lam_bar, reg, pc.p, pc.pinv))
    assert all(g >= -1e-10 for g in gaps)
    assert gaps[-1] < 1e-5 * (1 + abs(gaps[0])) and gaps[-1] < gaps[1] < gaps[0]


def test_dual_prox_large_lambda_gives_weighted_mean():
    # for huge lambda_bar the solution is the constant minimising ||c1 - s||_P
    n = 8
    s = W.gaussian((n, n), 3)
    pc = _small_precond(n * n, 4, 4)
    x, _ = px.prox_mixed_dual(s, 1e4, "tv", pc.pinv, pc.pinv_norm, 20000)
    one = np.ones((n, n))
    c = np.sum(pc.p(one) * s) / np.sum(pc.p(one) * one)
    assert np.allclose(x, c, atol=1e-6)


def test_dual_prox_plain_tiny_lambda_is_identity():
    s = W.gaussian((10, 10), 5)
    x, _ = px.prox_mixed_dual(s, 1e-12, "hs1", lambda v: v, 1.0, 10)
    assert np.allclose(x, s, atol=1e-10)


def test_projections_closed_forms():
    q = W.gaussian((2, 6, 6), 6) * 3
    p = px.project_dual_ball(q, "tv")
    nrm = np.sqrt(p[0] ** 2 + p[1] ** 2)
    assert np.all(nrm <= 1 + 1e-12)
    inside = np.sqrt(q[0] ** 2 + q[1] ** 2) <= 1
    assert np.allclose(p[:, inside], q[:, inside])
    # spectral clip of diag(3, -0.5) and of a rotated diag(2, -2)
    h = np.zeros((3, 1, 2))
    h[:, 0, 0] = (3.0, -0.5, 0.0)
    c, s_ = np.cos(0.3), np.sin(0.3)
    R = np.array([[c, -s_], [s_, c]])
    M = R @ np.diag([2.0, -2.0]) @ R.T
    h[:, 0, 1] = (M[0, 0], M[1, 1], M[0, 1])
    out = px.project_dual_ball(h, "hs1")
    assert np.allclose(out[:, 0, 0], (1.0, -0.5, 0.0))
    Mc = R @ np.diag([1.0, -1.0]) @ R.T
    assert np.allclose(out[:, 0, 1], (Mc[0, 0], Mc[1, 1], Mc[0, 1]))
    assert px.reg_value(np.zeros((4, 4)), "hs1") == 0.0


def _hessian_groups(x):
    """The symmetric 2 x 2 Hessian of every pixel as full matrices."""
    from oracle import operators as ops
    v = ops.hessian(x)
    M = np.empty(v.shape[1:] + (2, 2))
    M[..., 0, 0], M[..., 1, 1] = v[0], v[1]
    M[..., 0, 1] = M[..., 1, 0] = v[2]
    return M


def test_hessian_schatten_values_are_the_matrix_norms():
    # HS_phi of the appendix example: the Schatten-phi norm of every group,
    # checked against numpy's nuclear, Frobenius and spectral matrix norms
    x = W.gaussian((9, 7), 12)
    M = _hessian_groups(x)
    for reg, ordn in (("hs1", "nuc"), ("hs2", "fro"), ("hsinf", 2)):
        ref = sum(np.linalg.norm(M[i, j], ordn) for i in range(M.shape[0]) for j in range(M.shape[1]))
        assert abs(px.reg_value(x, reg) - ref) <= 1e-12 * (1 + ref)


@pytest.mark.parametrize("reg,ordn", [("hs2", "fro"), ("hsinf", "nuc")])
def test_schatten_dual_ball_projection_is_the_nearest_point(reg, ordn):
    # the dual ball of HS_2 is the Schatten-2 ball, of HS_inf the Schatten-1
    # ball (1/phi + 1/psi = 1); the projection of a group in the Frobenius
    # metric, found by a general constrained minimiser over symmetric 2 x 2
    # matrices
    from scipy.optimize import minimize
    rng = np.random.default_rng(7)
    q = rng.standard_normal((3, 1, 8)) * 1.5
    out = px.project_dual_ball(q, reg)
    for k in range(q.shape[-1]):
        M = np.array([[q[0, 0, k], q[2, 0, k]], [q[2, 0, k], q[1, 0, k]]])
        inside = np.linalg.norm(M, ordn) <= 1
        def obj(z):
            X = np.array([[z[0], z[2]], [z[2], z[1]]])
            return float(np.sum((X - M) ** 2))
        cons = {"type": "ineq",
                "fun": lambda z: 1.0 - np.linalg.norm(np.array([[z[0], z[2]], [z[2], z[1]]]), ordn)}
        best = None
        for z0 in (np.zeros(3), 0.3 * np.array([M[0, 0], M[1, 1], M[0, 1]])):
            r = minimize(obj, z0, constraints=[cons], method="SLSQP",
                         options={"ftol": 1e-14, "maxiter": 500})
            if best is None or r.fun < best.fun:
                best = r
        got = out[:, 0, k]
        if inside:
            assert np.allclose(got, q[:, 0, k], atol=1e-12)
        else:
            # on the unit sphere, and no feasible point the minimiser found
            # is nearer (the nuclear norm's kinks slow the minimiser down, so
            # compare distances rather than points)
            Xg = np.array([[got[0], got[2]], [got[2], got[1]]])
            assert abs(np.linalg.norm(Xg, ordn) - 1.0) < 1e-12
            assert obj(got) <= best.fun * (1 + 1e-7) + 1e-12, (reg, k, obj(got), best.fun)
            if reg == "hs2":
                assert np.allclose(got, best.x, atol=1e-6)


# --- constraint sets C != R^N (a box) ---------------------------------------

def test_box_projection_in_the_p_metric_matches_a_bound_constrained_qp():
    # prox^P_{delta_C}(z) = argmin_{lo <= x <= hi} 1/2 (x - z)^T P (x - z),
    # by Thm. 1's Newton iteration, against L-BFGS-B on the same QP
    from scipy.optimize import minimize
    N, K = 40, 5
    rng = np.random.default_rng(21)
    U = np.linalg.qr(rng.standard_normal((N, K)))[0].T
    for e in (np.array([3.0, 1.5, 0.8, -0.4, -0.7]), np.linspace(5.0, 0.1, K)):
        P = np.eye(N) + U.T @ (e[:, None] * U)
        for lo, hi, sc in ((0.0, np.inf, 1.0), (-0.3, 0.5, 1.0), (-1.0, 1.0, 3.0)):
            z = rng.standard_normal(N) * sc
            x, gamma, _ = px.prox_box_weighted(z, lo, hi, U, e)
            r = minimize(lambda v: 0.5 * (v - z) @ P @ (v - z), np.clip(z, lo, hi),
                         jac=lambda v: P @ (v - z), method="L-BFGS-B",
                         bounds=[(lo, None if np.isinf(hi) else hi)] * N,
                         options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 20000})
            assert np.all(x >= lo - 1e-15) and np.all(x <= hi + 1e-15)
            assert np.allclose(x, r.x, atol=1e-6), (lo, hi, np.abs(x - r.x).max())


def test_box_projection_with_identity_metric_is_the_clip():
    z = W.gaussian((50,), 31) * 2
    x, _, _ = px.prox_box_weighted(z, -0.5, 0.25, np.zeros((0, 50)), np.zeros(0))
    assert np.array_equal(x, np.clip(z, -0.5, 0.25))


def test_constrained_dual_prox_matches_smoothed_primal_and_its_gap_vanishes():
    # argmin_{x >= 0} 1/2||x - s||_P^2 + lam_bar TV(x) on a 6 x 6 image: the
    # dual iteration with x(Q) = prox^P_{delta_C}(.) against L-BFGS-B with the
    # bound on the primal with TV smoothed by eps (error O(eps))
    from scipy.optimize import minimize
    from oracle import operators as ops
    n, lam_bar, lo, eps = 6, 0.15, 0.0, 1e-7
    s = W.gaussian((n, n), 41)
    pc = _small_precond(n * n, 4, 2)
    proj = lambda z: px.prox_box_weighted(z.reshape(-1), lo, np.inf, pc.U, pc.e)[0].reshape(z.shape)
    x, Q = px.prox_mixed_dual(s, lam_bar, "tv", pc.pinv, pc.pinv_norm, 4000, proj_c=proj)
    assert np.all(x >= lo - 1e-12)
    gap = px.constrained_gap(x, Q, lam_bar, "tv")
    assert -1e-10 <= gap < 1e-6

    def obj(v):
        xx = v.reshape(n, n)
        d = xx - s
        g = ops.grad(xx)
        t = np.sqrt(g[0] ** 2 + g[1] ** 2 + eps * eps)
        val = 0.5 * np.sum(d * pc.p(d)) + lam_bar * np.sum(t)
        grad = pc.p(d) + lam_bar * ops.grad_adjoint(g / t[None])
        return val, grad.reshape(-1)
    r = minimize(obj, np.maximum(s, 0).reshape(-1), jac=True, method="L-BFGS-B",
                 bounds=[(lo, None)] * (n * n),
                 options={"ftol": 1e-16, "gtol": 1e-11, "maxiter": 50000, "maxcor": 50})
    assert np.allclose(x.reshape(-1), r.x, atol=2e-4), np.abs(x.reshape(-1) - r.x).max()


def test_constrained_dual_prox_tiny_lambda_is_the_weighted_projection():
    n = 7
    s = W.gaussian((n, n), 43)
    pc = _small_precond(n * n, 4, 3)
    proj = lambda z: px.prox_box_weighted(z.reshape(-1), 0.0, np.inf, pc.U, pc.e)[0].reshape(z.shape)
    x, _ = px.prox_mixed_dual(s, 1e-12, "tv", pc.pinv, pc.pinv_norm, 5, proj_c=proj)
    assert np.allclose(x, proj(s), atol=1e-10)
    assert not np.allclose(proj(s), np.clip(s, 0, None))   # the metric matters


# --- l1 prox with the diagonal-plus-low-rank metric (Thm. 1) ---------------

def _prox_l1_brute(s, lam_bar, P, iters=20000):
    """Proximal gradient on 1/2||x-s||_P^2 + lam_bar||x||_1, step 1/||P||."""
    Lp = np.linalg.eigvalsh(P).max()
    x = s.copy()
    for _ in range(iters):
        x = px.soft(x - (P @ (x - s)) / Lp, lam_bar / Lp)
    return x


@pytest.mark.parametrize("tail", ["sqrt", "plain"])
def test_l1_prox_matches_brute_force_and_subgradient(tail):
    N, K = 40, 4
    pc = _small_precond(N, K, 7, tail)
    s = W.gaussian((N,), 8)
    lam_bar = 0.4
    x, gamma, steps = px.prox_l1_weighted(s, lam_bar, pc.U, pc.e)
    P = np.stack([pc.p(e) for e in np.eye(N)])
    assert np.allclose(x, _prox_l1_brute(s, lam_bar, P), atol=1e-8)
    # optimality: r = -P(x - s)/lam_bar is a subgradient of ||.||_1 at x
    r = -(P @ (x - s)) / lam_bar
    nz = x != 0
    assert np.allclose(r[nz], np.sign(x[nz]), atol=1e-9)
    assert np.all(np.abs(r[~nz]) <= 1 + 1e-9)
    assert steps < 50


def test_l1_prox_reduces_to_soft_threshold_and_scalar_root():
    N = 30
    s = W.gaussian((N,), 9)
    U = np.linalg.qr(W.gaussian((N, 3), 10))[0].T
    x, _, _ = px.prox_l1_weighted(s, 0.5, U, np.zeros(3))
    assert np.allclose(x, px.soft(s, 0.5))
    x0, _, _ = px.prox_l1_weighted(s, 0.5, np.zeros((0, N)), np.zeros(0))
    assert np.allclose(x0, px.soft(s, 0.5))
    # K = 1: gamma solves a scalar monotone equation; bisection brute force
    u = U[:1]
    e = np.array([2.5])
    Fs = lambda g: g - e[0] * (u[0] @ (px.soft(s - g * u[0], 0.5) - s))
    lo, hi = -100.0, 100.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if Fs(mid) > 0:
            hi = mid
        else:
            lo = mid
    _, g, _ = px.prox_l1_weighted(s, 0.5, u, e)
    assert abs(g[0] - 0.5 * (lo + hi)) < 1e-10


# --- Huber data term -------------------------------------------------------

def test_huber_value_and_gradient_by_finite_differences():
    n = 8
    h = W.gaussian_psf(3, 0.8)
    y = W.gaussian((n // 2, n // 2), 11) * 0.05
    p = sv.Problem("blurdown", n, y, 0.0, "l1", h=h, factor=2, levels=3,
                   loss="huber", delta=0.02)
    x = W.gaussian((n, n), 12) * 0.05
    g = p.grad_f(x)
    d = W.gaussian((n, n), 13)
    eps = 1e-6
    fd = (p.f(x + eps * d) - p.f(x - eps * d)) / (2 * eps)
    assert abs(fd - np.sum(g * d)) < 1e-6 * (1 + abs(fd))
    r = np.array([0.01, -0.05])
    p2 = sv.Problem("identity", 1, np.zeros(2), 0.0, "l1", loss="huber", delta=0.02)
    assert abs(p2.f(r) - (0.01 ** 2 / 0.04 + 0.05 - 0.01)) < 1e-15


# --- WAPG ------------------------------------------------------------------

def _tiny_wavelet_deblur():
    n = 16
    h = W.gaussian_psf(9, 1.5)
    prob = sv.Problem("blur", n, None, 2e-3, "l1", h=h, levels=3)
    xt = W.phantom_blocks(n, 0)
    prob.y = prob.A(ops.haar_analysis(xt, 3)) + 0.01 * W.gaussian((n, n), 0)
    return prob


def test_wapg_rate_bound_and_same_optimum_with_and_without_precond():
    prob = _tiny_wavelet_deblur()
    n = prob.n
    L = sv.lipschitz(prob, None, W.gaussian((n, n), 14), 300)
    assert abs(L - 1.0) < 1e-6          # normalised PSF: lambda_max(A^T A) = 1
    x, costs = sv.wapg(prob, None, 1.0 / (1.01 * L), 1200)
    Om = W.omega(24, n, n, 15)
    pc, _ = sv.build_precond(prob, Om, tail="plain")
    Lp = sv.lipschitz(prob, pc, W.gaussian((n, n), 14), 300)
    assert Lp < 0.5 * L                 # steep spectrum at this size
    xp, costs_p = sv.wapg(prob, pc, 1.0 / (1.01 * Lp), 1200)
    Fstar = min(costs.min(), costs_p.min())
    assert abs(costs[-1] - costs_p[-1]) < 1e-7 * Fstar
    # O(1/k^2) bound with x^1 = 0: F(x^k) - F* <= 2 L ||x^1 - x*||_P^2 / (k+1)^2
    k = np.arange(1, len(costs) + 1)
    bound = 2 * (1.01 * L) * np.sum(x * x) / (k + 1) ** 2
    assert np.all(costs - Fstar <= bound * (1 + 1e-6) + 1e-12)
    bound_p = 2 * (1.01 * Lp) * np.sum(xp * pc.p(xp)) / (k + 1) ** 2
    assert np.all(costs_p - Fstar <= bound_p * (1 + 1e-6) + 1e-12)
    # the preconditioned method gets within 1e-6 of F* in fewer iterations
    kp = np.argmax(costs_p - Fstar <= 1e-6 * Fstar)
    k0 = np.argmax(costs - Fstar <= 1e-6 * Fstar)
    assert kp < k0


def test_wapg_with_nonnegativity_reaches_the_same_feasible_optimum_with_and_without_precond():
    # C = {x >= 0}: every iterate is feasible, and the plain and the
    # preconditioned method (P-weighted projection inside the dual iteration)
    # approach the same constrained optimum
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=5, n=16)
    prob.box = (0.0, np.inf)
    n = prob.n
    L = sv.lipschitz(prob, None, W.gaussian((n, n), 14), 200)
    x, costs = sv.wapg(prob, None, 1.0 / (1.01 * L), 400, inner=30)
    pc, _ = sv.build_precond(prob, W.omega(12, n, n, 16), tail="plain")
    Lp = sv.lipschitz(prob, pc, W.gaussian((n, n), 14), 200)
    xp, costs_p = sv.wapg(prob, pc, 1.0 / (1.01 * Lp), 400, inner=30)
    assert x.min() >= 0.0 and xp.min() >= 0.0
    assert abs(costs[-1] - costs_p[-1]) < 1e-5 * costs[-1]
    assert np.allclose(x, xp, atol=1e-2 * np.abs(x).max())   # TV optima are flat in places
    # the unconstrained optimum violates the bound here, so C is active
    xu, _ = sv.wapg(sv.problem_from_workload(wl, seed=5, n=16)[0], None, 1.0 / (1.01 * L), 400, inner=30)
    assert xu.min() < -1e-3


def test_wapg_tv_decreases_cost():
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=1, n=24)
    L = sv.lipschitz(prob, None, W.gaussian((24, 24), 16), 200)
    _, costs = sv.wapg(prob, None, 1 / (1.01 * L), 60, inner=20)
    assert costs[-1] < costs[0] and costs[-1] <= costs.min() * (1 + 1e-3)


def test_wapg_first_iterates_follow_alg3_by_hand():
    # x^1 = u^1 = 0, t^0 = 1:  x^2 = soft(alpha A^T y);  u^2 = x^2 (t^0 = 1);
    # x^3 = soft(x^2 - alpha grad f(x^2));  u^3 = x^3 + (t^1 - 1)/t^2 (x^3 - x^2)
    # with t^1 = (1 + sqrt 5)/2 and t^2 = (1 + sqrt(1 + 4 t1^2))/2;
    # x^4 = soft(u^3 - alpha grad f(u^3)).
    prob = _tiny_wavelet_deblur()
    alpha, lam = 0.9, prob.lam
    soft = lambda z: np.sign(z) * np.maximum(np.abs(z) - alpha * lam, 0)
    x2 = soft(alpha * prob.At(prob.y))
    x3 = soft(x2 - alpha * prob.grad_f(x2))
    t1 = (1 + 5 ** 0.5) / 2
    t2 = (1 + (1 + 4 * t1 * t1) ** 0.5) / 2
    u3 = x3 + (t1 - 1) / t2 * (x3 - x2)
    x4 = soft(u3 - alpha * prob.grad_f(u3))
    for k, ref in ((1, x2), (2, x3), (3, x4)):
        xk, _ = sv.wapg(prob, None, alpha, k, record_cost=False)
        assert np.allclose(xk, ref, atol=1e-15)


def test_workload_inputs_are_seeded_and_shaped():
    a = W.phantom_blocks(64, 3)
    b = W.phantom_blocks(64, 3)
    assert np.array_equal(a, b) and a.min() >= 0 and a.max() <= 1
    ct = W.phantom_ellipses(64, 3)
    assert ct.max() <= 0.04 + 1e-15 and ct.min() >= 0
    salt, pepper = W.salt_pepper_masks((32, 32), 0)
    assert salt.sum() == pepper.sum() == round(0.05 * 1024) and not np.any(salt & pepper)
    h = W.gaussian_psf(7, 1.2)
    assert abs(h.sum() - 1) < 1e-15 and np.allclose(h, h.T) and np.allclose(h, h[::-1, ::-1])
    r = W.round_bf16(np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 3.14159]))
    assert np.array_equal(r, [1.0, 1.0, 1 + 2 ** -6, 3.140625])
