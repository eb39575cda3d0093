"""FP64 oracle: weighted proximal maps (Sec. I-D definition, Thm. 1, Sec. III-B).

Test infrastructure only.

- `prox_mixed_dual`: the P-weighted prox of lambda_bar ||L x||_{1,phi} with
  C = R^N, solved through its dual (eqs. (21)-(29)): accelerated projected
  gradient on the dual variable Q, x(Q) = s - lambda_bar P^{-1} L^T Q, dual
  gradient -2 lambda_bar L x(Q), step 1 / (2 lambda_bar^2 ||L||^2 ||P^{-1}||)
  (reading of the garbled Lipschitz constant: 2 lambda_bar^2 ||L P^{-1} L^T||
  <= 2 lambda_bar^2 ||L||^2 / sigma_min(P)).
- `prox_l1_weighted`: the P-weighted prox of lambda_bar ||.||_1 for
  P = I + U diag(e) U^T through Thm. 1: gamma solves
  F(gamma) = gamma - diag(e) U^T (soft(s - U gamma) - s) = 0, found by a
  semismooth Newton method with backtracking on ||F||.
"""
from __future__ import annotations

import numpy as np

from . import operators as ops


# --------------------------------------------------------------------------
# regulariser pieces

# Hessian Schatten-phi priors (the paper's HS_phi, phi = 1, 2, inf): the
# groups are the symmetric 2 x 2 Hessians of the appendix example
HESSIAN_REGS = ("hs1", "hs2", "hsinf")


def reg_L(x, reg):
    return ops.hessian(x) if reg in HESSIAN_REGS else ops.grad(x)


def reg_Lt(q, reg):
    return ops.hessian_adjoint(q) if reg in HESSIAN_REGS else ops.grad_adjoint(q)


def sym2_eig(v):
    """Eigen-decomposition of the symmetric 2 x 2 groups (v11, v22, v12)."""
    m = np.empty(v.shape[:-3] + v.shape[-2:] + (2, 2))
    m[..., 0, 0] = v[..., 0, :, :]
    m[..., 1, 1] = v[..., 1, :, :]
    m[..., 0, 1] = m[..., 1, 0] = v[..., 2, :, :]
    return np.linalg.eigh(m)


def reg_value(x, reg):
    """||L x||_{1,phi} for 'tv' (phi=2), 'tv_aniso' (phi=1), 'hs1', 'hs2',
    'hsinf' (Schatten-1, -2, -inf norm of each Hessian group: the l1, l2,
    l_inf norm of its eigenvalues), 'l1' (plain l1 of x itself)."""
    if reg == "l1":
        return float(np.sum(np.abs(x)))
    v = reg_L(x, reg)
    if reg == "tv":
        return float(np.sum(np.sqrt(v[..., 0, :, :] ** 2 + v[..., 1, :, :] ** 2)))
    if reg == "tv_aniso":
        return float(np.sum(np.abs(v)))
    if reg in HESSIAN_REGS:
        w, _ = sym2_eig(v)
        if reg == "hs1":
            return float(np.sum(np.abs(w)))
        if reg == "hs2":
            return float(np.sum(np.sqrt(np.sum(w * w, axis=-1))))
        return float(np.sum(np.max(np.abs(w), axis=-1)))
    raise ValueError(reg)


def project_l1_ball(w):
    """Euclidean projection of every row of w onto the unit l1 ball: the
    sort-and-threshold rule (soft threshold at the theta that makes the
    magnitudes sum to 1, for rows outside the ball)."""
    w = np.asarray(w, dtype=np.float64)
    a = np.abs(w)
    out = w.copy()
    outside = a.sum(axis=-1) > 1.0
    if not np.any(outside):
        return out
    u = -np.sort(-a[outside], axis=-1)          # descending magnitudes
    css = np.cumsum(u, axis=-1)
    j = np.arange(1, u.shape[-1] + 1)
    cond = u - (css - 1.0) / j > 0
    rho = cond.shape[-1] - 1 - np.argmax(cond[..., ::-1], axis=-1)   # last index where cond holds
    theta = (css[np.arange(len(rho)), rho] - 1.0) / (rho + 1)
    out[outside] = np.sign(w[outside]) * np.maximum(a[outside] - theta[:, None], 0.0)
    return out


def project_dual_ball(q, reg):
    """Projection onto B_{inf,psi} (eq. (23)), 1/phi + 1/psi = 1.

    'tv'      : each (q1, q2) onto the unit l2 ball
    'tv_aniso': each entry clipped to [-1, 1]
    'hs1'     : each symmetric 2 x 2 group onto the unit spectral-norm ball,
                i.e. its eigenvalues clipped to [-1, 1]
    'hs2'     : onto the unit Frobenius (Schatten-2) ball: the eigenvalues
                onto the unit l2 ball
    'hsinf'   : onto the unit nuclear-norm (Schatten-1) ball: the eigenvalues
                onto the unit l1 ball
    (the Frobenius metric of the groups counts v12 = v21 twice, so
    projecting the eigenvalues is the projection of the group)
    """
    if reg == "tv":
        nrm = np.sqrt(q[..., 0, :, :] ** 2 + q[..., 1, :, :] ** 2)
        return q / np.maximum(1.0, nrm)[..., None, :, :]
    if reg == "tv_aniso":
        return np.clip(q, -1.0, 1.0)
    if reg in HESSIAN_REGS:
        w, V = sym2_eig(q)
        if reg == "hs1":
            w = np.clip(w, -1.0, 1.0)
        elif reg == "hs2":
            w = w / np.maximum(1.0, np.sqrt(np.sum(w * w, axis=-1)))[..., None]
        else:
            w = project_l1_ball(w.reshape(-1, 2)).reshape(w.shape)
        m = np.einsum("...ik,...k,...jk->...ij", V, w, V)
        out = np.empty_like(q)
        out[..., 0, :, :] = m[..., 0, 0]
        out[..., 1, :, :] = m[..., 1, 1]
        out[..., 2, :, :] = m[..., 0, 1]
        return out
    raise ValueError(reg)


L_NORM2_BOUND = {"tv": 8.0, "tv_aniso": 8.0, "hs1": 34.0, "hs2": 34.0, "hsinf": 34.0}


def prox_mixed_dual(s, lam_bar, reg, pinv, pinv_norm, n_inner, q0=None,
                    lnorm2=None, proj_c=None):
    """argmin_{x in C} 1/2 ||x - s||_P^2 + lam_bar ||L x||_{1,phi}.

    pinv: callable v -> P^{-1} v (identity for the plain method).
    proj_c: None for C = R^N, else the P-weighted projection onto C
    (prox^P_{delta_C}, a callable z -> x): then x(Q) = proj_c(s - lam_bar
    P^{-1} L^T Q) (eq. (26)), the dual gradient -2 lam_bar L x(Q) (eq. (28)) and the same
    step (prox^P_{delta_C} is nonexpansive in the P-norm, so the Lipschitz
    bound of the unconstrained case holds).
    Returns (x, Q).  The returned x is built from the last projected Q, not
    from the extrapolated point (eq. (29)).
    """
    xq = (lambda z: z) if proj_c is None else proj_c
    if lnorm2 is None:
        lnorm2 = L_NORM2_BOUND[reg]
    if q0 is None:
        q0 = np.zeros_like(reg_L(s, reg))
    step = 1.0 / (lam_bar * lnorm2 * pinv_norm)
    Q = np.array(q0, dtype=np.float64, copy=True)
    R = Q.copy()
    tau = 1.0
    for _ in range(n_inner):
        x = xq(s - lam_bar * pinv(reg_Lt(R, reg)))
        Qn = project_dual_ball(R + step * reg_L(x, reg), reg)
        tau_n = (1.0 + np.sqrt(1.0 + 4.0 * tau * tau)) / 2.0
        R = Qn + ((tau - 1.0) / tau_n) * (Qn - Q)
        Q, tau = Qn, tau_n
    x = xq(s - lam_bar * pinv(reg_Lt(Q, reg)))
    return x, Q


def dual_gap(s, x_of_q, Q, lam_bar, reg, p_apply, pinv):
    """Primal minus dual value of the WPM at Q (both written out directly):
    primal 1/2||x - s||_P^2 + lam_bar ||L x||,  dual
    lam_bar <L^T Q, s> - lam_bar^2/2 <L^T Q, P^{-1} L^T Q>."""
    d = x_of_q - s
    primal = 0.5 * float(np.sum(d * p_apply(d))) + lam_bar * reg_value(x_of_q, reg)
    t = reg_Lt(Q, reg)
    dual = lam_bar * float(np.sum(t * s)) - 0.5 * lam_bar ** 2 * float(np.sum(t * pinv(t)))
    return primal - dual


# --------------------------------------------------------------------------
# l1 prox with a diagonal-plus-low-rank metric (Thm. 1)

def soft(z, t):
    """prox of t ||.||_1: sign(z) max(|z| - t, 0)."""
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


def constrained_gap(x_of_q, Q, lam_bar, reg):
    """Primal minus dual value of the constrained WPM at Q, with x(Q) the
    minimiser of the Lagrangian over C (eq. (26)): lam_bar (||L x||_{1,phi}
    - <Q, L x>), nonnegative for Q in the dual ball."""
    return lam_bar * (reg_value(x_of_q, reg) - ops.pair(Q, reg_L(x_of_q, reg), reg))


def prox_box_weighted(z, lo, hi, U, e, gamma0=None, tol=1e-12, maxit=100,
                      max_halvings=30):
    """prox^P_{delta_C}(z) for the box C = {lo <= x <= hi}, P = I + U^T
    diag(e) U: Thm. 1 with h = delta_C, whose unweighted prox is the clip:
    gamma solves F(gamma) = gamma - diag(e) U (clip(z - U^T gamma) - z) = 0,
    semismooth Newton with the Jacobian I + diag(e) U D U^T, D the pixels
    strictly inside the box, and backtracking on ||F||.
    Returns (x, gamma, newton_steps)."""
    K = U.shape[0]
    gamma = np.zeros(K) if gamma0 is None else np.array(gamma0, np.float64)
    if K == 0:
        return np.clip(z, lo, hi), gamma, 0

    def F(g):
        r = z - g @ U
        return g - e * (U @ (np.clip(r, lo, hi) - z)), r

    Fg, r = F(gamma)
    steps = 0
    for steps in range(maxit):
        nF = np.linalg.norm(Fg)
        if nF <= tol * (1.0 + np.linalg.norm(gamma)):
            break
        active = (r > lo) & (r < hi)
        Ua = U[:, active]
        J = np.eye(K) + e[:, None] * (Ua @ Ua.T)
        delta = np.linalg.solve(J, -Fg)
        t = 1.0
        for _ in range(max_halvings):
            g_try = gamma + t * delta
            F_try, r_try = F(g_try)
            if np.linalg.norm(F_try) <= (1.0 - 1e-4 * t) * nF:
                break
            t *= 0.5
        gamma, Fg, r = g_try, F_try, r_try
    return np.clip(z - gamma @ U, lo, hi), gamma, steps


def prox_l1_weighted(s, lam_bar, U, e, gamma0=None, tol=1e-12, maxit=100,
                     max_halvings=30):
    """argmin_x lam_bar ||x||_1 + 1/2 ||x - s||_P^2, P = I + U^T diag(e) U.

    s: (N,), U: (K, N) orthonormal rows, e: (K,) with 1 + e > 0.
    Returns (x, gamma, newton_steps).
    """
    K = U.shape[0]
    gamma = np.zeros(K) if gamma0 is None else np.array(gamma0, np.float64)
    if K == 0:
        return soft(s, lam_bar), gamma, 0

    def F(g):
        r = s - g @ U
        return g - e * (U @ (soft(r, lam_bar) - s)), r

    Fg, r = F(gamma)
    steps = 0
    for steps in range(maxit):
        nF = np.linalg.norm(Fg)
        if nF <= tol * (1.0 + np.linalg.norm(gamma)):
            break
        active = np.abs(r) > lam_bar
        Ua = U[:, active]
        J = np.eye(K) + e[:, None] * (Ua @ Ua.T)
        delta = np.linalg.solve(J, -Fg)
        t = 1.0
        for _ in range(max_halvings):
            g_try = gamma + t * delta
            F_try, r_try = F(g_try)
            if np.linalg.norm(F_try) <= (1.0 - 1e-4 * t) * nF:
                break
            t *= 0.5
        gamma, Fg, r = g_try, F_try, r_try
    return soft(s - gamma @ U, lam_bar), gamma, steps
