"""FP64 oracle: problem definitions, cost, WAPG (Alg. 3) and the sketch.

Test infrastructure only.

Problem (eq. (4), and eq. (23) for an invertible wavelet L):
    min_x f(x) + lam g(x),  f = 1/2 ||A x - y||^2  or  sum_m h_delta((A x - y)_m)
with the Huber reading h_delta(r) = r^2 / (2 delta) for |r| <= delta and
|r| - delta / 2 otherwise (the super-resolution workload names a Huber data
term; the paper's own super-resolution uses l_p data terms).  For the wavelet
regulariser the unknown is xbar = W x, the operator is A W^T and
g = ||xbar||_1 (all coefficients, as in eq. (30)).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import nystrom as nys
from . import operators as ops
from . import prox as px


@dataclasses.dataclass
class Problem:
    op: str                      # 'blur' | 'blurdown' | 'ct' | 'fan' | 'identity'
    n: int
    y: np.ndarray
    lam: float
    reg: str                     # 'tv' | 'tv_aniso' | 'hs1' | 'l1'
    h: Optional[np.ndarray] = None
    factor: int = 1
    views: int = 0
    bins: int = 0
    levels: int = 0              # wavelet levels of the reparametrisation
    wavelet: str = "haar"        # 'haar' | 'db4' (periodised Daubechies-4)
    loss: str = "ls"
    delta: float = 0.0
    box: Optional[tuple] = None  # (lo, hi): x restricted to C = {lo <= x <= hi}
    fan: tuple = (0.0, 0.0, 1.0)  # 'fan': source radius, detector radius, bin spacing

    # A and A^T of the (possibly reparametrised) problem
    def A(self, x):
        if self.levels:
            x = ops.wavelet_synthesis(x, self.levels, self.wavelet)
        if self.op == "blur":
            return ops.blur(x, self.h)
        if self.op == "blurdown":
            return ops.blurdown(x, self.h, self.factor)
        if self.op == "ct":
            return ops.joseph(x, self.views, self.bins)
        if self.op == "fan":
            return ops.fan_joseph(x, self.views, self.bins, *self.fan)
        if self.op == "identity":
            return np.array(x, dtype=np.float64)
        raise ValueError(self.op)

    def At(self, r):
        if self.op == "blur":
            z = ops.blur_adjoint(r, self.h)
        elif self.op == "blurdown":
            z = ops.blurdown_adjoint(r, self.h, self.factor)
        elif self.op == "ct":
            z = ops.joseph_adjoint(r, self.n)
        elif self.op == "fan":
            z = ops.fan_joseph_adjoint(r, self.n, *self.fan)
        elif self.op == "identity":
            z = np.array(r, dtype=np.float64)
        else:
            raise ValueError(self.op)
        if self.levels:
            z = ops.wavelet_analysis(z, self.levels, self.wavelet)
        return z

    # data term
    def f(self, x) -> float:
        r = self.A(x) - self.y
        if self.loss == "huber":
            d = self.delta
            a = np.abs(r)
            return float(np.sum(np.where(a <= d, r * r / (2 * d), a - d / 2)))
        return 0.5 * float(np.sum(r * r))

    def grad_f(self, x):
        r = self.A(x) - self.y
        if self.loss == "huber":
            r = np.clip(r / self.delta, -1.0, 1.0)
        return self.At(r)

    def curvature(self) -> float:
        """Upper bound of f'' per unit of A^T A: 1 (LS) or 1/delta (Huber)."""
        return 1.0 / self.delta if self.loss == "huber" else 1.0

    def cost(self, x) -> float:
        return self.f(x) + self.lam * px.reg_value(x, self.reg)

    def phi(self, v):
        """Phi v = A^T A v (the sketched operator)."""
        return self.At(self.A(v))


def sketch(problem: Problem, Omega: np.ndarray) -> np.ndarray:
    """Alg. 1 step 2: Y = Phi Omega, one column (image) at a time."""
    return np.stack([problem.phi(Omega[k]) for k in range(Omega.shape[0])])


@dataclasses.dataclass
class Precond:
    """P from eq. (11) with s_K <- sqrt(s_K) optionally (Sec. III-B)."""
    U: np.ndarray        # (K, N)
    shat: np.ndarray     # (K,)
    mu: float
    tail: str = "sqrt"

    def pinv(self, v):
        shp = v.shape
        return nys.pinv_apply(v.reshape(-1), self.U, self.shat, self.mu,
                              self.tail).reshape(shp)

    def p(self, v):
        shp = v.shape
        return nys.p_apply(v.reshape(-1), self.U, self.shat, self.mu,
                           self.tail).reshape(shp)

    @property
    def e(self):
        """P = I + U^T diag(e) U."""
        sK = nys.tail_value(self.shat, self.tail)
        return (self.shat + self.mu) / (sK + self.mu) - 1.0

    @property
    def pinv_norm(self):
        return nys.pinv_norm(self.shat, self.mu, self.tail)


def build_precond(problem, Omega, nu_mode="spectral", tail="sqrt", mu=None):
    """Sketch + Alg. 1 + eq. (11).  mu defaults to the shift nu (reading)."""
    Y = sketch(problem, Omega).reshape(Omega.shape[0], -1)
    r = nys.nystrom(Y, Omega.reshape(Omega.shape[0], -1), nu_mode)
    mu = r["nu"] if mu is None else mu
    return Precond(r["U"], r["shat"], mu, tail), r


def lipschitz(problem, pc: Optional[Precond], v0, iters):
    """L_f^P = lambda_max(P^{-1} grad^2 f) bound by the power method (eq. (20))."""
    shp = v0.shape
    if pc is None:
        M = lambda v: problem.phi(v.reshape(shp)).reshape(-1)
    else:
        M = lambda v: pc.pinv(problem.phi(v.reshape(shp))).reshape(-1)
    return problem.curvature() * nys.power_iteration(M, v0.reshape(-1), iters)


def rate_constant(problem, pc: Optional[Precond], x_star, v0, iters, x1=None):
    """L_f^P ||x^1 - x*||_P^2, the constant of the O(1/k^2) bound on WAPG's cost
    gap (twice it over (k + 1)^2, stated after eq. (20), Sec. III-B), whose
    dependence on the sketch size the CT experiments study.  x^1 is the start
    of Alg. 3 (zero unless given); L_f^P by the power method of `lipschitz`;
    P = I without a preconditioner."""
    L = lipschitz(problem, pc, v0, iters)
    d = (np.zeros_like(x_star) if x1 is None else np.asarray(x1, np.float64)) - x_star
    pd = d if pc is None else pc.p(d)
    d2 = float(np.sum(d * pd))
    return dict(L=L, pdist2=d2, value=L * d2)


def wapg(problem: Problem, pc: Optional[Precond], alpha: float, outer: int,
         inner: int = 20, warm_start: bool = True, ssn_tol: float = 1e-12,
         ssn_maxit: int = 100, x0=None, record_cost: bool = True):
    """Alg. 3 with u^1 = x^1 = 0 (reading) and t^0 = 1.

    pc=None is the plain method (P = I), which is APG.
    Returns (x, costs) where costs[k] = F(x after k+1 iterations).
    """
    n = problem.n
    x = np.zeros((n, n)) if x0 is None else np.array(x0, np.float64)
    u = x.copy()
    t_prev = 1.0
    lam_bar = alpha * problem.lam
    Q = None
    gamma = None
    costs = []
    pinv = (lambda v: v) if pc is None else pc.pinv
    pnorm = 1.0 if pc is None else pc.pinv_norm
    for _ in range(outer):
        s = u - alpha * pinv(problem.grad_f(u))
        if problem.reg == "l1":
            if pc is None:
                x_new = px.soft(s, lam_bar)
            else:
                xv, gamma, _ = px.prox_l1_weighted(
                    s.reshape(-1), lam_bar, pc.U, pc.e,
                    gamma if warm_start else None, ssn_tol, ssn_maxit)
                x_new = xv.reshape(n, n)
        else:
            proj_c = None
            if problem.box is not None:
                lo, hi = problem.box
                if pc is None:
                    proj_c = lambda z: np.clip(z, lo, hi)
                else:
                    proj_c = lambda z: px.prox_box_weighted(
                        z.reshape(-1), lo, hi, pc.U, pc.e, None, ssn_tol,
                        ssn_maxit)[0].reshape(z.shape)
            x_new, Q = px.prox_mixed_dual(s, lam_bar, problem.reg, pinv, pnorm,
                                          inner, Q if warm_start else None,
                                          proj_c=proj_c)
        t = (1.0 + np.sqrt(1.0 + 4.0 * t_prev * t_prev)) / 2.0
        u = x_new + ((t_prev - 1.0) / t) * (x_new - x)
        x, t_prev = x_new, t
        if record_cost:
            costs.append(problem.cost(x))
    return x, np.array(costs)


def problem_from_workload(wl, seed: int = 0, n: Optional[int] = None,
                          views: Optional[int] = None, bins: Optional[int] = None):
    """Build the synthetic problem of a workload with the oracle's operator."""
    import workloads as W
    n = wl.n if n is None else n
    if wl.op in ("ct", "fan"):
        views = wl.views if views is None else views
        bins = wl.bins if bins is None else bins
        xt = W.phantom_ellipses(n, seed)
        p = Problem(wl.op, n, None, wl.lam, wl.reg, views=views, bins=bins, fan=wl.fan)
        clean = p.A(xt)
        y = clean + wl.noise_rel_max * np.max(clean) * W.gaussian(clean.shape, seed)
    else:
        xt = W.phantom_blocks(n, seed)
        h = W.gaussian_psf(wl.psf_k, wl.psf_sigma)
        levels = 3 if wl.reg == "l1haar3" else 0
        reg = "l1" if wl.reg == "l1haar3" else wl.reg
        p = Problem(wl.op, n, None, wl.lam, reg, h=h, factor=wl.factor,
                    levels=levels, loss=wl.loss, delta=wl.huber_delta)
        clean = p.A(ops.haar_analysis(xt, levels) if levels else xt)
        y = clean + wl.noise_sigma * W.gaussian(clean.shape, seed)
        if wl.salt_pepper:
            salt, pepper = W.salt_pepper_masks(y.shape, seed, wl.salt_pepper)
            y = np.where(salt, 1.0, np.where(pepper, 0.0, y))
    p.y = y
    return p, xt
