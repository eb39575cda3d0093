"""FP64 oracle of the alternating minimisation method (Alg. 2) for the
l_p - l_q problem, with its x-update solved by CG or by PCG preconditioned
with the Nystrom preconditioner of Phi_k rebuilt at every outer iteration.

Test infrastructure only.

Problem (Sec. III-A, component-wise form):
    min_x 1/p sum_m |(A x - y)_m|^p + lambda/q sum_l |(L x)_l|^q
with L the first differences of the TV regulariser, every component its own
group (the anisotropic l_1 norm for q = 1).  The half-quadratic identity
|r|^p = min_{beta > 0} beta r^2 + 1 / (b_p beta^{a_p}) with minimiser
beta* = p/2 |r|^{p-2} gives the weights of the x-update:
    W_f = diag(|A x - y|^{p-2}),  W_g = diag(|L x|^{q-2})
(element-wise, with |r| replaced by |r|_eps = sqrt(r^2 + eps) everywhere, the
paper's rule for r = 0 applied to every entry), and the x-update is the
linear system Phi_k x = A^T W_f y with Phi_k = A^T W_f A + lambda L^T W_g L.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

from . import nystrom as nys
from . import operators as ops


def half_quadratic_constants(p: float):
    """a_p = p / (2 - p) and b_p of the half-quadratic identity (0 < p < 2)."""
    a = p / (2.0 - p)
    b = 2.0 ** (2.0 / (2.0 - p)) / ((2.0 - p) * p ** (p / (2.0 - p)))
    return a, b


def weights(r: np.ndarray, p: float, eps: float) -> np.ndarray:
    """(2/p) beta* = |r|_eps^(p-2), element-wise."""
    return (r * r + eps) ** ((p - 2.0) / 2.0)


def lp_objective(x, A, y, lam, p, q, eps):
    """The smoothed objective 1/p sum |r|_eps^p + lambda/q sum |Lx|_eps^q."""
    r = A(x) - y
    g = ops.grad(x)
    return (float(np.sum((r * r + eps) ** (p / 2.0))) / p +
            lam * float(np.sum((g * g + eps) ** (q / 2.0))) / q)


def pcg(apply_phi: Callable, b: np.ndarray, x0: np.ndarray, tol: float, maxit: int,
        pinv: Optional[Callable] = None):
    """Preconditioned conjugate gradients on Phi x = b from x0; stops when
    ||b - Phi x|| <= tol ||b|| (checked after each update) or after maxit
    iterations.  Returns (x, iterations)."""
    x = np.array(x0, np.float64, copy=True)
    r = b - apply_phi(x)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return np.zeros_like(b), 0
    if float(np.linalg.norm(r)) <= tol * nb:
        return x, 0
    z = pinv(r) if pinv else r.copy()
    d = z.copy()
    rz = float(np.vdot(r, z))
    it = 0
    while it < maxit:
        q = apply_phi(d)
        alpha = rz / float(np.vdot(d, q))
        x = x + alpha * d
        r = r - alpha * q
        it += 1
        if float(np.linalg.norm(r)) <= tol * nb:
            break
        z = pinv(r) if pinv else r.copy()
        rz_new = float(np.vdot(r, z))
        d = z + (rz_new / rz) * d
        rz = rz_new
    return x, it


@dataclasses.dataclass
class IrmResult:
    x: np.ndarray
    outer: int
    cg_iters: list
    shat: list


def irm(A, At, y, lam, p, q, eps, x0, max_outer, outer_tol, cg_tol, cg_maxit,
        omega: Optional[np.ndarray] = None, tail: str = "plain", mu=None):
    """Alg. 2.  With `omega` (ell x n1 x n2) the x-update is PCG with the
    Nystrom preconditioner of Phi_k (Alg. 1 on Y = Phi_k Omega, eq. (11)),
    rebuilt at every outer iteration; without it, plain CG.  Every x-update
    starts from the previous iterate."""
    x = np.array(x0, np.float64, copy=True)
    shp = x.shape
    its, shats = [], []
    k = 0
    for k in range(1, max_outer + 1):
        wf = weights(A(x) - y, p, eps)
        wg = weights(ops.grad(x), q, eps)

        def phi(v, wf=wf, wg=wg):
            v = v.reshape(shp)
            return (At(wf * A(v)) + lam * ops.grad_adjoint(wg * ops.grad(v))).reshape(-1)

        b = At(wf * y).reshape(-1)
        pinv = None
        if omega is not None:
            ell = omega.shape[0]
            Y = np.stack([phi(omega[j]) for j in range(ell)])
            r = nys.nystrom(Y, omega.reshape(ell, -1))
            m = r["nu"] if mu is None else mu
            U, sh = r["U"], r["shat"]
            shats.append(sh)
            pinv = lambda v, U=U, sh=sh, m=m: nys.pinv_apply(v, U, sh, m, tail)
        xn, it = pcg(phi, b, x.reshape(-1), cg_tol, cg_maxit, pinv)
        its.append(it)
        xn = xn.reshape(shp)
        done = np.linalg.norm(xn - x) <= outer_tol * np.linalg.norm(xn)
        x = xn
        if done:
            break
    return IrmResult(x, k, its, shats)
