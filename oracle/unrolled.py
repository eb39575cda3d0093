"""FP64 oracle of the unrolled WAPG map x_K(y, lambda) and its gradient.

Test infrastructure only.  The forward is Alg. 3 with the P-weighted TV prox
solved by dual accelerated projected gradient (eqs. (21)-(29)) for fixed
iteration counts, written with torch CPU tensors so that torch's reverse-mode
chain rule supplies the reference gradient.  The linear pieces call the
oracle's own operators (A, A^T from `operators`, P^{-1} from `nystrom`, L and
L^T from `operators`): each enters as a linear map whose vector-Jacobian
product is its (pinned) adjoint.  Nothing here uses the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import operators as ops


class _Linear(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, fwd, adj):
        ctx.adj = adj
        return torch.from_numpy(np.asarray(fwd(x.detach().numpy()), np.float64))

    @staticmethod
    def backward(ctx, g):
        return torch.from_numpy(np.asarray(ctx.adj(g.detach().numpy()), np.float64)), None, None


def _lin(x, fwd, adj):
    return _Linear.apply(x, fwd, adj)


def unrolled(problem, pc, alpha: float, n_outer: int, n_inner: int, y: torch.Tensor,
             lam: torch.Tensor, lnorm2: float = 8.0, aniso: bool = False) -> torch.Tensor:
    """x_K for one instance.  problem: oracle.solver.Problem (its y unused);
    pc: oracle.solver.Precond or None (P = I); y, lam: float64 torch tensors."""
    n = problem.n
    A = lambda v: _lin(v, problem.A, problem.At)
    At = lambda r: _lin(r, problem.At, problem.A)
    if pc is None:
        Pinv = lambda v: v
        pnorm = 1.0
    else:
        Pinv = lambda v: _lin(v, pc.pinv, pc.pinv)
        pnorm = pc.pinv_norm
    Lop = lambda v: _lin(v, ops.grad, ops.grad_adjoint)
    Lt = lambda q: _lin(q, ops.grad_adjoint, ops.grad)

    def proj(v):
        if aniso:
            return torch.clamp(v, -1.0, 1.0)
        # the 1e-300 floor keeps the derivative of the norm finite at v = 0
        # (where the projection is the identity); it changes no value
        nrm = torch.sqrt(v[0] ** 2 + v[1] ** 2 + 1e-300)
        return v / torch.clamp(nrm, min=1.0)[None]

    x = torch.zeros((n, n), dtype=torch.float64)
    u = x.clone()
    Q = torch.zeros((2, n, n), dtype=torch.float64)
    lb = alpha * lam
    eta = 1.0 / (lb * lnorm2 * pnorm)
    t_prev = 1.0
    for _ in range(n_outer):
        s = u - alpha * Pinv(At(A(u) - y))
        R, Qp = Q, Q
        tau = 1.0
        for _ in range(n_inner):
            z = s - lb * Pinv(Lt(R))
            Qn = proj(R + eta * Lop(z))
            tau_n = (1.0 + np.sqrt(1.0 + 4.0 * tau * tau)) / 2.0
            R = Qn + ((tau - 1.0) / tau_n) * (Qn - Qp)
            Qp, tau = Qn, tau_n
        Q = Qp
        x_new = s - lb * Pinv(Lt(Q))
        t = (1.0 + np.sqrt(1.0 + 4.0 * t_prev * t_prev)) / 2.0
        u = x_new + ((t_prev - 1.0) / t) * (x_new - x)
        x, t_prev = x_new, t
    return x
