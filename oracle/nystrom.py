"""FP64 oracle: randomized Nystrom approximation, preconditioner, step size.

Test infrastructure only.  Columns of the tall matrices are stored as rows
here (Omega, Y, U have shape (K, N)); the formulas below are written for the
paper's N x K orientation and transposed on entry.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

EPS64 = 2.0 ** -52


class NotPositiveDefinite(RuntimeError):
    pass


def shift(Y: np.ndarray, Omega: np.ndarray, mode: str = "spectral",
          eps: float = EPS64) -> float:
    """Nystrom shift nu.

    'paper'    : eps * ||Omega||_F                      (Alg. 1, step 3)
    'spectral' : sqrt(N) * eps * ||Y||_2, the workloads' own choice, with the
                 spectral norm of the N x K matrix Y.
    """
    if mode == "paper":
        return eps * float(np.linalg.norm(Omega))
    N = Y.shape[1]
    return float(np.sqrt(N) * eps * np.linalg.norm(Y.T, 2))


def nystrom(Y: np.ndarray, Omega: np.ndarray, nu_mode: str = "spectral",
            eps: float = EPS64, max_escalations: int = 6):
    """Alg. 1, steps 3-8, in the paper's order.

    Y, Omega: (K, N).  Returns dict(U=(K_eff, N), shat=(K_eff,) descending,
    nu=shift used, S=singular values of B).  If the Cholesky factorisation of
    Omega^T Y_nu fails, nu is multiplied by 10 and the steps are repeated, at
    most `max_escalations` times (reading: the paper is silent on failure).
    Columns whose clipped eigenvalue is 0 are dropped (reading).
    """
    Om = np.asarray(Omega, np.float64).T          # N x K
    Yt = np.asarray(Y, np.float64).T              # N x K
    nu = shift(Y, Omega, nu_mode, eps)
    for attempt in range(max_escalations + 1):
        Yv = Yt + nu * Om                          # step 4
        G = Om.T @ Yv
        G = 0.5 * (G + G.T)                        # symmetrise (silent in paper)
        try:
            C = np.linalg.cholesky(G)              # step 5, lower: C C^T = G
        except np.linalg.LinAlgError:
            if attempt == max_escalations:
                raise NotPositiveDefinite(f"Cholesky failed with nu={nu}")
            nu *= 10.0
            continue
        # step 6: B = Y_nu C^{-T}  <=>  B^T = C^{-1} Y_nu^T
        B = solve_triangular(C, Yv.T, lower=True).T
        U, S, _ = np.linalg.svd(B, full_matrices=False)   # step 7
        shat = np.maximum(0.0, S ** 2 - nu)                  # step 8
        keep = shat > 0
        return dict(U=U[:, keep].T.copy(), shat=shat[keep], nu=nu, S=S,
                    escalations=attempt)
    raise AssertionError("unreachable")


def tail_value(shat: np.ndarray, tail: str = "sqrt") -> float:
    """The value used for s_K in the preconditioner: the smallest retained
    eigenvalue, or its square root (the paper's heuristic, Sec. III-B)."""
    sK = float(shat[-1])
    return float(np.sqrt(sK)) if tail == "sqrt" else sK


def pinv_apply(v: np.ndarray, U: np.ndarray, shat: np.ndarray, mu: float,
               tail: str = "sqrt") -> np.ndarray:
    """P^{-1} v = (s_K + mu) U (S + mu I)^{-1} U^T v + (I - U U^T) v, eq. (11).

    v may be a stack (..., N); U is (K, N) with orthonormal rows.
    """
    sK = tail_value(shat, tail)
    c = v @ U.T                                     # U^T v, shape (..., K)
    return (sK + mu) * ((c / (shat + mu)) @ U) + v - c @ U


def p_apply(v: np.ndarray, U: np.ndarray, shat: np.ndarray, mu: float,
            tail: str = "sqrt") -> np.ndarray:
    """P v = U (S + mu I) U^T v / (s_K + mu) + (I - U U^T) v, eq. (11)."""
    sK = tail_value(shat, tail)
    c = v @ U.T
    return ((c * (shat + mu)) @ U) / (sK + mu) + v - c @ U


def pinv_norm(shat: np.ndarray, mu: float, tail: str = "sqrt") -> float:
    """||P^{-1}||_2 = max(1, max_i (s_K + mu) / (s_i + mu))."""
    sK = tail_value(shat, tail)
    return float(max(1.0, np.max((sK + mu) / (shat + mu))))


def power_iteration(apply_M, v0: np.ndarray, iters: int) -> float:
    """Largest eigenvalue of M = P^{-1} H by the power method.

    P^{-1} H is similar to the symmetric P^{-1/2} H P^{-1/2}, so its spectrum
    is real and non-negative.  Fixed count: w = M v, lambda = ||w||,
    v = w / lambda.  Used for the step size alpha = 1 / (1.01 L) of Alg. 3.
    """
    v = v0 / np.linalg.norm(v0)
    lam = 0.0
    for _ in range(iters):
        w = apply_M(v)
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam
