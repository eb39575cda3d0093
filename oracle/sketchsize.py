"""FP64 oracle: the sketch-size rule of Thm. 2 (Sec. II).

Test infrastructure only.  Thm. 2 (the paper quotes it from Frangella et al.)
concerns the regularised system (Phi + mu I) x = b: with the preconditioner
P of eq. (11) built from K = 2 ceil(1.5 d_eff(mu) + 1) sketch columns, where
d_eff(mu) = tr(Phi (Phi + mu I)^{-1}) is the effective dimension, the
expected condition number of P^{-1/2} (Phi + mu I) P^{-1/2} is below 28.

The functions below evaluate d_eff from a spectrum or from a dense matrix,
the spectra of the workloads' Phi = A^T A in closed form (periodic blur: the
squared magnitude of the PSF's DFT; blur followed by 2x decimation: the
four-alias symbol of A A^T, whose values are the nonzero eigenvalues of
A^T A) or densely (any operator on a small image), the rule itself, and the
preconditioned condition number of a dense Phi.
"""
from __future__ import annotations

import math

import numpy as np

from . import nystrom as nys


def deff_from_eigs(eigs: np.ndarray, mu: float) -> float:
    """d_eff(mu) = sum_i lam_i / (lam_i + mu) over the eigenvalues of Phi."""
    lam = np.clip(np.asarray(eigs, np.float64).ravel(), 0.0, None)
    return float(np.sum(lam / (lam + mu)))


def deff_dense(Phi: np.ndarray, mu: float) -> float:
    """d_eff(mu) = tr(Phi (Phi + mu I)^{-1}), by a dense solve."""
    n = Phi.shape[0]
    X = np.linalg.solve(Phi + mu * np.eye(n), Phi)     # (Phi + mu I)^{-1} Phi
    return float(np.trace(X))


def sketch_size_rule(deff: float) -> int:
    """K = 2 ceil(1.5 d_eff + 1) (Thm. 2)."""
    return 2 * int(math.ceil(1.5 * deff + 1.0))


def blur_eigs(h: np.ndarray, n1: int, n2: int) -> np.ndarray:
    """Eigenvalues of A^T A for the periodic blur by the k x k PSF h on an
    n1 x n2 image: A is circulant, so they are |DFT(h placed at the origin)|^2."""
    k = h.shape[0]
    c = (k - 1) // 2
    pad = np.zeros((n1, n2))
    for a in range(k):
        for b in range(k):
            pad[(a - c) % n1, (b - c) % n2] += h[a, b]
    return np.abs(np.fft.fft2(pad)) ** 2


def blurdown_eigs(h: np.ndarray, n1: int, n2: int, factor: int = 2) -> np.ndarray:
    """Nonzero spectrum of A^T A for A = S H (periodic blur, then keep every
    factor-th sample on both axes): the eigenvalues of the circulant A A^T on
    the coarse grid, whose symbol at coarse frequency w is the mean of
    |h^|^2 over the factor^2 fine frequencies that alias onto w."""
    fine = blur_eigs(h, n1, n2)
    m1, m2 = n1 // factor, n2 // factor
    sym = np.zeros((m1, m2))
    for p in range(factor):
        for q in range(factor):
            sym += fine[p * m1:(p + 1) * m1, q * m2:(q + 1) * m2]
    return sym / factor ** 2


def dense_phi(apply_A, apply_At, n1: int, n2: int) -> np.ndarray:
    """Phi = A^T A as a dense N x N matrix, column by column from unit images."""
    N = n1 * n2
    Phi = np.zeros((N, N))
    e = np.zeros((n1, n2))
    for j in range(N):
        e.flat[j] = 1.0
        Phi[:, j] = np.asarray(apply_At(apply_A(e))).ravel()
        e.flat[j] = 0.0
    return 0.5 * (Phi + Phi.T)


def preconditioned_condition(Phi: np.ndarray, mu: float, K: int, seed: int,
                             tail: str = "plain") -> float:
    """kappa(P^{-1/2} (Phi + mu I) P^{-1/2}) with P of eq. (11) built by Alg. 1
    from a K-column Gaussian sketch of the dense Phi (the eigenvalues of that
    matrix are those of P^{-1} (Phi + mu I), which is similar to it)."""
    n = Phi.shape[0]
    Omega = np.random.default_rng(seed).standard_normal((K, n))
    r = nys.nystrom(Omega @ Phi, Omega)                    # Y = Phi Omega, rows = columns
    U, shat = r["U"], r["shat"]
    Pinv = nys.pinv_apply(np.eye(n), U, shat, mu, tail)    # rows: P^{-1} e_i
    M = Pinv @ (Phi + mu * np.eye(n))
    ev = np.sort(np.real(np.linalg.eigvals(M)))
    return float(ev[-1] / ev[0])
