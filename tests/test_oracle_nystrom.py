"""Pins of the oracle's Alg. 1, preconditioner and power method."""
import numpy as np
import pytest

import workloads as W
from oracle import nystrom as nys
from oracle import operators as ops
from oracle import solver as sv


def _psd_low_rank(N, r, seed):
    G = W.gaussian((N, r), seed)
    return G @ G.T


def test_exact_recovery_of_low_rank_psd():
    N, K, r = 60, 12, 7
    Phi = _psd_low_rank(N, r, 1)
    Om = W.omega(K, 1, N, 2).reshape(K, N)
    Y = Om @ Phi            # rows are the columns Phi omega_k (Phi symmetric)
    res = nys.nystrom(Y, Om)
    U, s = res["U"], res["shat"]
    approx = U.T @ np.diag(s) @ U
    assert np.linalg.norm(approx - Phi) < 1e-9 * np.linalg.norm(Phi)
    ev = np.sort(np.linalg.eigvalsh(Phi))[::-1][:r]
    assert np.allclose(s[:r], ev, rtol=1e-9)
    # U has orthonormal rows
    assert np.allclose(U @ U.T, np.eye(U.shape[0]), atol=1e-10)


def test_matches_nystrom_formula_on_well_conditioned_case():
    # eq. (9): Phi<Omega> = (Phi Omega)(Omega^T Phi Omega)^+ (Phi Omega)^T
    N, K = 50, 10
    ev = np.linspace(1.0, 2.0, N)
    Q, _ = np.linalg.qr(W.gaussian((N, N), 3))
    Phi = Q @ np.diag(ev) @ Q.T
    Om = W.omega(K, 1, N, 4).reshape(K, N).T      # N x K
    Y = Phi @ Om
    ref = Y @ np.linalg.pinv(Om.T @ Y) @ Y.T
    res = nys.nystrom(Y.T, Om.T)
    approx = res["U"].T @ np.diag(res["shat"]) @ res["U"]
    assert np.linalg.norm(approx - ref) < 1e-11 * np.linalg.norm(ref)
    # rank <= K, PSD, and Loewner order Phi<Omega> <= Phi
    w = np.linalg.eigvalsh(Phi - approx)
    assert w.min() > -1e-10


def test_full_sketch_of_blur_recovers_fft_spectrum():
    # 16 x 16 image, K = N: the Nystrom approximation is Phi itself
    n = 16
    N = n * n
    h = W.gaussian_psf(5, 1.0)
    prob = sv.Problem("blur", n, None, 0.0, "tv", h=h)
    Om = W.omega(N, n, n, 5)
    Y = sv.sketch(prob, Om).reshape(N, N)
    res = nys.nystrom(Y, Om.reshape(N, N))
    k = 5
    c = 2
    hp = np.zeros((n, n))
    for a in range(k):
        for b in range(k):
            hp[(a - c) % n, (b - c) % n] = h[a, b]
    closed = np.sort(np.abs(np.fft.fft2(hp)).ravel() ** 2)[::-1]
    m = len(res["shat"])
    # eigenvalues above the shift are recovered; the rest are clipped away
    big = closed > 1e-8
    assert np.allclose(res["shat"][: big.sum()], closed[big], rtol=1e-7, atol=1e-12)
    assert m <= N


def test_shift_modes_and_escalation():
    N, K = 40, 6
    Om = W.omega(K, 1, N, 6).reshape(K, N)
    Phi = _psd_low_rank(N, 20, 7)
    Y = Om @ Phi
    nu_p = nys.shift(Y, Om, "paper")
    assert abs(nu_p - nys.EPS64 * np.linalg.norm(Om)) < 1e-30
    nu_s = nys.shift(Y, Om, "spectral")
    assert abs(nu_s - np.sqrt(N) * nys.EPS64 * np.linalg.svd(Y, compute_uv=False)[0]) < 1e-25
    # an indefinite operator makes Omega^T Y indefinite: escalation then error
    Yneg = -Y
    with pytest.raises(nys.NotPositiveDefinite):
        nys.nystrom(Yneg, Om, max_escalations=2)


def _precond_case(tail):
    N, K = 80, 8
    ev = np.concatenate([np.linspace(50, 10, K), np.linspace(2, 0.1, N - K)])
    Q, _ = np.linalg.qr(W.gaussian((N, N), 8))
    Phi = Q @ np.diag(ev) @ Q.T
    Om = W.omega(K, 1, N, 9).reshape(K, N)
    res = nys.nystrom(Om @ Phi, Om)
    return res["U"], res["shat"], Phi


@pytest.mark.parametrize("tail", ["sqrt", "plain"])
def test_preconditioner_inverse_and_spectrum(tail):
    U, s, _ = _precond_case(tail)
    mu = 1e-3
    N = U.shape[1]
    v = W.gaussian((N,), 10)
    pv = nys.p_apply(v, U, s, mu, tail)
    assert np.allclose(nys.pinv_apply(pv, U, s, mu, tail), v, atol=1e-12)
    sK = np.sqrt(s[-1]) if tail == "sqrt" else s[-1]
    # eigenvectors: columns of U with (s_K + mu)/(s_i + mu); complement with 1
    for i in range(U.shape[0]):
        out = nys.pinv_apply(U[i], U, s, mu, tail)
        assert np.allclose(out, (sK + mu) / (s[i] + mu) * U[i], atol=1e-12)
    w = v - (v @ U.T) @ U
    assert np.allclose(nys.pinv_apply(w, U, s, mu, tail), w, atol=1e-12)
    assert abs(nys.pinv_norm(s, mu, tail) - max(1.0, (sK + mu) / (s[-1] + mu))) < 1e-15
    if tail == "plain":
        # the last direction is left unscaled: the last column of U-bar is 0
        assert np.allclose(nys.pinv_apply(U[-1], U, s, mu, tail), U[-1], atol=1e-12)


def test_power_iteration_on_known_spectrum():
    N = 50
    ev = np.concatenate([[3.0], np.linspace(2.0, 0.1, N - 1)])
    Q, _ = np.linalg.qr(W.gaussian((N, N), 11))
    M = Q @ np.diag(ev) @ Q.T
    lam = nys.power_iteration(lambda v: M @ v, W.gaussian((N,), 12), 200)
    assert abs(lam - 3.0) < 1e-10
    # similar to a symmetric matrix: P^{-1} H has a real top eigenvalue
    U, s, Phi = _precond_case("plain")
    lam = nys.power_iteration(lambda v: nys.pinv_apply(Phi @ v, U, s, 0.0, "plain"),
                              W.gaussian((Phi.shape[0],), 13), 2000)
    Pinv = np.stack([nys.pinv_apply(e, U, s, 0.0, "plain") for e in np.eye(Phi.shape[0])])
    ref = np.max(np.real(np.linalg.eigvals(Pinv @ Phi)))
    assert abs(lam - ref) < 1e-6 * ref


def test_preconditioning_lowers_lipschitz_constant_on_steep_spectrum():
    U, s, Phi = _precond_case("plain")
    N = Phi.shape[0]
    Pinv = np.stack([nys.pinv_apply(e, U, s, 0.0, "plain") for e in np.eye(N)])
    Lp = np.max(np.real(np.linalg.eigvals(Pinv @ Phi)))
    L = np.max(np.linalg.eigvalsh(Phi))
    assert L == pytest.approx(50.0)
    assert Lp < 0.4 * L
