"""Pins of the WAPG rate constant L_f^P ||x^1 - x*||_P^2 (`rate_constant`):
its metric from eq. (11)'s P on the sketched subspace and off it, L_f^P of a
periodic blur without a preconditioner (the top of |DFT(h)|^2) and with a
full sketch (the closed spectrum of P^{-1} A^T A)."""
import numpy as np

import workloads as W
from oracle import nystrom as nys
from oracle import solver as sv


def _blur(n, k, sigma, lam=1e-3, seed=0):
    h = W.gaussian_psf(k, sigma)
    prob = sv.Problem("blur", n, None, lam, "tv", h=h)
    prob.y = prob.A(W.phantom_blocks(n, seed)) + 0.01 * W.gaussian((n, n), seed)
    return prob, h


def _blur_spectrum(h, n):
    """Eigenvalues of A^T A for the periodic blur: |DFT of the wrapped PSF|^2."""
    k = h.shape[0]
    H = np.zeros((n, n))
    for a in range(k):
        for b in range(k):
            H[(a - k // 2) % n, (b - k // 2) % n] += h[a, b]
    return np.sort((np.abs(np.fft.fft2(H)) ** 2).ravel())


def test_plain_constant_is_the_top_blur_eigenvalue_times_the_distance():
    n = 16
    prob, h = _blur(n, 5, 1.0)
    lam_max = _blur_spectrum(h, n)[-1]
    xs = W.phantom_blocks(n, 3)
    v0 = W.gaussian((n, n), 1, stream=7)
    r = sv.rate_constant(prob, None, xs, v0, 400)
    assert abs(r["L"] - lam_max) <= 1e-9 * lam_max
    assert abs(r["pdist2"] - np.sum(xs * xs)) <= 1e-12 * np.sum(xs * xs)
    assert abs(r["value"] - lam_max * np.sum(xs * xs)) <= 1e-8 * r["value"]
    # x^1 = x* gives zero
    assert sv.rate_constant(prob, None, xs, v0, 5, x1=xs)["pdist2"] == 0.0


def test_metric_is_eq6_p_on_and_off_the_sketched_subspace():
    n, K = 12, 6
    prob, _ = _blur(n, 5, 1.2)
    om = W.omega(K, n, n, 4)
    for tail in ("plain", "sqrt"):
        pc, r = sv.build_precond(prob, om, tail=tail)
        sK = float(r["shat"][-1]) if tail == "plain" else float(np.sqrt(r["shat"][-1]))
        v0 = W.gaussian((n, n), 2, stream=7)
        for k in range(pc.U.shape[0]):
            uk = pc.U[k].reshape(n, n)
            got = sv.rate_constant(prob, pc, -uk, v0, 3)["pdist2"]
            want = (r["shat"][k] + pc.mu) / (sK + pc.mu)
            assert abs(got - want) <= 1e-10 * want
        # a direction orthogonal to the sketched subspace keeps its norm
        d = W.gaussian((n * n,), 5)
        d -= pc.U.T @ (pc.U @ d)
        got = sv.rate_constant(prob, pc, -d.reshape(n, n), v0, 3)["pdist2"]
        assert abs(got - d @ d) <= 1e-10 * (d @ d)


def test_full_sketch_constant_is_the_closed_spectrum():
    """K = N: the Nystrom approximation is A^T A itself, so P^{-1} A^T A has the
    eigenvalues (s_min + mu) s_i / (s_i + mu) (eq. (11), plain tail) and L_f^P
    is their largest."""
    n = 8
    prob, h = _blur(n, 3, 0.6)
    s = _blur_spectrum(h, n)
    om = W.omega(n * n, n, n, 6)
    pc, r = sv.build_precond(prob, om, tail="plain")
    assert abs(r["shat"][-1] - s[0]) <= 1e-8 * s[-1]
    want = (s[0] + pc.mu) * s[-1] / (s[-1] + pc.mu)
    v0 = W.gaussian((n, n), 3, stream=7)
    got = sv.rate_constant(prob, pc, np.zeros((n, n)), v0, 50)["L"]
    assert abs(got - want) <= 1e-7 * want
