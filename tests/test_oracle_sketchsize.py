"""Pins of the sketch-size oracle (Thm. 2, Sec. II): d_eff as a trace against
d_eff as an eigenvalue sum, its limits, the closed-form spectra of the blur
and blur-plus-decimation operators against dense eigendecompositions, the
rule K = 2 ceil(1.5 d_eff + 1), and Thm. 2's bound E[kappa] < 28 on dense
blur and CT operators with the preconditioner of eq. (11)."""
import numpy as np
import pytest

import workloads as W
from oracle import operators as ops
from oracle import sketchsize as sz


def _psd(n, r, seed):
    G = np.random.default_rng(seed).standard_normal((n, r))
    return G @ G.T


@pytest.mark.parametrize("mu", [1e-3, 1.0, 1e2])
def test_deff_trace_equals_eigenvalue_sum(mu):
    Phi = _psd(40, 30, 1)
    eigs = np.linalg.eigvalsh(Phi)
    assert abs(sz.deff_dense(Phi, mu) - sz.deff_from_eigs(eigs, mu)) < 1e-10 * 40


def test_deff_limits_rank_and_zero():
    # a rank-30 spectrum in 40 dimensions
    eigs = np.concatenate([np.zeros(10), np.geomspace(1e-3, 1e2, 30)])
    top = eigs[-1]
    # mu -> 0: every nonzero eigenvalue counts once (rank 30); mu -> inf: 0
    assert abs(sz.deff_from_eigs(eigs, 1e-13 * top) - 30.0) < 1e-6
    assert abs(sz.deff_dense(np.diag(eigs), 1e-13 * top) - 30.0) < 1e-6
    assert sz.deff_from_eigs(eigs, 1e9 * top) < 1e-6
    # monotone decreasing in mu
    mus = top * np.logspace(-6, 3, 12)
    d = [sz.deff_from_eigs(eigs, m) for m in mus]
    assert all(a > b for a, b in zip(d, d[1:]))


def test_blur_spectrum_matches_dense_eigendecomposition():
    n, h = 12, W.gaussian_psf(5, 1.1)
    Phi = sz.dense_phi(lambda x: ops.blur(x, h), lambda y: ops.blur_adjoint(y, h), n, n)
    dense = np.sort(np.linalg.eigvalsh(Phi))
    closed = np.sort(sz.blur_eigs(h, n, n).ravel())
    assert np.max(np.abs(dense - closed)) < 1e-12 * closed[-1]


def test_blurdown_spectrum_matches_dense_eigendecomposition():
    n, h = 12, W.gaussian_psf(5, 1.2)
    Phi = sz.dense_phi(lambda x: ops.blurdown(x, h, 2), lambda y: ops.blurdown_adjoint(y, h, 2),
                       n, n)
    dense = np.sort(np.linalg.eigvalsh(Phi))
    closed = np.sort(sz.blurdown_eigs(h, n, n, 2).ravel())
    m = closed.size                                  # (n / 2)^2 nonzero eigenvalues
    assert m == (n // 2) ** 2
    assert np.max(np.abs(dense[-m:] - closed)) < 1e-12 * closed[-1]
    assert np.max(np.abs(dense[:-m])) < 1e-12 * closed[-1]


def test_rule_values():
    assert sz.sketch_size_rule(0.0) == 2
    assert sz.sketch_size_rule(10.0) == 32
    assert sz.sketch_size_rule(10.1) == 34
    assert sz.sketch_size_rule(2.0 / 3.0) == 4


def _mu_for(eigs, target):
    """mu with d_eff(mu) = target (bisection on log mu)."""
    lo, hi = 1e-16 * eigs.max(), 1e6 * eigs.max()
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if sz.deff_from_eigs(eigs, mid) > target:
            lo = mid
        else:
            hi = mid
    return np.sqrt(lo * hi)


def _theorem2(Phi, target, seeds):
    eigs = np.linalg.eigvalsh(Phi)
    mu = _mu_for(eigs, target)
    d = sz.deff_from_eigs(eigs, mu)
    K = sz.sketch_size_rule(d)
    kap = [sz.preconditioned_condition(Phi, mu, K, s) for s in seeds]
    plain = (eigs.max() + mu) / (max(eigs.min(), 0.0) + mu)
    return float(np.mean(kap)), plain, K


def test_theorem2_bound_on_a_steep_spectrum():
    """Phi with eigenvalues 10^(-i/4) in a random basis (N = 300), mu = 1e-8:
    the unpreconditioned condition number is ~1e8, d_eff ~ 33.  With the
    rule's K the preconditioned condition number averages below 28; with a
    quarter of it, it does not."""
    N = 300
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((N, N)))
    lam = 10.0 ** (-np.arange(N) / 4.0)
    Phi = (Q * lam) @ Q.T
    Phi = 0.5 * (Phi + Phi.T)
    mu = 1e-8
    d = sz.deff_from_eigs(lam, mu)
    K = sz.sketch_size_rule(d)
    assert 25 < d < 40 and K < N
    kap = np.mean([sz.preconditioned_condition(Phi, mu, K, s) for s in range(8)])
    assert kap < 28.0
    small = np.mean([sz.preconditioned_condition(Phi, mu, K // 4, s) for s in range(4)])
    assert small > 28.0


@pytest.mark.parametrize("kind", ["blur", "ct"])
def test_theorem2_bound_on_dense_operators(kind):
    """The workloads' operators on 16 x 16 images (a 9 x 9 Gaussian blur;
    parallel-beam Joseph with 30 views and 23 bins), mu such that d_eff = 20."""
    n = 16
    if kind == "blur":
        h = W.gaussian_psf(9, 1.5)
        Phi = sz.dense_phi(lambda x: ops.blur(x, h), lambda y: ops.blur_adjoint(y, h), n, n)
    else:
        Phi = sz.dense_phi(lambda x: ops.joseph(x, 30, 23), lambda p: ops.joseph_adjoint(p, n),
                           n, n)
    kap, plain, K = _theorem2(Phi, 20.0, range(8))
    assert K == 64
    assert kap < 28.0 and kap < plain
