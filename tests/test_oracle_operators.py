"""Pins of the oracle's operators against closed forms and brute force."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import operators as ops

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _psf_symbol(h, n1, n2):
    """DFT of the PSF placed with its centre at index (0, 0)."""
    k = h.shape[0]
    c = (k - 1) // 2
    hp = np.zeros((n1, n2))
    for a in range(k):
        for b in range(k):
            hp[(a - c) % n1, (b - c) % n2] += h[a, b]
    return np.fft.fft2(hp)


@pytest.mark.parametrize("k,sigma,n1,n2", [(9, 1.5, 32, 32), (7, 1.2, 16, 24),
                                           (5, 0.8, 20, 20)])
def test_blur_is_fft_convolution(k, sigma, n1, n2):
    h = W.gaussian_psf(k, sigma)
    x = W.gaussian((n1, n2), 1)
    H = _psf_symbol(h, n1, n2)
    ref = np.real(np.fft.ifft2(np.fft.fft2(x) * H))
    assert np.allclose(ops.blur(x, h), ref, rtol=0, atol=1e-13)
    ref_t = np.real(np.fft.ifft2(np.fft.fft2(x) * np.conj(H)))
    assert np.allclose(ops.blur_adjoint(x, h), ref_t, rtol=0, atol=1e-13)


def test_blur_nonsymmetric_psf_adjoint_and_orientation():
    # a one-hot PSF at (a, b) shifts by (a - c, b - c): (Hx)[i,j] = x[i+c-a, j+c-b]
    h = np.zeros((5, 5))
    h[0, 3] = 1.0
    x = W.gaussian((12, 10), 2)
    y = ops.blur(x, h)
    assert np.array_equal(y, np.roll(x, (0 - 2, 3 - 2), axis=(0, 1)))
    g = W.gaussian((5, 5), 3)
    r = W.gaussian((12, 10), 4)
    lhs = np.sum(ops.blur(x, g) * r)
    rhs = np.sum(x * ops.blur_adjoint(r, g))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) + 1e-13


def test_blur_ata_eigenvalues_match_fft_closed_form():
    n = 12
    h = W.gaussian_psf(9, 1.5)
    M = np.zeros((n * n, n * n))
    for j in range(n * n):
        e = np.zeros(n * n)
        e[j] = 1
        M[:, j] = ops.blur_adjoint(ops.blur(e.reshape(n, n), h), h).reshape(-1)
    ev = np.sort(np.linalg.eigvalsh(M))
    closed = np.sort(np.abs(_psf_symbol(h, n, n)).ravel() ** 2)
    assert np.allclose(ev, closed, atol=1e-12)
    # normalised PSF: the top eigenvalue is exactly 1 (DC)
    assert abs(ev[-1] - 1.0) < 1e-12


def test_blurdown_adjoint_and_alias_symbol():
    n, f = 16, 2
    h = W.gaussian_psf(7, 1.2)
    x = W.gaussian((n, n), 5)
    y = W.gaussian((n // f, n // f), 6)
    lhs = np.sum(ops.blurdown(x, h, f) * y)
    rhs = np.sum(x * ops.blurdown_adjoint(y, h, f))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # A A^T on the low-resolution grid is circulant with symbol
    # (1/f^2) sum over the f^2 aliases of |H(w)|^2
    H2 = np.abs(_psf_symbol(h, n, n)) ** 2
    m = n // f
    sym = np.zeros((m, m))
    for a in range(f):
        for b in range(f):
            sym += H2[a * m:(a + 1) * m, b * m:(b + 1) * m]
    sym /= f * f
    aat = ops.blurdown(ops.blurdown_adjoint(y, h, f), h, f)
    ref = np.real(np.fft.ifft2(np.fft.fft2(y) * sym))
    assert np.allclose(aat, ref, atol=1e-13)


def test_haar_orthonormal_and_closed_form_basis():
    n = 16
    x = W.gaussian((n, n), 7)
    w = ops.haar_analysis(x, 3)
    assert np.allclose(ops.haar_synthesis(w, 3), x, atol=1e-14)
    assert abs(np.sum(w * w) - np.sum(x * x)) < 1e-12 * np.sum(x * x)  # Parseval
    assert np.allclose(ops.haar_analysis(ops.haar_synthesis(x, 3), 3), x, atol=1e-14)

    def basis(i, j):
        e = np.zeros((n, n))
        e[i, j] = 1.0
        return ops.haar_synthesis(e, 3)

    # coarsest approximation: constant 1/8 on the 8 x 8 block
    ref = np.zeros((n, n))
    ref[8:16, 0:8] = 1 / 8
    assert np.allclose(basis(8, 0), ref, atol=1e-15)
    # coarsest horizontal detail (position (0, 4) of the block): +1/8 on the
    # left half, -1/8 on the right half
    ref = np.zeros((n, n))
    ref[0:8, 0:4] = 1 / 8
    ref[0:8, 4:8] = -1 / 8
    assert np.allclose(basis(0, 4), ref, atol=1e-15)
    # coarsest diagonal detail (position (4, 4)): checkerboard of quadrants
    ref = np.zeros((n, n))
    ref[0:4, 0:4] = ref[4:8, 4:8] = 1 / 8
    ref[0:4, 4:8] = ref[4:8, 0:4] = -1 / 8
    assert np.allclose(basis(4, 4), ref, atol=1e-15)
    # second level vertical detail at (2, 0) of the block at (8, 8): rows 8-9
    # vs rows 10-11 of the 4 x 4 block at (8, 8), magnitude 1/4
    ref = np.zeros((n, n))
    ref[8:10, 8:12] = 1 / 4
    ref[10:12, 8:12] = -1 / 4
    assert np.allclose(basis(10, 8), ref, atol=1e-15)
    # finest diagonal detail at (1, 1): 1/2 [[1, -1], [-1, 1]]
    ref = np.zeros((n, n))
    ref[0, 0] = ref[1, 1] = 0.5
    ref[0, 1] = ref[1, 0] = -0.5
    assert np.allclose(basis(1, 1), ref, atol=1e-15)
    # a constant image has only the coarsest approximation coefficients, 8c
    c = ops.haar_analysis(np.full((n, n), 0.3), 3)
    mask = np.zeros((n, n), bool)
    mask[::8, ::8] = True
    assert np.allclose(c[mask], 2.4) and np.allclose(c[~mask], 0, atol=1e-15)


def _joseph_literal(x, V, B):
    """Pure-Python loop version of the projector for tiny sizes."""
    n = x.shape[0]
    c = (n - 1) / 2
    out = np.zeros((V, B))
    for v in range(V):
        th = math.pi * v / V
        ct, st = math.cos(th), math.sin(th)
        for b in range(B):
            s = b - (B - 1) / 2
            acc = 0.0
            for t in range(n):
                tc = t - c
                if abs(ct) >= abs(st):
                    f = (s - tc * st) / ct + c
                    j0 = math.floor(f)
                    w = f - j0
                    for j, wj in ((j0, 1 - w), (j0 + 1, w)):
                        if 0 <= j < n:
                            acc += wj * x[t, j] / abs(ct)
                else:
                    f = (s - tc * ct) / st + c
                    i0 = math.floor(f)
                    w = f - i0
                    for i, wi in ((i0, 1 - w), (i0 + 1, w)):
                        if 0 <= i < n:
                            acc += wi * x[i, t] / abs(st)
            out[v, b] = acc
    return out


def test_joseph_matches_literal_loop_and_is_exact_transpose():
    n, V, B = 8, 7, 13
    x = W.gaussian((n, n), 8)
    p = ops.joseph(x, V, B)
    assert np.allclose(p, _joseph_literal(x, V, B), atol=1e-13)
    # dense matrix brute force: the backprojector is its transpose
    A = np.stack([ops.joseph(e.reshape(n, n), V, B).reshape(-1)
                  for e in np.eye(n * n)], axis=1)
    At = np.stack([ops.joseph_adjoint(e.reshape(V, B), n).reshape(-1)
                   for e in np.eye(V * B)], axis=1)
    assert np.allclose(A.T, At, atol=1e-14)


def test_joseph_axis_aligned_views_give_exact_line_sums():
    # n = 64, B = 92 (both even): bin centres line up with pixel centres
    n, B, V = 64, 92, 4
    x = W.gaussian((n, n), 9)
    p = ops.joseph(x, V, B)
    off = (B - n) // 2
    # theta = 0: x = s, the ray for bin b is column b - off
    assert np.allclose(p[0, off:off + n], x.sum(axis=0), atol=1e-12)
    assert np.allclose(p[0, :off], 0) and np.allclose(p[0, off + n:], 0)
    # theta = pi / 2: y = s, the ray for bin b is row b - off
    assert np.allclose(p[2, off:off + n], x.sum(axis=1), atol=1e-9)


def test_joseph_disc_gives_chord_lengths():
    n, B, V = 128, 160, 6
    c = (n - 1) / 2
    yy, xx = np.mgrid[0:n, 0:n] - c
    r = 40.0
    disc = (xx ** 2 + yy ** 2 <= r * r).astype(float)
    p = ops.joseph(disc, V, B)
    s = np.arange(B) - (B - 1) / 2
    chord = 2 * np.sqrt(np.maximum(r * r - s * s, 0))
    for v in range(V):
        inner = np.abs(s) < r - 3
        err = np.abs(p[v, inner] - chord[inner])
        assert np.max(err) < 2.5 and np.mean(err) < 0.8


@pytest.mark.parametrize("reg", ["grad", "hessian"])
def test_difference_operators_follow_appendix_a_stencils(reg):
    with open(os.path.join(GOLDEN, "app_a_stencils.json")) as fh:
        st = json.load(fh)[reg]
    n = 9
    x = W.gaussian((n, n), 10)
    out = ops.grad(x) if reg == "grad" else ops.hessian(x)
    names = ["v1", "v2"] if reg == "grad" else ["v11", "v22", "v12"]
    for ch, name in enumerate(names):
        for i in range(2, n - 2):
            for j in range(2, n - 2):
                ref = sum(w * x[i + int(k.split(",")[0]), j + int(k.split(",")[1])]
                          for k, w in st[name].items())
                assert abs(out[ch, i, j] - ref) < 1e-14


def test_difference_operators_boundaries_and_adjoints():
    n1, n2 = 7, 9
    x = W.gaussian((n1, n2), 11)
    g = ops.grad(x)
    assert np.all(g[0, 0, :] == 0) and np.all(g[1, :, 0] == 0)
    q = W.gaussian((2, n1, n2), 12)
    assert abs(np.sum(g * q) - np.sum(x * ops.grad_adjoint(q))) < 1e-12
    hs = ops.hessian(x)
    q3 = W.gaussian((3, n1, n2), 13)
    lhs = ops.pair(q3, hs, "hs1")
    assert abs(lhs - np.sum(x * ops.hessian_adjoint(q3))) < 1e-12
    # replicate padding: v11 on the first row is X[1] - X[0]
    assert np.allclose(hs[0, 0, :], x[1, :] - x[0, :])
    # closed forms: ramp in i -> grad (1, 0); i*j -> v12 = 1 inside
    i, j = np.mgrid[0:n1, 0:n2].astype(float)
    assert np.allclose(ops.grad(i)[0, 1:, :], 1) and np.allclose(ops.grad(i)[1], 0)
    assert np.allclose(ops.hessian(i * j)[2, 1:-1, 1:-1], 1)
    assert np.allclose(ops.hessian(i * i)[0, 1:-1, :], 2)


@pytest.mark.parametrize("reg,bound", [("tv", 8.0), ("hs1", 34.0)])
def test_difference_operator_norm_bounds(reg, bound):
    n = 24
    L = ops.grad if reg == "tv" else ops.hessian
    Lt = ops.grad_adjoint if reg == "tv" else ops.hessian_adjoint
    v = W.gaussian((n, n), 14)
    lam = 0
    for _ in range(300):
        w = Lt(L(v))
        lam = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    assert lam <= bound and lam > 0.9 * bound - 4


# --- Daubechies-4 (next-row wavelet) ---------------------------------------

def test_db4_filter_is_orthonormal_with_four_vanishing_moments_and_minimum_phase():
    h = ops.daubechies_filter(4)
    assert len(h) == 8 and abs(h.sum() - np.sqrt(2)) < 1e-14
    for j in range(4):     # double-shift orthonormality
        assert abs(sum(h[k] * h[k + 2 * j] for k in range(8 - 2 * j)) - (j == 0)) < 1e-14
    g = np.array([(-1) ** k * h[7 - k] for k in range(8)])
    for m in range(4):     # the wavelet filter annihilates polynomials of degree < 4
        assert abs(sum(k ** m * g[k] for k in range(8))) < 1e-10
    assert abs(sum(k ** 4 * g[k] for k in range(8))) > 1e-3
    # minimum phase: apart from the fourfold zero at -1, every zero of
    # sum_k h_k z^(7-k) lies inside the unit circle, and the energy is front-loaded
    zeros = np.roots(h)
    far = zeros[np.abs(zeros + 1) > 1e-2]
    assert len(far) == 3 and np.all(np.abs(far) < 1)
    assert h[0] ** 2 + h[1] ** 2 > h[6] ** 2 + h[7] ** 2


@pytest.mark.parametrize("shape,levels", [((16, 16), 2), ((32, 16), 3), ((16, 16), 4)])
def test_db4_transform_is_orthonormal_and_inverted_by_its_transpose(shape, levels):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(shape)
    w = ops.db4_analysis(x, levels)
    assert abs(np.linalg.norm(w) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    assert np.allclose(ops.db4_synthesis(w, levels), x, atol=1e-12)
    # the dense matrix of the transform is orthogonal, and synthesis is its transpose
    N = x.size
    E = np.eye(N).reshape((N,) + shape)
    M = np.stack([ops.db4_analysis(e, levels).reshape(-1) for e in E], axis=1)
    assert np.allclose(M @ M.T, np.eye(N), atol=1e-12)
    z = rng.standard_normal(shape)
    assert np.allclose(ops.db4_synthesis(z, levels).reshape(-1), M.T @ z.reshape(-1), atol=1e-12)


def test_db4_details_vanish_on_cubics():
    # a cubic in the row index: the first-level detail rows of interior
    # (non-wrapping) coefficients vanish (four vanishing moments)
    n = 32
    t = np.arange(n, dtype=np.float64)
    x = np.tile((0.3 * t ** 3 - 2 * t ** 2 + t - 5)[:, None], (1, n))
    w = ops.db4_analysis(x, 1)
    # column transform: rows n/2 + i hold the details of rows 2i .. 2i + 7
    interior = [n // 2 + i for i in range(n // 2) if 2 * i + 7 < n]
    assert np.max(np.abs(w[interior, :n // 2])) < 1e-9 * np.max(np.abs(x))
    assert np.max(np.abs(w[n // 2 + n // 2 - 1, :n // 2])) > 1.0   # the wrapped one does not


# --- fan-beam Joseph (next-row geometry) ------------------------------------

def test_fan_joseph_is_the_exact_transpose():
    n, V, B = 8, 6, 11
    src, det, du = 20.0, 10.0, 1.3
    E = np.eye(n * n).reshape(n * n, n, n)
    A = ops.fan_joseph(E, V, B, src, det, du).reshape(n * n, V * B).T
    Et = np.eye(V * B).reshape(V * B, V, B)
    At = ops.fan_joseph_adjoint(Et, n, src, det, du).reshape(V * B, n * n).T
    assert np.allclose(At, A.T, atol=1e-13)


def test_fan_joseph_tends_to_the_parallel_beam_projector():
    # source at infinity: the rays of view v are the parallel rays at angle
    # 2 pi v / V with the detector coordinate u; views 0 .. V/2 - 1 cover the
    # parallel-beam views over 180 degrees
    n, V, B = 24, 8, 31
    x = np.random.default_rng(4).standard_normal((n, n))
    fan = ops.fan_joseph(x, V, B, 1e9, 0.0, 1.0)
    par = ops.joseph(x, V // 2, B)
    assert np.allclose(fan[: V // 2], par, atol=1e-6 * np.abs(par).max())


def test_fan_joseph_central_ray_through_a_disc():
    # a disc of radius r centred in the image: the central ray of every view
    # passes through the centre, so its line integral is the chord 2 r
    n, r = 96, 30.0
    c = (n - 1) / 2.0
    i, j = np.mgrid[0:n, 0:n]
    disc = ((i - c) ** 2 + (j - c) ** 2 <= r * r).astype(np.float64)
    p = ops.fan_joseph(disc, 12, 41, 150.0, 60.0, 1.5)
    assert np.all(np.abs(p[:, 20] - 2 * r) <= 1.5)
