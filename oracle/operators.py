"""FP64 oracle: forward/adjoint operators written as their plain definitions.

Test infrastructure only (see the package docstring).  Every operator acts on
the last two axes, so a stack of images (..., n1, n2) is processed at once.

Operators
- periodic blur H and its adjoint (Sec. IV-A; the PSF enters the definition as
  a k x k array, centre (k-1)/2):
      (H x)[i, j]  = sum_{a,b} h[a, b] x[(i + c - a) mod n1, (j + c - b) mod n2]
      (H^T y)[i, j] = sum_{a,b} h[a, b] y[(i - c + a) mod n1, (j - c + b) mod n2]
- blur + decimation A = S H, S keeps the samples (f i, f j) (Sec. IV-A).
- orthonormal Haar pyramid W (analysis) and W^T (synthesis), 'in place'
  coefficient layout: each level replaces the 2 x 2 groups of the current
  low-pass grid by (LL, HL; LH, HH) at the same positions; level l acts on the
  grid of stride 2^l.  The wavelet regulariser of Sec. III-B uses x = W^T xbar.
- parallel-beam ray-driven (Joseph) projector and its transpose (Sec. IV-B):
  unit pixels centred at the origin, pixel (i, j) at (x, y) = (j - c, i - c)
  with c = (n - 1) / 2; bin b at s = b - (B - 1) / 2; view v at
  theta = v pi / V; the ray is {p : p . (cos t, sin t) = s}.  If
  |cos t| >= |sin t| the ray is sampled on every pixel row with linear
  interpolation between the two neighbouring columns and weight 1/|cos t|,
  otherwise on every column between rows with weight 1/|sin t|; samples
  outside the image read zero.  The adjoint is the same loop with a scatter.
- first-order differences (TV) and second-order differences (Hessian) of
  App. A, with the boundary readings stated at each function.
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# periodic blur

def blur(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """H x: periodic convolution with the k x k PSF h."""
    k = h.shape[0]
    c = (k - 1) // 2
    out = np.zeros_like(x, dtype=np.float64)
    for a in range(k):
        for b in range(k):
            # np.roll(x, s)[i] = x[i - s]; s = a - c gives x[i + c - a]
            out += h[a, b] * np.roll(x, shift=(a - c, b - c), axis=(-2, -1))
    return out


def blur_adjoint(y: np.ndarray, h: np.ndarray) -> np.ndarray:
    """H^T y: periodic correlation with h."""
    k = h.shape[0]
    c = (k - 1) // 2
    out = np.zeros_like(y, dtype=np.float64)
    for a in range(k):
        for b in range(k):
            out += h[a, b] * np.roll(y, shift=(c - a, c - b), axis=(-2, -1))
    return out


# --------------------------------------------------------------------------
# blur followed by decimation

def blurdown(x: np.ndarray, h: np.ndarray, f: int) -> np.ndarray:
    """S H x, keeping rows and columns 0, f, 2f, ..."""
    return blur(x, h)[..., ::f, ::f]


def blurdown_adjoint(y: np.ndarray, h: np.ndarray, f: int) -> np.ndarray:
    """H^T S^T y: zero-filled upsampling, then correlation."""
    shape = y.shape[:-2] + (y.shape[-2] * f, y.shape[-1] * f)
    z = np.zeros(shape)
    z[..., ::f, ::f] = y
    return blur_adjoint(z, h)


# --------------------------------------------------------------------------
# orthonormal Haar pyramid, in-place layout

def _haar_2x2(a, b, c, d):
    # orthonormal 2-D Haar of one 2 x 2 group [[a, b], [c, d]]; the 4 x 4
    # matrix is symmetric and orthogonal, hence its own inverse
    return ((a + b + c + d) / 2, (a - b + c - d) / 2,
            (a + b - c - d) / 2, (a - b - c + d) / 2)


def haar_analysis(x: np.ndarray, levels: int) -> np.ndarray:
    """W x: `levels` levels of the 2-D orthonormal Haar transform."""
    y = np.array(x, dtype=np.float64, copy=True)
    for lev in range(levels):
        s = 2 ** lev
        g = y[..., ::s, ::s]          # current low-pass grid (a view)
        a, b = g[..., 0::2, 0::2].copy(), g[..., 0::2, 1::2].copy()
        c, d = g[..., 1::2, 0::2].copy(), g[..., 1::2, 1::2].copy()
        ll, hl, lh, hh = _haar_2x2(a, b, c, d)
        g[..., 0::2, 0::2], g[..., 0::2, 1::2] = ll, hl
        g[..., 1::2, 0::2], g[..., 1::2, 1::2] = lh, hh
    return y


def haar_synthesis(w: np.ndarray, levels: int) -> np.ndarray:
    """W^T w: inverse of haar_analysis (coarsest level first)."""
    y = np.array(w, dtype=np.float64, copy=True)
    for lev in reversed(range(levels)):
        s = 2 ** lev
        g = y[..., ::s, ::s]
        ll, hl = g[..., 0::2, 0::2].copy(), g[..., 0::2, 1::2].copy()
        lh, hh = g[..., 1::2, 0::2].copy(), g[..., 1::2, 1::2].copy()
        a, b, c, d = _haar_2x2(ll, hl, lh, hh)
        g[..., 0::2, 0::2], g[..., 0::2, 1::2] = a, b
        g[..., 1::2, 0::2], g[..., 1::2, 1::2] = c, d
    return y


# --------------------------------------------------------------------------
# Daubechies-4 wavelets (8 taps, 4 vanishing moments), periodised, in the
# quadrant (Mallat) layout: level j works on the top-left (n/2^j) x (n/2^j)
# band, rows then columns, leaving [LL | HL ; LH | HH] there.

def daubechies_filter(p: int = 4) -> np.ndarray:
    """The minimum-phase Daubechies scaling filter with p vanishing moments
    (2p taps), by spectral factorisation: |H|^2 = 2 cos^{2p}(w/2) Q(sin^2(w/2))
    with Q(y) = sum_{k<p} C(p-1+k, k) y^k; each root y of Q gives the pair
    z, 1/z of z^2 - (2 - 4y) z + 1 = 0, and the root inside the unit circle is
    kept; h(z) is proportional to (z + 1)^p prod (z - z_j), normalised to a
    sum of sqrt(2) (coefficients from the highest power down)."""
    from math import comb
    q = [comb(p - 1 + k, k) for k in range(p)]
    zs = []
    for y in np.roots(q[::-1]):
        b = 1.0 - 2.0 * y
        disc = np.sqrt(b * b - 1.0 + 0j)
        z1, z2 = b + disc, b - disc
        zs.append(z1 if abs(z1) < 1.0 else z2)
    poly = np.array([1.0 + 0j])
    for _ in range(p):
        poly = np.convolve(poly, [1.0, 1.0])
    for z in zs:
        poly = np.convolve(poly, [1.0, -z])
    h = np.real(poly)
    return h * (np.sqrt(2.0) / h.sum())


def _qmf(h):
    """Wavelet filter g_k = (-1)^k h_{L-1-k}."""
    L = len(h)
    return np.array([(-1) ** k * h[L - 1 - k] for k in range(L)])


def _dwt1_matrix(m: int, h) -> np.ndarray:
    """The m x m periodised one-level analysis: rows i < m/2 give
    a_i = sum_k h_k x[(2i + k) mod m], rows m/2 + i give d_i with g."""
    g = _qmf(h)
    W = np.zeros((m, m))
    for i in range(m // 2):
        for k in range(len(h)):
            W[i, (2 * i + k) % m] += h[k]
            W[m // 2 + i, (2 * i + k) % m] += g[k]
    return W


def db4_analysis(x: np.ndarray, levels: int) -> np.ndarray:
    """W x: `levels` levels of the 2-D periodised Daubechies-4 transform."""
    h = daubechies_filter(4)
    y = np.array(x, dtype=np.float64, copy=True)
    m1, m2 = y.shape[-2], y.shape[-1]
    for _ in range(levels):
        Wr, Wc = _dwt1_matrix(m2, h), _dwt1_matrix(m1, h)
        band = y[..., :m1, :m2]
        y[..., :m1, :m2] = Wc @ (band @ Wr.T)
        m1, m2 = m1 // 2, m2 // 2
    return y


def db4_synthesis(w: np.ndarray, levels: int) -> np.ndarray:
    """W^T w: the inverse of db4_analysis (coarsest level first)."""
    h = daubechies_filter(4)
    y = np.array(w, dtype=np.float64, copy=True)
    n1, n2 = y.shape[-2], y.shape[-1]
    for lev in reversed(range(levels)):
        m1, m2 = n1 >> lev, n2 >> lev
        Wr, Wc = _dwt1_matrix(m2, h), _dwt1_matrix(m1, h)
        band = y[..., :m1, :m2]
        y[..., :m1, :m2] = Wc.T @ (band @ Wr)
    return y


def wavelet_analysis(x, levels, kind="haar"):
    return haar_analysis(x, levels) if kind == "haar" else db4_analysis(x, levels)


def wavelet_synthesis(w, levels, kind="haar"):
    return haar_synthesis(w, levels) if kind == "haar" else db4_synthesis(w, levels)


# --------------------------------------------------------------------------
# parallel-beam Joseph projector

def _joseph_view(n: int, n_bins: int, theta: float):
    """Sample positions of every ray of one view.

    Returns (row_idx, col_idx_lo, weight_hi, scale, along_rows) where for a
    ray/step pair the sample is (1 - w) X[lo] + w X[lo + 1] along the
    interpolation axis, arrays shaped (n_bins, n).
    """
    c = (n - 1) / 2.0
    s = np.arange(n_bins, dtype=np.float64) - (n_bins - 1) / 2.0
    t = np.arange(n, dtype=np.float64) - c      # coordinate of the stepped axis
    ct, st = np.cos(theta), np.sin(theta)
    if abs(ct) >= abs(st):
        # step over rows (y = t), interpolate along x
        f = (s[:, None] - t[None, :] * st) / ct + c
        scale = 1.0 / abs(ct)
        along_rows = True
    else:
        # step over columns (x = t), interpolate along y
        f = (s[:, None] - t[None, :] * ct) / st + c
        scale = 1.0 / abs(st)
        along_rows = False
    lo = np.floor(f).astype(np.int64)
    w = f - lo
    return lo, w, scale, along_rows


def joseph(x: np.ndarray, n_views: int, n_bins: int) -> np.ndarray:
    """Projection of an n x n image (or a stack) to (..., n_views, n_bins)."""
    n = x.shape[-1]
    lead = x.shape[:-2]
    xs = x.reshape((-1, n, n))
    out = np.zeros((xs.shape[0], n_views, n_bins))
    step = np.broadcast_to(np.arange(n)[None, :], (n_bins, n))
    for v in range(n_views):
        lo, w, scale, along_rows = _joseph_view(n, n_bins, np.pi * v / n_views)
        for q, wq in ((lo, 1.0 - w), (lo + 1, w)):
            ok = (q >= 0) & (q < n)
            qc = np.clip(q, 0, n - 1)
            if along_rows:
                vals = xs[:, step, qc]          # X[row = step, col = q]
            else:
                vals = xs[:, qc, step]          # X[row = q, col = step]
            out[:, v, :] += scale * np.sum(np.where(ok, wq * vals, 0.0), axis=-1)
    return out.reshape(lead + (n_views, n_bins))


def joseph_adjoint(p: np.ndarray, n: int) -> np.ndarray:
    """Transpose of `joseph`: the same sampling loop, scattering instead."""
    n_views, n_bins = p.shape[-2:]
    lead = p.shape[:-2]
    ps = p.reshape((-1, n_views, n_bins))
    out = np.zeros((ps.shape[0], n * n))
    step = np.broadcast_to(np.arange(n)[None, :], (n_bins, n))
    for v in range(n_views):
        lo, w, scale, along_rows = _joseph_view(n, n_bins, np.pi * v / n_views)
        for q, wq in ((lo, 1.0 - w), (lo + 1, w)):
            ok = (q >= 0) & (q < n)
            if along_rows:
                flat = step * n + q
            else:
                flat = q * n + step
            idx = flat[ok]
            for m in range(ps.shape[0]):
                contrib = (scale * wq * ps[m, v, :, None])[ok]
                out[m] += np.bincount(idx, weights=contrib, minlength=n * n)
    return out.reshape(lead + (n, n))


# --------------------------------------------------------------------------
# fan-beam Joseph projector (flat detector)
#
# View v at theta = 2 pi v / V: central ray direction d0 = (-sin, cos), source
# S = -R_s d0, a flat detector through R_d d0 along e = (cos, sin), bin b at
# u = (b - (B-1)/2) du.  Every ray is a line n . p = s with the unit normal n
# proportional to (R_s + R_d) e - u d0 and s = n . S = u R_s / sqrt((R_s +
# R_d)^2 + u^2); Joseph's sampling of the parallel-beam projector applies to
# it with (cos, sin) = n.  As R_s -> inf (R_d fixed) n -> e and s -> u: the
# parallel-beam projector with the detector coordinate u.

def fan_rays(n_views: int, n_bins: int, src: float, det: float, du: float):
    """Per-ray normals and offsets, arrays (n_views, n_bins): cos, sin, s."""
    th = 2.0 * np.pi * np.arange(n_views, dtype=np.float64) / n_views
    u = (np.arange(n_bins, dtype=np.float64) - (n_bins - 1) / 2.0) * du
    e = np.stack([np.cos(th), np.sin(th)], axis=-1)            # (V, 2)
    d0 = np.stack([-np.sin(th), np.cos(th)], axis=-1)
    nv = (src + det) * e[:, None, :] - u[None, :, None] * d0[:, None, :]
    nrm = np.sqrt((src + det) ** 2 + u * u)[None, :]
    cs, sn = nv[..., 0] / nrm, nv[..., 1] / nrm
    s = (u * src)[None, :] / nrm
    return cs, sn, np.broadcast_to(s, cs.shape).copy()


def _joseph_rays(n: int, cs, sn, s):
    """Joseph samples of arbitrary lines n . p = s (1-D arrays of rays):
    (lo, w, scale, along_rows) per ray, lo / w shaped (rays, n)."""
    c = (n - 1) / 2.0
    t = np.arange(n, dtype=np.float64) - c
    rows = np.abs(cs) >= np.abs(sn)
    a = np.where(rows, cs, sn)
    b = np.where(rows, sn, cs)
    f = (s[:, None] - t[None, :] * b[:, None]) / a[:, None] + c
    lo = np.floor(f).astype(np.int64)
    return lo, f - lo, 1.0 / np.abs(a), rows


def fan_joseph(x: np.ndarray, n_views: int, n_bins: int, src: float, det: float,
               du: float) -> np.ndarray:
    """Fan-beam projection of an n x n image (or a stack) to (..., V, B)."""
    n = x.shape[-1]
    lead = x.shape[:-2]
    xs = x.reshape((-1, n, n))
    cs, sn, s = fan_rays(n_views, n_bins, src, det, du)
    out = np.zeros((xs.shape[0], n_views, n_bins))
    step = np.broadcast_to(np.arange(n)[None, :], (n_bins, n))
    for v in range(n_views):
        lo, w, scale, rows = _joseph_rays(n, cs[v], sn[v], s[v])
        for q, wq in ((lo, 1.0 - w), (lo + 1, w)):
            ok = (q >= 0) & (q < n)
            qc = np.clip(q, 0, n - 1)
            r = np.where(rows[:, None], step, qc)
            col = np.where(rows[:, None], qc, step)
            vals = xs[:, r, col]
            out[:, v, :] += scale * np.sum(np.where(ok, wq * vals, 0.0), axis=-1)
    return out.reshape(lead + (n_views, n_bins))


def fan_joseph_adjoint(p: np.ndarray, n: int, src: float, det: float, du: float) -> np.ndarray:
    """Transpose of `fan_joseph`: the same samples, scattered."""
    n_views, n_bins = p.shape[-2:]
    lead = p.shape[:-2]
    ps = p.reshape((-1, n_views, n_bins))
    cs, sn, s = fan_rays(n_views, n_bins, src, det, du)
    out = np.zeros((ps.shape[0], n * n))
    step = np.broadcast_to(np.arange(n)[None, :], (n_bins, n))
    for v in range(n_views):
        lo, w, scale, rows = _joseph_rays(n, cs[v], sn[v], s[v])
        for q, wq in ((lo, 1.0 - w), (lo + 1, w)):
            ok = (q >= 0) & (q < n)
            flat = np.where(rows[:, None], step * n + q, q * n + step)
            idx = flat[ok]
            for m in range(ps.shape[0]):
                contrib = (scale[:, None] * wq * ps[m, v, :, None])[ok]
                out[m] += np.bincount(idx, weights=contrib, minlength=n * n)
    return out.reshape(lead + (n, n))


# --------------------------------------------------------------------------
# regularisation operators (App. A)

def grad(x: np.ndarray) -> np.ndarray:
    """First-order differences v_l = (X[i,j]-X[i-1,j], X[i,j]-X[i,j-1]).

    Reading of the boundary: the difference is 0 on the first row (first
    component) and on the first column (second component).
    Output shape (..., 2, n1, n2).
    """
    d1 = np.zeros_like(x, dtype=np.float64)
    d2 = np.zeros_like(x, dtype=np.float64)
    d1[..., 1:, :] = x[..., 1:, :] - x[..., :-1, :]
    d2[..., :, 1:] = x[..., :, 1:] - x[..., :, :-1]
    return np.stack([d1, d2], axis=-3)


def grad_adjoint(q: np.ndarray) -> np.ndarray:
    """Adjoint of `grad`, written as the literal transpose of its loops."""
    q1, q2 = q[..., 0, :, :], q[..., 1, :, :]
    out = np.zeros(q1.shape)
    # d1[i] = x[i] - x[i-1] for i >= 1
    out[..., 1:, :] += q1[..., 1:, :]
    out[..., :-1, :] -= q1[..., 1:, :]
    out[..., :, 1:] += q2[..., :, 1:]
    out[..., :, :-1] -= q2[..., :, 1:]
    return out


def _rep(x, di, dj):
    """X[i + di, j + dj] with replicate padding."""
    n1, n2 = x.shape[-2:]
    i = np.clip(np.arange(n1) + di, 0, n1 - 1)
    j = np.clip(np.arange(n2) + dj, 0, n2 - 1)
    return x[..., i, :][..., :, j]


def hessian(x: np.ndarray) -> np.ndarray:
    """Second-order differences (v11, v22, v12) of App. A, replicate padding.

    v11 = X[i-1,j] - 2X[i,j] + X[i+1,j]
    v22 = X[i,j-1] - 2X[i,j] + X[i,j+1]
    v12 = v21 = (X[i+1,j+1] - X[i+1,j-1] - X[i-1,j+1] + X[i-1,j-1]) / 4
    Output shape (..., 3, n1, n2).
    """
    v11 = _rep(x, -1, 0) - 2 * x + _rep(x, 1, 0)
    v22 = _rep(x, 0, -1) - 2 * x + _rep(x, 0, 1)
    v12 = (_rep(x, 1, 1) - _rep(x, 1, -1) - _rep(x, -1, 1) + _rep(x, -1, -1)) / 4
    return np.stack([v11, v22, v12], axis=-3)


def _rep_adjoint(q, di, dj):
    """Adjoint of q -> _rep(., di, dj): scatter-add to the clipped indices."""
    n1, n2 = q.shape[-2:]
    i = np.clip(np.arange(n1) + di, 0, n1 - 1)
    j = np.clip(np.arange(n2) + dj, 0, n2 - 1)
    tmp = np.zeros(q.shape)
    np.add.at(tmp, (Ellipsis, slice(None), j), q)
    out = np.zeros(q.shape)
    np.add.at(out, (Ellipsis, i, slice(None)), tmp)
    return out


def hessian_adjoint(q: np.ndarray) -> np.ndarray:
    """Adjoint of `hessian` for symmetric 2 x 2 groups in the Frobenius
    pairing <Q, V> = q11 v11 + q22 v22 + 2 q12 v12 (v12 = v21 counted twice)."""
    q11, q22, q12 = q[..., 0, :, :], q[..., 1, :, :], q[..., 2, :, :]
    out = (_rep_adjoint(q11, -1, 0) - 2 * q11 + _rep_adjoint(q11, 1, 0)
           + _rep_adjoint(q22, 0, -1) - 2 * q22 + _rep_adjoint(q22, 0, 1))
    out += 2 * (_rep_adjoint(q12, 1, 1) - _rep_adjoint(q12, 1, -1)
                - _rep_adjoint(q12, -1, 1) + _rep_adjoint(q12, -1, -1)) / 4
    return out


def pair(q: np.ndarray, v: np.ndarray, reg: str) -> float:
    """Dual pairing <Q, V> used by the adjoints above."""
    if reg in ("hs1", "hs2", "hsinf"):
        return float(np.sum(q[..., 0, :, :] * v[..., 0, :, :])
                     + np.sum(q[..., 1, :, :] * v[..., 1, :, :])
                     + 2 * np.sum(q[..., 2, :, :] * v[..., 2, :, :]))
    return float(np.sum(q * v))
