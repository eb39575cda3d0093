"""GPU parity of the operators and of the sketch against the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import operators as ops
from oracle import solver as sv
from gpu_util import BF16_ELEM, TOL, banner, check, dev, host, need_gpu, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n1,n2,k,sigma", [(100, 72, 9, 1.5), (128, 128, 9, 1.5),
                                           (33, 47, 15, 3.0), (16, 16, 5, 0.8)])
def test_blur_forward_adjoint(dt, n1, n2, k, sigma):
    P = need_gpu()
    banner(f"blur {dt} {n1}x{n2} k={k}")
    h = W.gaussian_psf(k, sigma)
    h[0, 1] += 0.01            # break the symmetry so H != H^T is exercised
    op = P.Operator(P.OP_BLUR, n1, n2, psf=h)
    x = W.gaussian((3, n1, n2), 1)
    xd = dev(x, dt)
    xr = host(xd)
    y = P.op_forward(op, xd)
    check(host(y), ops.blur(xr, h), TOL[dt])
    z = P.op_adjoint(op, y)
    check(host(z), ops.blur_adjoint(host(y), h), TOL[dt])


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n,k,levels", [(512, 7, 0), (96, 7, 3), (40, 5, 0), (64, 9, 3)])
def test_blurdown_and_haar(dt, n, k, levels):
    P = need_gpu()
    banner(f"blurdown {dt} n={n} k={k} levels={levels}")
    h = W.gaussian_psf(k, 1.2)
    op = P.Operator(P.OP_BLURDOWN, n, n, psf=h, factor=2, wavelet_levels=levels)
    x = W.gaussian((2, n, n), 2)
    xd = dev(x, dt)
    xr = host(xd)
    ref = ops.blurdown(ops.haar_synthesis(xr, levels) if levels else xr, h, 2)
    y = P.op_forward(op, xd)
    assert y.shape == (2, n // 2, n // 2)
    check(host(y), ref, TOL[dt])
    yr = host(y)
    ref_t = ops.blurdown_adjoint(yr, h, 2)
    if levels:
        ref_t = ops.haar_analysis(ref_t, levels)
    check(host(P.op_adjoint(op, y)), ref_t, TOL[dt])


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_haar_identity_operator(dt):
    P = need_gpu()
    banner(f"haar identity {dt}")
    n = 48
    op = P.Operator(P.OP_IDENTITY, n, n, wavelet_levels=3)
    w = W.gaussian((2, n, n), 3)
    wd = dev(w, dt)
    check(host(P.op_forward(op, wd)), ops.haar_synthesis(host(wd), 3), TOL[dt])
    check(host(P.op_adjoint(op, wd)), ops.haar_analysis(host(wd), 3), TOL[dt])


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n1,n2,levels", [(64, 64, 4), (96, 48, 3), (32, 32, 5), (16, 16, 1)])
def test_db4_identity_operator(dt, n1, n2, levels):
    """Periodised Daubechies-4 (the CT experiments' daub4): W^T and W against
    the oracle's transform, down to bands narrower than the filter."""
    P = need_gpu()
    banner(f"db4 identity {dt} {n1}x{n2} levels={levels}")
    op = P.Operator(P.OP_IDENTITY, n1, n2, wavelet_levels=levels, wavelet="db4")
    w = W.gaussian((2, n1, n2), 33)
    wd = dev(w, dt)
    check(host(P.op_forward(op, wd)), ops.db4_synthesis(host(wd), levels), TOL[dt])
    check(host(P.op_adjoint(op, wd)), ops.db4_analysis(host(wd), levels), TOL[dt])


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_blurdown_db4_operator_and_sketch(dt):
    P = need_gpu()
    banner(f"blurdown db4 {dt}")
    n, k, levels = 64, 7, 4
    h = W.gaussian_psf(k, 1.2)
    op = P.Operator(P.OP_BLURDOWN, n, n, psf=h, factor=2, wavelet_levels=levels, wavelet="db4")
    prob = sv.Problem("blurdown", n, None, 0.0, "l1", h=h, factor=2, levels=levels, wavelet="db4")
    if dt != "bf16":
        xd = dev(W.gaussian((2, n, n), 34), dt)
        y = P.op_forward(op, xd)
        check(host(y), ops.blurdown(ops.db4_synthesis(host(xd), levels), h, 2), TOL[dt])
        z = P.op_adjoint(op, y)
        check(host(z), ops.db4_analysis(ops.blurdown_adjoint(host(y), h, 2), levels), TOL[dt])
    om = dev(W.omega(3, n, n, 35), dt)
    Y = P.nys_sketch(op, om)
    check(host(Y), sv.sketch(prob, host(om)), TOL[dt], BF16_ELEM if dt == "bf16" else None)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n,V,B", [(32, 24, 45), (64, 90, 92), (47, 13, 70)])
def test_joseph_pair(dt, n, V, B):
    P = need_gpu()
    banner(f"joseph {dt} n={n} V={V} B={B}")
    op = P.Operator(P.OP_PARALLEL_BEAM, n, n, views=V, bins=B)
    x = W.gaussian((2, n, n), 4)
    xd = dev(x, dt)
    p = P.op_forward(op, xd)
    assert p.shape == (2, V, B)
    check(host(p), ops.joseph(host(xd), V, B), TOL[dt])
    q = dev(W.gaussian((2, V, B), 5), dt)
    check(host(P.op_adjoint(op, q)), ops.joseph_adjoint(host(q), n), TOL[dt])
    # adjoint identity inside the GPU arithmetic
    lhs = float((p.double() * q.double()).sum())
    rhs = float((xd.double() * P.op_adjoint(op, q).double()).sum())
    assert abs(lhs - rhs) <= 10 * TOL[dt] * abs(lhs)


@pytest.mark.parametrize("dt,n,ell", [("f64", 128, 32), ("f64", 40, 7), ("f32", 100, 5)])
def test_sketch_blur(dt, n, ell):
    P = need_gpu()
    banner(f"sketch blur {dt} n={n} ell={ell}")
    h = W.gaussian_psf(9, 1.5)
    op = P.Operator(P.OP_BLUR, n, n, psf=h)
    om = dev(W.omega(ell, n, n, 6), dt)
    Y = P.nys_sketch(op, om)
    prob = sv.Problem("blur", n, None, 0.0, "tv", h=h)
    check(host(Y), sv.sketch(prob, host(om)), TOL[dt], BF16_ELEM if dt == "bf16" else None)


@pytest.mark.parametrize("dt,n,ell,k,sep", [("bf16", 128, 5, 7, True), ("f32", 128, 3, 7, True),
                                             ("bf16", 96, 4, 7, True), ("f32", 72, 2, 7, True),
                                             ("bf16", 192, 3, 9, True), ("f32", 64, 2, 5, True),
                                             ("f32", 128, 2, 3, True), ("f32", 128, 2, 7, False),
                                             ("bf16", 64, 3, 9, False)])
def test_sketch_super_resolution(dt, n, ell, k, sep):
    """Fused separable path for n divisible by 64 and a rank-1 PSF, fused 2-D
    path for other PSFs, unfused chain otherwise."""
    P = need_gpu()
    banner(f"sketch SR {dt} n={n} ell={ell} k={k} sep={sep}")
    h = W.gaussian_psf(k, 1.2)
    if not sep:
        h = h + 0.02 * W.gaussian((k, k), 30)      # rank > 1
    op = P.Operator(P.OP_BLURDOWN, n, n, psf=h, factor=2, wavelet_levels=3)
    om = dev(W.omega(ell, n, n, 7), dt)
    Y = P.nys_sketch(op, om)
    prob = sv.Problem("blurdown", n, None, 0.0, "l1", h=h, factor=2, levels=3)
    ref = sv.sketch(prob, host(om))
    got = host(Y)
    check(got, ref, TOL[dt], BF16_ELEM if dt == "bf16" else None)
    # element-wise: within one bf16 ulp (2^-8 relative) plus FP32 accumulation
    if dt == "bf16":
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


def test_joseph_full_size_ct_f32():
    """512^2 image, 720 views x 736 bins (the CT workload's launch shape):
    forward and adjoint against the oracle on a phantom and a sinogram."""
    P = need_gpu()
    banner("joseph full size 512^2 720x736 f32")
    n, V, B = 512, 720, 736
    op = P.Operator(P.OP_PARALLEL_BEAM, n, n, views=V, bins=B)
    xd = dev(W.phantom_ellipses(n, 11), "f32")
    p = P.op_forward(op, xd)
    check(host(p), ops.joseph(host(xd), V, B), TOL["f32"])
    q = dev(W.gaussian((V, B), 12), "f32")
    check(host(P.op_adjoint(op, q)), ops.joseph_adjoint(host(q), n), TOL["f32"])


@pytest.mark.parametrize("n,V,B,cols", [(64, 90, 92, 36), (8, 10, 300, 1), (1004, 6, 1424, 1)])
def test_joseph_forward_launch_forms_f32(n, V, B, cols):
    """The FP32 forward without the split of its steps (enough workgroups to
    fill the chip), with workgroups whose bins all miss the image (the
    image's shadow is narrower than the detector), and on a large image."""
    P = need_gpu()
    banner(f"joseph forward forms f32 n={n} V={V} B={B} cols={cols}")
    op = P.Operator(P.OP_PARALLEL_BEAM, n, n, views=V, bins=B)
    xd = dev(W.gaussian((cols, n, n), 13), "f32")
    check(host(P.op_forward(op, xd)), ops.joseph(host(xd), V, B), TOL["f32"])


def test_sketch_ct_f32():
    P = need_gpu()
    banner("sketch CT f32")
    n, V, B, ell = 48, 30, 70, 3
    op = P.Operator(P.OP_PARALLEL_BEAM, n, n, views=V, bins=B)
    om = dev(W.omega(ell, n, n, 8), "f32")
    Y = P.nys_sketch(op, om)
    ref = ops.joseph_adjoint(ops.joseph(host(om), V, B), n)
    check(host(Y), ref, TOL["f32"])


# the last case has the source radius below the image side: its adjoint is
# the atomically scattered one, the others' the gathered one
FAN_CASES = [(32, 24, 45, (64.0, 32.0, 1.0)), (47, 13, 70, (90.0, 45.0, 1.3)),
             (64, 36, 92, (128.0, 64.0, 1.5)), (32, 20, 50, (30.0, 10.0, 1.0))]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n,V,B,geo", FAN_CASES)
def test_fan_pair(dt, n, V, B, geo):
    """Fan-beam Joseph projector (views over 360 degrees, flat detector) and
    its transpose (gathered per pixel, or scattered per ray) against the
    oracle."""
    P = need_gpu()
    banner(f"fan {dt} n={n} V={V} B={B} geo={geo}")
    op = P.Operator(P.OP_FAN_BEAM, n, n, views=V, bins=B, fan=geo)
    x = W.gaussian((2, n, n), 4)
    xd = dev(x, dt)
    p = P.op_forward(op, xd)
    assert p.shape == (2, V, B)
    check(host(p), ops.fan_joseph(host(xd), V, B, *geo), TOL[dt])
    q = dev(W.gaussian((2, V, B), 5), dt)
    z = P.op_adjoint(op, q)
    check(host(z), ops.fan_joseph_adjoint(host(q), n, *geo), TOL[dt])
    lhs = float((p.double() * q.double()).sum())
    rhs = float((xd.double() * z.double()).sum())
    assert abs(lhs - rhs) <= 10 * TOL[dt] * abs(lhs)


def test_fan_full_size_f32():
    """The paper's fan-beam acquisition: 512^2 image, 100 views over 360
    degrees, 1024 detector bins (source and detector radii 1024 and 512
    pixels, bins 1.5 pixels apart), forward and adjoint against the oracle."""
    P = need_gpu()
    banner("fan full size 512^2 100x1024 f32")
    n, V, B, geo = 512, 100, 1024, (1024.0, 512.0, 1.5)
    op = P.Operator(P.OP_FAN_BEAM, n, n, views=V, bins=B, fan=geo)
    xd = dev(W.phantom_ellipses(n, 11), "f32")
    p = P.op_forward(op, xd)
    check(host(p), ops.fan_joseph(host(xd), V, B, *geo), TOL["f32"])
    q = dev(W.gaussian((V, B), 12), "f32")
    check(host(P.op_adjoint(op, q)), ops.fan_joseph_adjoint(host(q), n, *geo), TOL["f32"])


@pytest.mark.parametrize("wavelet,levels", [("haar", 2), ("db4", 3)])
def test_fan_in_wavelet_coordinates(wavelet, levels):
    """A W^T with the fan-beam projector (the CT experiments' wavelet prior in
    coefficient coordinates), forward and adjoint against the oracle, FP64."""
    P = need_gpu()
    banner(f"fan {wavelet}-{levels}")
    n, V, B, geo = 48, 20, 72, (96.0, 48.0, 1.2)
    op = P.Operator(P.OP_FAN_BEAM, n, n, views=V, bins=B, fan=geo, wavelet_levels=levels,
                    wavelet=wavelet)
    prob = sv.Problem("fan", n, None, 0.0, "l1", views=V, bins=B, levels=levels,
                      wavelet=wavelet, fan=geo)
    xd = dev(W.gaussian((n, n), 40), "f64")
    check(host(P.op_forward(op, xd)), prob.A(host(xd)), TOL["f64"])
    q = dev(W.gaussian((V, B), 41), "f64")
    check(host(P.op_adjoint(op, q)), prob.At(host(q)), TOL["f64"])


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_sketch_fan(dt):
    P = need_gpu()
    banner(f"sketch fan {dt}")
    n, V, B, ell, geo = 48, 30, 70, 3, (96.0, 48.0, 1.2)
    op = P.Operator(P.OP_FAN_BEAM, n, n, views=V, bins=B, fan=geo)
    om = dev(W.omega(ell, n, n, 8), dt)
    Y = P.nys_sketch(op, om)
    ref = ops.fan_joseph_adjoint(ops.fan_joseph(host(om), V, B, *geo), n, *geo)
    check(host(Y), ref, TOL[dt], BF16_ELEM if dt == "bf16" else None)


def test_sketch_sr_full_size_sampled_columns():
    """512^2 super-resolution workload, ell = 64, BF16: the timed launch
    configuration; the oracle checks 3 sampled columns."""
    P = need_gpu()
    banner("sketch SR full size 512^2 ell=64 bf16")
    wl = W.workload("sr512_haar_bf16")
    n, ell = wl.n, wl.ell
    h = W.gaussian_psf(wl.psf_k, wl.psf_sigma)
    op = P.Operator(P.OP_BLURDOWN, n, n, psf=h, factor=2, wavelet_levels=3)
    om = dev(W.omega(ell, n, n, 0), "bf16")
    Y = P.nys_sketch(op, om)
    prob = sv.Problem("blurdown", n, None, 0.0, "l1", h=h, factor=2, levels=3)
    omh = host(om)
    for k in (0, 31, 63):
        ref = prob.phi(omh[k])
        got = host(Y[k])
        check(got, ref, TOL["bf16"], BF16_ELEM, what=f"column {k}")


def test_operator_argument_errors():
    P = need_gpu()
    with pytest.raises(P.NysError):
        P.Operator(P.OP_BLUR, 16, 16, psf=np.ones((4, 4)) / 16)       # even PSF
    with pytest.raises(P.NysError):
        P.Operator(P.OP_BLURDOWN, 15, 16, psf=np.ones((3, 3)) / 9, factor=2)
    with pytest.raises(P.NysError):
        P.Operator(P.OP_PARALLEL_BEAM, 16, 12, views=4, bins=5)
    with pytest.raises(P.NysError):
        P.Operator(P.OP_FAN_BEAM, 16, 16, views=4, bins=5, fan=(0.0, 8.0, 1.0))   # no source radius
