"""GPU parity of the Nystrom factorisation, P^{-1}, the weighted prox and
WAPG against the FP64 oracle (inputs fed identically to both sides)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import nystrom as onys
from oracle import operators as ops
from oracle import prox as opx
from oracle import solver as sv
from gpu_util import BF16_ELEM, TOL, banner, check, dev, host, need_gpu, rel

pytestmark = pytest.mark.gpu


def _blur_case(n, ell, seed=0, k=9, sigma=1.5):
    h = W.gaussian_psf(k, sigma)
    prob = sv.Problem("blur", n, None, 0.0, "tv", h=h)
    om = W.omega(ell, n, n, seed)
    Y = sv.sketch(prob, om)
    return prob, om, Y


def _ct_case(n, V, B, ell, seed=0):
    prob = sv.Problem("ct", n, None, 0.0, "hs1", views=V, bins=B)
    om = W.omega(ell, n, n, seed)
    Y = sv.sketch(prob, om)
    return prob, om, Y


@pytest.mark.parametrize("case,dt,tail", [("blur", "f64", "sqrt"), ("blur", "f64", "plain"),
                                          ("ct", "f32", "sqrt"), ("ct", "bf16", "plain")])
def test_factor_spectrum_and_pinv(case, dt, tail):
    P = need_gpu()
    banner(f"factor {case} {dt} {tail}")
    if case == "blur":
        prob, om, Y = _blur_case(40, 12)
    else:
        prob, om, Y = _ct_case(32, 40, 48, 10)
    ell, n = om.shape[0], om.shape[1]
    omd, Yd = dev(om, dt), dev(Y, dt)
    # the oracle sees exactly the rounded inputs
    omr, Yr = host(omd).reshape(ell, -1), host(Yd).reshape(ell, -1)
    ref = onys.nystrom(Yr, omr)
    udt = torch.float64 if dt == "f64" else torch.float32
    pc = P.nys_factor(omd, Yd, ell, tail=tail, u_dtype=udt)
    info = pc.info()
    assert info["status"] == 0
    k = len(ref["shat"])
    tol = TOL["f64"] if dt == "f64" else 1e-5
    # nu comes from ||Y||_2 of the Gram; FP32/BF16 inputs are accumulated in FP32
    assert abs(info["nu"] - ref["nu"]) <= (1e-10 if dt == "f64" else 1e-5) * ref["nu"]
    check(info["shat"][:k], ref["shat"], tol, what="shat")
    # P^{-1} v and P v on probes (U itself is not unique)
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], tail)
    v = W.gaussian((3, n * n), 11)
    vd = dev(v, "f64" if dt == "f64" else "f32")
    got = host(P.nys_apply(pc, vd, inverse=True))
    want = np.stack([opc.pinv(host(vd)[c]) for c in range(3)])
    check(got, want, tol, what="P^-1 v")
    got_p = host(P.nys_apply(pc, vd, inverse=False))
    want_p = np.stack([opc.p(host(vd)[c]) for c in range(3)])
    check(got_p, want_p, tol, what="P v")
    # U U^T on probes
    U = host(pc.U()).reshape(ell, -1)
    proj = (host(vd) @ U.T) @ U
    proj_ref = (host(vd) @ ref["U"].T) @ ref["U"]
    check(proj, proj_ref, tol, what="U U^T v")
    # orthonormal columns
    assert np.allclose(U @ U.T, np.eye(ell), atol=(1e-10 if dt == "f64" else 2e-5))


def _steep_psd_sketch(n, ell, r=150, seed=0):
    """Y = Phi Omega for Phi = Q diag(lam) Q^T + c I (Q: N x r orthonormal),
    exactly in FP64: a PSD operator whose top spectrum decays like the CT
    normal operator's (lam_i = 1e4 / (i + 1)^2, c = 0.05), at any image size."""
    N = n * n
    Q, _ = np.linalg.qr(W.gaussian((N, r), seed + 1))
    lam = 1e4 / (np.arange(r) + 1.0) ** 2
    om = W.omega(ell, n, n, seed + 2).reshape(ell, N)
    Y = ((om @ Q) * lam) @ Q.T + 0.05 * om
    return om, Y


# the timed factorisation paths: BF16 Omega and Y through the BF16 MFMA Gram
# with several 32 x 32 tile rows (ell = 64: 4, ell = 100: 7), at N >= 128^2;
# the 512^2 super-resolution sketch at its own ell = 64; a steep spectrum
@pytest.mark.parametrize("case,ell", [("blur128", 64), ("blur128", 100), ("sr512", 64),
                                      ("steep128", 100)])
def test_factor_bf16_multi_tile(case, ell):
    P = need_gpu()
    banner(f"factor bf16 {case} ell={ell}")
    if case == "blur128":
        n = 128
        prob = sv.Problem("blur", n, None, 0.0, "tv", h=W.gaussian_psf(9, 1.5))
        om = W.omega(ell, n, n, 50)
        omd = dev(om, "bf16")
        Yd = dev(sv.sketch(prob, host(omd)), "bf16")
    elif case == "sr512":
        wl = W.workload("sr512_haar_bf16")
        n = wl.n
        h = W.gaussian_psf(wl.psf_k, wl.psf_sigma)
        prob = sv.Problem("blurdown", n, None, 0.0, "l1", h=h, factor=2, levels=3)
        omd = dev(W.omega(ell, n, n, 51), "bf16")
        Yd = dev(sv.sketch(prob, host(omd)), "bf16")
    else:
        n = 128
        om, Y = _steep_psd_sketch(n, ell, seed=52)
        omd, Yd = dev(om.reshape(ell, n, n), "bf16"), dev(Y.reshape(ell, n, n), "bf16")
    omr, Yr = host(omd).reshape(ell, -1), host(Yd).reshape(ell, -1)
    ref = onys.nystrom(Yr, omr)
    pc = P.nys_factor(omd, Yd, ell, u_dtype=torch.float32)
    info = pc.info()
    assert info["status"] == 0
    k = len(ref["shat"])
    tol = TOL["bf16"]
    assert abs(info["nu"] - ref["nu"]) <= 1e-5 * ref["nu"]
    check(info["shat"][:k], ref["shat"], tol, BF16_ELEM, what="shat")
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    v = W.gaussian((2, n * n), 53)
    vd = dev(v, "f32")
    vh = host(vd)
    check(host(P.nys_apply(pc, vd, inverse=True)), np.stack([opc.pinv(r) for r in vh]), tol,
          BF16_ELEM, what="P^-1 v")
    check(host(P.nys_apply(pc, vd, inverse=False)), np.stack([opc.p(r) for r in vh]), tol,
          BF16_ELEM, what="P v")


def test_ct_configuration_pinv_and_hs1_prox():
    """The CT workload's shapes: 512^2 unknowns, ell = 100, FP32 U (the P^{-1}
    kernels in 64 + 32 + 16-row pieces and the partial-sum tail), then the
    P-weighted HS1 prox with 20 dual iterations, against the oracle on the
    same rounded inputs.  Phi has a steep top spectrum like the CT normal
    operator's."""
    P = need_gpu()
    banner("CT configuration 512^2 ell=100: P^-1 and HS1 prox, f32")
    n, ell = 512, 100
    om, Y = _steep_psd_sketch(n, ell, seed=60)
    omd, Yd = dev(om.reshape(ell, n, n), "f32"), dev(Y.reshape(ell, n, n), "f32")
    ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
    pc = P.nys_factor(omd, Yd, ell, u_dtype=torch.float32)
    info = pc.info()
    assert info["status"] == 0
    check(info["shat"][:len(ref["shat"])], ref["shat"], TOL["f32"], what="shat")
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    vd = dev(W.gaussian((2, n, n), 61), "f32")
    vh = host(vd)
    check(host(P.nys_apply(pc, vd, inverse=True)), np.stack([opc.pinv(r) for r in vh]),
          TOL["f32"], what="P^-1 v")
    # s: the CT phantom family (values 0 - 0.04) plus noise at 5 % of its range;
    # lam_bar at the noise level keeps the dual ball constraints active
    s = W.phantom_ellipses(n, 62) + 0.002 * W.gaussian((n, n), 63)
    sd = dev(s, "f32")
    lam_bar = 1e-3
    rd = P.reg_desc("hs1", n, n, n_inner=20)
    state = P.prox_state(rd, pc, sd.dtype)
    x = P.prox_weighted(rd, lam_bar, pc, sd, state)
    xr, _ = opx.prox_mixed_dual(host(sd), lam_bar, "hs1", opc.pinv, opc.pinv_norm, 20)
    check(host(x), xr, TOL["f32"], what="HS1 prox")


@pytest.mark.parametrize("reg,ell", [("hs1", 100), ("hs1", 128), ("tv", 128)])
def test_fused_prox_rows_in_lds_and_read_again(reg, ell):
    """The fused dual iteration keeps 80 rows of U in registers, the next
    ones (about 20, as LDS allows at two workgroups per CU) in LDS, and reads
    any further ones again for the partials: ell = 100 takes registers and
    LDS, ell = 128 all three.  FP32 on ragged 48^2 tiles, the warm-started
    second call included, against the oracle."""
    P = need_gpu()
    banner(f"fused prox {reg} ell={ell}: rows in registers, LDS and read again")
    n = 48
    om, Y = _steep_psd_sketch(n, ell, r=ell + 40, seed=70)
    omd, Yd = dev(om.reshape(ell, n, n), "f32"), dev(Y.reshape(ell, n, n), "f32")
    ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
    pc = P.nys_factor(omd, Yd, ell, u_dtype=torch.float32)
    assert pc.info()["status"] == 0
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    s = W.phantom_ellipses(n, 72) + 0.002 * W.gaussian((n, n), 73)
    sd = dev(s, "f32")
    lam_bar = 1e-3
    rd = P.reg_desc(reg, n, n, n_inner=12)
    state = P.prox_state(rd, pc, sd.dtype)
    x = P.prox_weighted(rd, lam_bar, pc, sd, state)
    xr, Q = opx.prox_mixed_dual(host(sd), lam_bar, reg, opc.pinv, opc.pinv_norm, 12)
    check(host(x), xr, TOL["f32"], what=f"{reg} prox")
    x2 = P.prox_weighted(rd, lam_bar, pc, sd, state)
    xr2, _ = opx.prox_mixed_dual(host(sd), lam_bar, reg, opc.pinv, opc.pinv_norm, 12, q0=Q)
    check(host(x2), xr2, TOL["f32"], what=f"{reg} prox, warm start")


def test_factor_exact_recovery_low_rank():
    """Phi = G G^T of rank 5 < ell = 8: U S U^T reproduces Phi."""
    P = need_gpu()
    banner("factor exact low rank")
    N, ell, r = 300, 8, 5
    G = W.gaussian((N, r), 12)
    Phi = G @ G.T
    om = W.omega(ell, 1, N, 13).reshape(ell, N)
    Y = om @ Phi
    pc = P.nys_factor(dev(om), dev(Y), ell, u_dtype=torch.float64)
    info = pc.info()
    U = host(pc.U()).reshape(ell, N)
    k = info["k_eff"]
    approx = U[:r].T @ np.diag(info["shat"][:r]) @ U[:r]
    assert np.linalg.norm(approx - Phi) < 1e-9 * np.linalg.norm(Phi)
    assert np.allclose(info["shat"][:r], np.sort(np.linalg.eigvalsh(Phi))[::-1][:r], rtol=1e-9)
    assert k >= r


def test_factor_not_pd_is_reported():
    P = need_gpu()
    banner("factor not PD")
    N, ell = 64, 4
    om = W.omega(ell, 1, N, 14).reshape(ell, N)
    Y = -om * 3.0                         # Phi = -3 I: indefinite Gram
    pc = P.nys_factor(dev(om), dev(Y), ell, max_escalations=2, u_dtype=torch.float64)
    assert pc.info()["status"] == 3       # NYS_ENOTPD


@pytest.mark.parametrize("reg,dt,with_pc", [("tv", "f64", True), ("tv", "f64", False),
                                            ("hs1", "f64", True), ("tv_aniso", "f32", True),
                                            ("hs1", "f32", False), ("hs2", "f64", True),
                                            ("hs2", "f32", False), ("hsinf", "f64", True),
                                            ("hsinf", "f32", True)])
def test_prox_dual(reg, dt, with_pc):
    P = need_gpu()
    banner(f"prox dual {reg} {dt} pc={with_pc}")
    n1 = n2 = 37
    prob, om, Y = _blur_case(n1, 6)
    s = W.gaussian((n1, n2), 15)
    lam_bar = 0.05
    sd = dev(s, dt)
    if with_pc:
        omd, Yd = dev(om, "f64"), dev(Y, "f64")
        ref = onys.nystrom(host(Yd).reshape(6, -1), host(omd).reshape(6, -1))
        opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
        udt = torch.float64 if dt == "f64" else torch.float32
        pc = P.nys_factor(omd, Yd, 6, u_dtype=udt)
        pinv, pnorm = opc.pinv, opc.pinv_norm
    else:
        pc, pinv, pnorm = None, (lambda v: v), 1.0
    rd = P.reg_desc(reg, n1, n2, n_inner=25)
    state = P.prox_state(rd, pc, sd.dtype)
    x = P.prox_weighted(rd, lam_bar, pc, sd, state)
    xr, Q = opx.prox_mixed_dual(host(sd), lam_bar, reg, pinv, pnorm, 25)
    check(host(x), xr, TOL[dt])
    # warm start: a second call continues from the stored Q
    x2 = P.prox_weighted(rd, lam_bar, pc, sd, state)
    xr2, _ = opx.prox_mixed_dual(host(sd), lam_bar, reg, pinv, pnorm, 25, q0=Q)
    check(host(x2), xr2, TOL[dt], what="warm start")


@pytest.mark.parametrize("reg,dt,with_pc,box", [("tv", "f64", True, (0.0, np.inf)),
                                                ("tv", "f32", True, (0.0, np.inf)),
                                                ("hs1", "f64", True, (-0.2, 0.3)),
                                                ("tv", "f32", False, (-0.1, 0.4))])
def test_prox_dual_box(reg, dt, with_pc, box):
    """C = {lo <= x <= hi}: x(Q) = prox^P_{delta_C}(.) in every dual iteration
    (the P-weighted projection by the semismooth Newton method with the clip)."""
    P = need_gpu()
    banner(f"prox dual box {reg} {dt} pc={with_pc} box={box}")
    n1 = n2 = 29
    prob, om, Y = _blur_case(n1, 6)
    s = W.gaussian((n1, n2), 17) * 0.5
    lam_bar = 0.05
    sd = dev(s, dt)
    lo, hi = box
    if with_pc:
        omd, Yd = dev(om, "f64"), dev(Y, "f64")
        ref = onys.nystrom(host(Yd).reshape(6, -1), host(omd).reshape(6, -1))
        opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
        udt = torch.float64 if dt == "f64" else torch.float32
        pc = P.nys_factor(omd, Yd, 6, u_dtype=udt)
        pinv, pnorm = opc.pinv, opc.pinv_norm
        proj = lambda z: opx.prox_box_weighted(z.reshape(-1), lo, hi, opc.U, opc.e)[0].reshape(z.shape)
    else:
        pc, pinv, pnorm = None, (lambda v: v), 1.0
        proj = lambda z: np.clip(z, lo, hi)
    rd = P.reg_desc(reg, n1, n2, n_inner=25, box=box)
    state = P.prox_state(rd, pc, sd.dtype)
    x = P.prox_weighted(rd, lam_bar, pc, sd, state)
    xr, Q = opx.prox_mixed_dual(host(sd), lam_bar, reg, pinv, pnorm, 25, proj_c=proj)
    xh = host(x)
    assert xh.min() >= lo - 1e-6 and xh.max() <= hi + 1e-6
    check(xh, xr, TOL[dt])
    # the box is active: the unconstrained prox leaves it
    xu, _ = opx.prox_mixed_dual(host(sd), lam_bar, reg, pinv, pnorm, 25)
    assert xu.min() < lo - 1e-3 or xu.max() > hi + 1e-3


# ell = 8 and 40 / 64 take the register eliminations sized 32 and 64 (40: a
# ragged last group of columns), ell = 100 the elimination of the whole block;
# the plain tail gives e up to s_1 / s_ell - 1 >> 1, the sqrt tail e < 0
@pytest.mark.parametrize("dt,tail,ell", [("f64", "sqrt", 8), ("f64", "plain", 8), ("f32", "sqrt", 8),
                                         ("f32", "sqrt", 40), ("f32", "plain", 64),
                                         ("f32", "sqrt", 100), ("f64", "plain", 64)])
def test_prox_l1_ssn(dt, tail, ell):
    P = need_gpu()
    banner(f"prox l1 ssn {dt} {tail} ell={ell}")
    n = 48
    h = W.gaussian_psf(7, 1.2)
    prob = sv.Problem("blurdown", n, None, 0.0, "l1", h=h, factor=2, levels=3)
    om = W.omega(ell, n, n, 16)
    Y = sv.sketch(prob, om)
    omd, Yd = dev(om, "f64"), dev(Y, "f64")
    ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], tail)
    udt = torch.float64 if dt == "f64" else torch.float32
    pc = P.nys_factor(omd, Yd, ell, tail=tail, u_dtype=udt)
    s = W.gaussian((n, n), 17) * 0.1
    sd = dev(s, dt)
    lam_bar = 0.05
    rd = P.reg_desc("l1", n, n)
    state = P.prox_state(rd, pc, sd.dtype)
    x = P.prox_weighted(rd, lam_bar, pc, sd, state)
    xr, g, _ = opx.prox_l1_weighted(host(sd).reshape(-1), lam_bar, opc.U, opc.e)
    check(host(x).reshape(-1), xr, (1e-9 if dt == "f64" else 2e-5))
    # plain: soft threshold
    x0 = P.prox_weighted(rd, lam_bar, None, sd)
    check(host(x0), opx.soft(host(sd), lam_bar), TOL[dt])


@pytest.mark.parametrize("ell,tail", [(40, "sqrt"), (64, "plain")])
def test_prox_l1_ssn_repeated_calls(ell, tail):
    """FP32 prox calls on one preconditioner with drifting centres (as in the
    outer iterations), then a jump to an unrelated centre and a new
    preconditioner: later calls start from stored factors of an earlier
    Jacobian, and every result matches the oracle's prox."""
    P = need_gpu()
    banner(f"prox l1 ssn repeated ell={ell} {tail}")
    n = 48
    h = W.gaussian_psf(7, 1.2)
    prob = sv.Problem("blurdown", n, None, 0.0, "l1", h=h, factor=2, levels=3)
    om = W.omega(ell, n, n, 16)
    Y = sv.sketch(prob, om)
    omd, Yd = dev(om, "f64"), dev(Y, "f64")
    ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], tail)
    pc = P.nys_factor(omd, Yd, ell, tail=tail, u_dtype=torch.float32)
    rd = P.reg_desc("l1", n, n)
    state = P.prox_state(rd, pc, torch.float32)
    lam_bar = 0.05
    s0 = W.gaussian((n, n), 17) * 0.1
    drift = W.gaussian((n, n), 18) * 0.002
    centres = [s0 + k * drift for k in range(8)] + [W.gaussian((n, n), 19) * 0.1]
    for k, s in enumerate(centres):
        sd = dev(s, "f32")
        x = P.prox_weighted(rd, lam_bar, pc, sd, state)
        xr, _, _ = opx.prox_l1_weighted(host(sd).reshape(-1), lam_bar, opc.U, opc.e)
        check(host(x).reshape(-1), xr, 2e-5, what=f"centre {k}")
    # a new factorisation of another sketch: the stored factors belong to the old one
    om2 = W.omega(ell, n, n, 26)
    Y2 = sv.sketch(prob, om2)
    ref2 = onys.nystrom(Y2.reshape(ell, -1), om2.reshape(ell, -1))
    opc2 = sv.Precond(ref2["U"], ref2["shat"], ref2["nu"], tail)
    pc2 = P.nys_factor(dev(om2, "f64"), dev(Y2, "f64"), ell, tail=tail, u_dtype=torch.float32)
    state2 = P.prox_state(rd, pc2, torch.float32)
    for s in centres[:3]:
        sd = dev(s, "f32")
        x = P.prox_weighted(rd, lam_bar, pc2, sd, state2)
        xr, _, _ = opx.prox_l1_weighted(host(sd).reshape(-1), lam_bar, opc2.U, opc2.e)
        check(host(x).reshape(-1), xr, 2e-5)


def _solve_pair(P, prob_kind, dt, with_pc, iters):
    if prob_kind == "deblur_tv":
        wl = W.workload("deblur128_tv_f64")
        prob, _ = sv.problem_from_workload(wl, seed=2, n=40)
        op = P.Operator(P.OP_BLUR, 40, 40, psf=prob.h)
        reg, lam, loss, delta, ell = "tv", prob.lam, P.LOSS_LS, 0.0, 8
    elif prob_kind == "sr_l1":
        wl = W.workload("sr512_haar_bf16")
        prob, _ = sv.problem_from_workload(wl, seed=3, n=64)
        op = P.Operator(P.OP_BLURDOWN, 64, 64, psf=prob.h, factor=2, wavelet_levels=3)
        reg, lam, loss, delta, ell = "l1", prob.lam, P.LOSS_HUBER, prob.delta, 8
    elif prob_kind == "sr_l1_db4":
        # the same problem in 4-level Daubechies-4 coordinates
        wl = W.workload("sr512_haar_bf16")
        prob, _ = sv.problem_from_workload(wl, seed=3, n=64)
        prob.levels, prob.wavelet = 4, "db4"
        op = P.Operator(P.OP_BLURDOWN, 64, 64, psf=prob.h, factor=2, wavelet_levels=4, wavelet="db4")
        reg, lam, loss, delta, ell = "l1", prob.lam, P.LOSS_HUBER, prob.delta, 8
    elif prob_kind == "fan_tv":
        # fan-beam CT (views over 360 degrees, flat detector) with TV
        wl = W.workload("ct512_hs1_f32")
        geo, V, B = (64.0, 32.0, 1.0), 24, 56
        prob = sv.Problem("fan", 32, None, wl.lam, "tv", views=V, bins=B, fan=geo)
        clean = prob.A(W.phantom_ellipses(32, 4))
        prob.y = clean + wl.noise_rel_max * np.max(clean) * W.gaussian(clean.shape, 4)
        op = P.Operator(P.OP_FAN_BEAM, 32, 32, views=V, bins=B, fan=geo)
        reg, lam, loss, delta, ell = "tv", prob.lam, P.LOSS_LS, 0.0, 10
    elif prob_kind == "fan_l1_db4":
        # fan-beam CT with the l1 prior on 2-level Daubechies-4 coefficients
        wl = W.workload("ct512_hs1_f32")
        geo, V, B = (64.0, 32.0, 1.0), 24, 56
        prob = sv.Problem("fan", 32, None, 2e-3, "l1", views=V, bins=B, levels=2,
                          wavelet="db4", fan=geo)
        clean = prob.A(ops.wavelet_analysis(W.phantom_ellipses(32, 5), 2, "db4"))
        prob.y = clean + wl.noise_rel_max * np.max(clean) * W.gaussian(clean.shape, 5)
        op = P.Operator(P.OP_FAN_BEAM, 32, 32, views=V, bins=B, fan=geo, wavelet_levels=2,
                        wavelet="db4")
        reg, lam, loss, delta, ell = "l1", prob.lam, P.LOSS_LS, 0.0, 10
    else:
        wl = W.workload("ct512_hs1_f32")
        prob, _ = sv.problem_from_workload(wl, seed=4, n=32, views=36, bins=48)
        op = P.Operator(P.OP_PARALLEL_BEAM, 32, 32, views=36, bins=48)
        reg, lam, loss, delta, ell = "hs1", prob.lam, P.LOSS_LS, 0.0, 10
    n = prob.n
    yd = dev(prob.y, dt)
    prob.y = host(yd)
    pc = opc = None
    if with_pc:
        om = W.omega(ell, n, n, 20)
        omd = dev(om, dt)
        Yref = sv.sketch(prob, host(omd))
        Yd = dev(Yref, dt)
        ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
        opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
        pc = P.nys_factor(omd, Yd, ell, u_dtype=torch.float64 if dt == "f64" else torch.float32)
    alpha = 0.9 / sv.lipschitz(prob, opc, W.gaussian((n, n), 21), 200)
    rd = P.reg_desc(reg, n, n, n_inner=10)
    x, costs, info = P.solve(op, yd, rd, lam, pc, iters, alpha=alpha, loss=loss, delta=delta)
    xr, cr = sv.wapg(prob, opc, alpha, iters, inner=10)
    return host(x), host(costs), xr, cr


def test_solve_nonnegative_matches_oracle():
    """WAPG (Alg. 3) with C = {x >= 0} and the P-weighted projection inside the
    dual iterations, against the oracle's iterates and costs."""
    P = need_gpu()
    banner("solve deblur tv nonneg f64 pc")
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=2, n=40)
    prob.box = (0.0, np.inf)
    op = P.Operator(P.OP_BLUR, 40, 40, psf=prob.h)
    n, ell, iters = prob.n, 8, 12
    yd = dev(prob.y, "f64")
    om = W.omega(ell, n, n, 20)
    omd = dev(om, "f64")
    Yref = sv.sketch(prob, host(omd))
    Yd = dev(Yref, "f64")
    ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    pc = P.nys_factor(omd, Yd, ell, u_dtype=torch.float64)
    alpha = 0.9 / sv.lipschitz(prob, opc, W.gaussian((n, n), 21), 200)
    rd = P.reg_desc("tv", n, n, n_inner=10, box=(0.0, np.inf))
    x, costs, info = P.solve(op, yd, rd, prob.lam, pc, iters, alpha=alpha, loss=P.LOSS_LS, delta=0.0)
    xr, cr = sv.wapg(prob, opc, alpha, iters, inner=10)
    assert host(x).min() >= 0.0
    check(host(x), xr, TOL["f64"], what="x")
    check(host(costs), cr, TOL["f64"], what="costs")


@pytest.mark.parametrize("kind,dt,with_pc", [("deblur_tv", "f64", False), ("deblur_tv", "f64", True),
                                             ("sr_l1", "f32", False), ("sr_l1", "f32", True),
                                             ("sr_l1_db4", "f64", True), ("sr_l1_db4", "f32", True),
                                             ("ct_hs1", "f32", True), ("fan_tv", "f64", True),
                                             ("fan_tv", "f32", False), ("fan_l1_db4", "f64", True)])
def test_solve_matches_oracle(kind, dt, with_pc):
    P = need_gpu()
    banner(f"solve {kind} {dt} pc={with_pc}")
    iters = 15
    x, c, xr, cr = _solve_pair(P, kind, dt, with_pc, iters)
    tol = TOL[dt]
    check(x, xr, tol, what="x after 15 iterations")
    check(c, cr, tol, what="costs")


def test_sr_full_size_solve_matches_oracle():
    """The super-resolution workload at its full size (512^2 -> 256^2, Haar-3,
    Huber, ell = 64, FP32 U and solver): the launch configuration the bench
    times (fused forward operator, (AU)^T psi, fused step evaluation, chord
    steps from the stored inverse, Gauss-Jordan Newton solves) against the
    oracle's FP64 iterates; the preconditioner is built on both sides from the
    oracle's sketch of the same Omega."""
    P = need_gpu()
    banner("solve SR full size 512^2 ell=64 f32")
    wl = W.workload("sr512_haar_bf16")
    prob, _ = sv.problem_from_workload(wl, seed=3)
    n, ell, iters = prob.n, 64, 6
    assert n == 512
    op = P.Operator(P.OP_BLURDOWN, n, n, psf=prob.h, factor=2, wavelet_levels=3)
    yd = dev(prob.y, "f32")
    prob.y = host(yd)
    om = W.omega(ell, n, n, 20)
    Yref = sv.sketch(prob, om)
    ref = onys.nystrom(Yref.reshape(ell, -1), om.reshape(ell, -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    pc = P.nys_factor(dev(om, "f32"), dev(Yref, "f32"), ell, u_dtype=torch.float32)
    alpha = 0.9 / sv.lipschitz(prob, opc, W.gaussian((n, n), 21), 60)
    rd = P.reg_desc("l1", n, n)
    x, costs, info = P.solve(op, yd, rd, prob.lam, pc, iters, alpha=alpha, loss=P.LOSS_HUBER,
                             delta=prob.delta)
    xr, cr = sv.wapg(prob, opc, alpha, iters, ssn_tol=1e-10)
    ex, ec = rel(host(x), xr), np.max(np.abs(host(costs) - cr) / np.abs(cr))
    banner(f"full size SR: x rel err {ex:.2e}, cost rel err {ec:.2e}")
    assert ex < 2e-6      # measured 1.3e-7: FP32 arithmetic, FP64 reductions
    assert ec < 1e-7      # measured 2.8e-9


def test_solve_power_method_step():
    P = need_gpu()
    banner("solve power method")
    n = 32
    h = W.gaussian_psf(9, 1.5)
    op = P.Operator(P.OP_BLUR, n, n, psf=h)
    y = dev(W.gaussian((n, n), 22))
    v0 = dev(W.gaussian((n, n), 23))
    rd = P.reg_desc("tv", n, n, n_inner=5)
    _, _, info = P.solve(op, y, rd, 1e-3, None, 1, power_v0=v0, power_iters=300)
    # normalised PSF: lambda_max(A^T A) = 1 (DC), approached from below
    assert 0.99 < info["L"] <= 1.0 + 1e-12
    prob = sv.Problem("blur", n, host(y), 1e-3, "tv", h=h)
    Lr = sv.lipschitz(prob, None, host(v0), 300)
    assert abs(info["L"] - Lr) < 1e-10


def _deblur_pc(P, dt, ell, n=40):
    """A 40^2 deblurring problem with the preconditioner built on both sides
    from the oracle's sketch of the same Omega."""
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=2, n=n)
    om = W.omega(ell, n, n, 20)
    omd = dev(om, dt)
    Yd = dev(sv.sketch(prob, host(omd)), dt)
    ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    pc = P.nys_factor(omd, Yd, ell, u_dtype=torch.float64 if dt == "f64" else torch.float32)
    return prob, opc, pc


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_pnorm2_matches_oracle(dt):
    """(a - b)^T P (a - b), with P^{-1}, and P = I, against the oracle's P."""
    P = need_gpu()
    banner(f"pnorm2 {dt}")
    prob, opc, pc = _deblur_pc(P, dt, 8)
    n = prob.n
    ad, bd = dev(W.gaussian((n, n), 30), dt), dev(W.gaussian((n, n), 31), dt)
    d = host(ad) - host(bd)
    for inverse in (False, True):
        got = P.pnorm2(pc, ad, bd, inverse=inverse)
        ref = float(np.sum(d * (opc.pinv(d) if inverse else opc.p(d))))
        assert abs(got - ref) <= TOL[dt] * abs(ref)
    got = P.pnorm2(pc, ad)
    ref = float(np.sum(host(ad) * opc.p(host(ad))))
    assert abs(got - ref) <= TOL[dt] * abs(ref)
    got = P.pnorm2(None, ad, bd)
    assert abs(got - float(np.sum(d * d))) <= TOL[dt] * float(np.sum(d * d))


@pytest.mark.parametrize("ell", [0, 4, 16])
def test_rate_constant_matches_oracle_across_sketch_sizes(ell):
    """L_f^P ||x^1 - x*||_P^2 (x^1 = 0, x* from 40 oracle WAPG iterations) for
    plain APG and two sketch sizes, FP64."""
    P = need_gpu()
    banner(f"rate constant ell={ell}")
    if ell:
        prob, opc, pc = _deblur_pc(P, "f64", ell)
    else:
        wl = W.workload("deblur128_tv_f64")
        prob, _ = sv.problem_from_workload(wl, seed=2, n=40)
        opc = pc = None
    n = prob.n
    op = P.Operator(P.OP_BLUR, n, n, psf=prob.h)
    yd = dev(prob.y, "f64")
    prob.y = host(yd)
    v0 = W.gaussian((n, n), 21)
    alpha = 0.9 / sv.lipschitz(prob, opc, v0, 200)
    xs, _ = sv.wapg(prob, opc, alpha, 40, inner=10, record_cost=False)
    rd = P.reg_desc("tv", n, n, n_inner=10)
    got = P.rate_constant(op, yd, rd, prob.lam, pc, dev(xs, "f64"), power_iters=60,
                          power_v0=dev(v0, "f64"))
    ref = sv.rate_constant(prob, opc, xs, v0, 60)
    assert abs(got["L"] - ref["L"]) <= 1e-9 * ref["L"]
    assert abs(got["pdist2"] - ref["pdist2"]) <= 1e-10 * ref["pdist2"]
    assert abs(got["value"] - ref["value"]) <= 1e-9 * ref["value"]


def test_solve_tv_at_size_with_a_preconditioner():
    """WAPG with the P-weighted TV prox at 384^2, ell = 64, FP32 (the
    gradient step's coefficient partials stay held while the prox applies
    P^{-1} in each of its 20 dual iterations), 3 outer iterations against the
    oracle on the same rounded inputs; P from a steep synthetic sketch."""
    P = need_gpu()
    banner("solve TV 384^2 ell=64 f32 with P")
    n, ell, iters = 384, 64, 3
    wl = W.workload("deblur128_tv_f64")
    prob, _ = sv.problem_from_workload(wl, seed=5, n=n)
    op = P.Operator(P.OP_BLUR, n, n, psf=prob.h)
    yd = dev(prob.y, "f32")
    prob.y = host(yd)
    om, Y = _steep_psd_sketch(n, ell, seed=70)
    omd, Yd = dev(om.reshape(ell, n, n), "f32"), dev(Y.reshape(ell, n, n), "f32")
    ref = onys.nystrom(host(Yd).reshape(ell, -1), host(omd).reshape(ell, -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    pc = P.nys_factor(omd, Yd, ell, u_dtype=torch.float32)
    alpha = 0.3
    rd = P.reg_desc("tv", n, n, n_inner=20)
    x, costs, info = P.solve(op, yd, rd, prob.lam, pc, iters, alpha=alpha)
    assert info["status"] == 0
    xr, cr = sv.wapg(prob, opc, alpha, iters, inner=20)
    check(host(x), xr, TOL["f32"], what="x after 3 iterations")
    check(host(costs), cr, TOL["f32"], what="costs")
