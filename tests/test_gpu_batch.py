"""Batched reconstruction (many periodic-blur problems in one graph launch)
against the FP64 oracle, instance by instance.

Each instance: sketch Y = A^T A Omega (Alg. 1, step 2), shifted Nystrom
factorisation (Alg. 1, steps 3-7), power-method step (eq. (15) constant) and
WAPG (Alg. 3) with the P-weighted TV / HS1 prox.  Sizes are small enough for
the oracle and leave ragged stencil tiles (n not a multiple of 64 or of the
tile height); PSF sizes, sketch sizes and weights differ per instance.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import banner, dev, host, need_gpu, rel
from oracle import nystrom as onys
from oracle import solver as sv

pytestmark = pytest.mark.gpu

# (n, psf size, psf sigma, ell, lambda)
SPECS = [
    (16, 3, 0.8, 8, 2e-3),
    (24, 5, 1.0, 16, 1e-3),
    (40, 7, 1.5, 20, 5e-4),
    (32, 11, 2.5, 64, 3e-3),
    (72, 9, 1.5, 32, 1e-3),
]


def _instances(seed0, specs=SPECS, reg="tv"):
    out = []
    for i, (n, k, sg, ell, lam) in enumerate(specs):
        h = W.gaussian_psf(k, sg)
        xt = W.phantom_blocks(n, seed0 + i)
        prob = sv.Problem("blur", n, None, lam, reg, h=h)
        y = prob.A(xt) + 0.01 * W.gaussian((n, n), seed0 + i)
        yd = dev(y, "f32")
        prob.y = host(yd)
        out.append(dict(prob=prob, psf=h, y=yd, lam=lam, ell=ell,
                        omega=dev(W.omega(ell, n, n, seed0 + i), "f32"),
                        v0=dev(W.gaussian((n, n), seed0 + 100 + i), "f32")))
    return out


def _host_pinv(z, U, shat, nu):
    """P^{-1} z of eq. (6) with the sqrt tail, from host copies (test-side)."""
    sK = np.sqrt(shat[shat > 0][-1])
    d = np.where(shat > 0, (sK + nu) / (shat + nu) - 1.0, 0.0)
    return z + U.T @ (d * (U @ z))


def _check_costs(c, cr):
    """FP32 iterates: the cost error is a rounding error at the scale of the
    data term, so it is bounded relative to the first cost (1e-5), and per
    iteration relative to the cost itself within 5e-4 (a preconditioner with
    ||P^{-1}|| ~ 20 amplifies FP32 rounding of the late, small costs)."""
    assert np.max(np.abs(c - cr)) < 1e-5 * abs(cr[0])
    assert np.max(np.abs(c - cr) / np.abs(cr)) < 5e-4


@pytest.mark.parametrize("reg", ["tv", "hs1", "hsinf"])
def test_batch_preconditioned_matches_oracle(reg):
    P = need_gpu()
    banner(f"batch preconditioned {reg}")
    inst = _instances(300, reg=reg)
    iters, inner, piters = 8, 10, 60
    plan = P.BatchSolver(inst, reg=P.REG_NAMES[reg], max_iter=iters,
                         n_inner=inner, power_iters=piters, record_costs=True, tune=True)
    plan.run()
    torch.cuda.synchronize()
    for i, it in enumerate(inst):
        prob, ell, n = it["prob"], it["ell"], it["prob"].n
        banner(f"batch instance {i} n={n} ell={ell}")
        Y, U = plan.sketch(i, n, n, ell)
        om = host(it["omega"])
        Yref = sv.sketch(prob, om)
        assert rel(host(Y), Yref) < 1e-5
        ref = onys.nystrom(host(Y).reshape(ell, -1), om.reshape(ell, -1))
        info = plan.info(i)
        assert info["status"] == 0
        shat = plan.shat(i, ell)
        assert rel(shat, ref["shat"]) < 1e-5
        z = W.gaussian((n * n,), 500 + i)
        opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
        got = _host_pinv(z, host(U), shat, info["nu"])
        assert rel(got, opc.pinv(z)) < 1e-4
        assert abs(info["pinv_norm"] - opc.pinv_norm) < 1e-4 * opc.pinv_norm
        Lr = sv.lipschitz(prob, opc, host(it["v0"]), piters)
        assert abs(info["L"] - Lr) < 1e-4 * Lr
        assert abs(info["alpha"] * 1.01 * info["L"] - 1.0) < 1e-12
        xr, cr = sv.wapg(prob, opc, info["alpha"], iters, inner=inner)
        assert rel(host(plan.x[i]), xr) < 1e-4
        _check_costs(host(plan.costs[i]), cr)


def test_batch_plain_apg_matches_oracle():
    P = need_gpu()
    banner("batch plain APG tv_aniso")
    inst = _instances(400, specs=SPECS[:4], reg="tv_aniso")
    iters, inner, piters = 10, 8, 80
    plan = P.BatchSolver(inst, reg=P.REG_TV_ANISO, max_iter=iters, n_inner=inner,
                         power_iters=piters, precondition=False, record_costs=True, tune=False)
    plan.run()
    torch.cuda.synchronize()
    for i, it in enumerate(inst):
        prob = it["prob"]
        info = plan.info(i)
        Lr = sv.lipschitz(prob, None, host(it["v0"]), piters)
        assert abs(info["L"] - Lr) < 1e-5 * Lr
        assert info["pinv_norm"] == 1.0
        xr, cr = sv.wapg(prob, None, info["alpha"], iters, inner=inner)
        assert rel(host(plan.x[i]), xr) < 1e-4
        _check_costs(host(plan.costs[i]), cr)


def test_batch_replay_is_bitwise_and_inputs_refill():
    """Graph replays give identical results; refilled inputs are picked up."""
    P = need_gpu()
    banner("batch replay")
    inst = _instances(600, specs=SPECS[:3])
    plan = P.BatchSolver(inst, max_iter=5, n_inner=5, power_iters=20, record_costs=True)
    x1 = [t.clone() for t in plan.run()]
    torch.cuda.synchronize()
    x2 = [t.clone() for t in plan.run()]
    torch.cuda.synchronize()
    for a, b in zip(x1, x2):
        assert torch.equal(a, b)
    # new measurements in place: the next run solves the new problem
    it = inst[1]
    prob = it["prob"]
    y_new = prob.A(W.phantom_blocks(prob.n, 999)) + 0.01 * W.gaussian((prob.n, prob.n), 998)
    it["y"].copy_(dev(y_new, "f32"))
    plan.run()
    torch.cuda.synchronize()
    prob.y = host(it["y"])
    info = plan.info(1)
    Y, U = plan.sketch(1, prob.n, prob.n, it["ell"])
    ref = onys.nystrom(host(Y).reshape(it["ell"], -1), host(it["omega"]).reshape(it["ell"], -1))
    opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
    xr, _ = sv.wapg(prob, opc, info["alpha"], 5, inner=5)
    assert rel(host(plan.x[1]), xr) < 1e-4
    assert torch.equal(plan.x[0], x1[0])


def test_batch_tile_table_and_errors():
    P = need_gpu()
    banner("batch tiles / errors")
    inst = _instances(700, specs=SPECS[:2])
    plan = P.BatchSolver(inst, max_iter=1, n_inner=1, power_iters=2, tune=True)
    tiles = plan.tiles()
    assert tiles and all(t[2] in (8, 16, 32, 64) for t in tiles)
    # the A^T A class of a k-tap PSF has 2k - 1 taps per axis
    assert {(2 * k - 1) for (_, k, _, _, _) in SPECS[:2]} <= {t[0] for t in tiles}
    bad = dict(inst[0])
    a = np.outer(np.arange(1.0, 4.0), np.arange(1.0, 4.0))
    a[0, 0] += 1.0                      # rank 2: not separable
    bad["psf"] = a / a.sum()
    with pytest.raises(P.NysError):
        P.BatchSolver([bad], max_iter=1, n_inner=1, power_iters=2)
    bad = dict(inst[0], ell=65)
    with pytest.raises(P.NysError):
        P.BatchSolver([bad], max_iter=1, n_inner=1, power_iters=2)


def test_batch_rectangular_wide_psf_and_sketch_only():
    """Rectangular images, a width that is not a multiple of 4, a PSF wider
    than the image (the periodic halo wraps more than once), and the
    sketch-only entry point on refilled test images."""
    P = need_gpu()
    banner("batch rectangular / wide PSF / sketch only")
    shapes = [(20, 36, 5, 1.0, 4, 1e-3), (12, 9, 15, 3.0, 4, 2e-3), (70, 44, 9, 1.5, 8, 5e-4)]
    inst = []
    for i, (n1, n2, k, sg, ell, lam) in enumerate(shapes):
        h = W.gaussian_psf(k, sg)
        prob = sv.Problem("blur", n1, None, lam, "tv", h=h)
        xt = W.phantom_blocks(max(n1, n2), 800 + i)[:n1, :n2]
        yd = dev(prob.A(xt) + 0.01 * W.gaussian((n1, n2), 800 + i), "f32")
        prob.y = host(yd)
        inst.append(dict(prob=prob, psf=h, y=yd, lam=lam, ell=ell, n1=n1, n2=n2,
                         omega=dev(W.omega(ell, n1, n2, 800 + i), "f32"),
                         v0=dev(W.gaussian((n1, n2), 900 + i), "f32")))
    plan = P.BatchSolver(inst, max_iter=4, n_inner=5, power_iters=30, record_costs=True)
    plan.run()
    torch.cuda.synchronize()
    for i, it in enumerate(inst):
        n1, n2, ell, prob = it["n1"], it["n2"], it["ell"], it["prob"]
        banner(f"batch rect instance {i} {n1}x{n2}")
        Y, U = plan.sketch(i, n1, n2, ell)
        om = host(it["omega"])
        assert rel(host(Y), sv.sketch(prob, om)) < 1e-5
        ref = onys.nystrom(host(Y).reshape(ell, -1), om.reshape(ell, -1))
        opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
        info = plan.info(i)
        assert rel(plan.shat(i, ell), ref["shat"]) < 1e-5
        xr, cr = sv.wapg(prob, opc, info["alpha"], 4, inner=5, x0=np.zeros((n1, n2)))
        assert rel(host(plan.x[i]), xr) < 1e-4
        _check_costs(host(plan.costs[i]), cr)
    for i, it in enumerate(inst):
        it["omega"].copy_(dev(W.omega(it["ell"], it["n1"], it["n2"], 950 + i), "f32"))
    plan.sketch_only()
    torch.cuda.synchronize()
    for i, it in enumerate(inst):
        Y, _ = plan.sketch(i, it["n1"], it["n2"], it["ell"])
        assert rel(host(Y), sv.sketch(it["prob"], host(it["omega"]))) < 1e-5
