"""Batched reconstruction (many periodic-blur problems in one graph launch)
against the FP64 oracle, instance by instance.

Each instance: sketch Y = A^T A Omega (Alg. 1, step 2), shifted Nystrom
factorisation (Alg. 1, steps 3-7), power-method step (the constant of eq. (20)) and
WAPG (Alg. 3) with the P-weighted TV / HS1 prox.  Sizes are small enough for
the oracle and leave ragged stencil tiles (n not a multiple of 64 or of the
tile height); PSF sizes, sketch sizes and weights differ per instance.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import TOL, banner, check, dev, host, need_gpu, rel
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
    """P^{-1} z of eq. (11) with the sqrt tail, from host copies (test-side)."""
    sK = np.sqrt(shat[shat > 0][-1])
    d = np.where(shat > 0, (sK + nu) / (shat + nu) - 1.0, 0.0)
    return z + U.T @ (d * (U @ z))


def _oracle_pc(Y, om, ell):
    r = onys.nystrom(Y.reshape(ell, -1), om.reshape(ell, -1))
    return sv.Precond(r["U"], r["shat"], r["nu"], "sqrt"), r


def _sketch_f32_accumulated(om, h):
    """Y = A^T A Omega evaluated in FP32 by the oracle side itself: the PSF's
    separable autocorrelation stencil (rows, then columns), one FP32 rounding
    per tap, as an FP32-accumulating sketch computes it."""
    k = h.shape[0]
    c = k // 2
    u = h[:, c] / np.sqrt(h[c, c])
    v = h[c, :] / np.sqrt(h[c, c])

    def autocorr(w):
        r = np.zeros(2 * k - 1)
        for d in range(k):
            r[k - 1 + d] = r[k - 1 - d] = np.dot(w[:k - d], w[d:])
        return r

    tr = autocorr(u).astype(np.float32)
    tc = autocorr(v).astype(np.float32)
    lo = -(k - 1)
    x = np.asarray(om, np.float32)
    acc = np.zeros_like(x)
    for a in range(2 * k - 1):
        acc = (np.float64(tr[a]) * np.roll(x, -(lo + a), -2) + acc).astype(np.float32)
    out = np.zeros_like(x)
    for b in range(2 * k - 1):
        out = (np.float64(tc[b]) * np.roll(acc, -(lo + b), -1) + out).astype(np.float32)
    return out.astype(np.float64)


class Floor:
    """The batched plan factorises its own FP32 sketch, whose sums accumulate
    in FP32 (the precision the sketch applies are specified to use), so
    results downstream of it carry that sketch error through the
    factorisation.  The oracle measures the effect on itself: it factorises
    its FP64 sketch and its own FP32-accumulated evaluation of the same
    stencil and compares.  A tolerance is the stated FP32 one, or three times
    that self-sensitivity where the factorisation's conditioning makes it
    larger (a 32^2 instance with a 11 x 11, sigma 2.5 PSF and ell = 64:
    Nystrom eigenvalues over many decades, where an FP32-accumulated sketch
    moves P^-1 by ~3e-5); two FP32 summation orders differ by a factor of
    about two in this error."""

    def __init__(self, prob, om, Yref, ell):
        self.pc64, self.ref = _oracle_pc(Yref, om, ell)
        self.pc32, _ = _oracle_pc(_sketch_f32_accumulated(om, prob.h), om, ell)
        self.prob = prob

    @staticmethod
    def tol(a64, a32):
        return max(TOL["f32"], 3.0 * rel(a32, a64))

    def pinv(self, z):
        a = self.pc64.pinv(z)
        return a, self.tol(a, self.pc32.pinv(z))

    def wapg(self, alpha, iters, inner, **kw):
        x64, c64 = sv.wapg(self.prob, self.pc64, alpha, iters, inner=inner, **kw)
        x32, c32 = sv.wapg(self.prob, self.pc32, alpha, iters, inner=inner, **kw)
        return x64, c64, self.tol(x64, x32), self.tol(np.asarray(c64), np.asarray(c32))


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
        check(host(Y), Yref, TOL["f32"], what="sketch")
        # the oracle factorises its own sketch
        fl = Floor(prob, om, Yref, ell)
        ref, opc = fl.ref, fl.pc64
        info = plan.info(i)
        assert info["status"] == 0
        shat = plan.shat(i, ell)
        check(shat, ref["shat"], TOL["f32"], what="shat")
        z = W.gaussian((n * n,), 500 + i)
        want, tol = fl.pinv(z)
        check(_host_pinv(z, host(U), shat, info["nu"]), want, tol, what="P^-1 z")
        assert abs(info["pinv_norm"] - opc.pinv_norm) < TOL["f32"] * opc.pinv_norm
        Lr = sv.lipschitz(prob, opc, host(it["v0"]), piters)
        assert abs(info["L"] - Lr) < TOL["f32"] * Lr
        assert abs(info["alpha"] * 1.01 * info["L"] - 1.0) < 1e-12
        xr, cr, tol_x, tol_c = fl.wapg(info["alpha"], iters, inner)
        check(host(plan.x[i]), xr, tol_x, what="x after 8 iterations")
        check(host(plan.costs[i]), cr, tol_c, what="costs")


def test_batch_preconditioned_cold_start_matches_oracle():
    """warm_start off: every prox starts from Q = 0 (and c = 0), against the
    oracle's WAPG with the same start."""
    P = need_gpu()
    banner("batch preconditioned tv cold start")
    inst = _instances(350, specs=SPECS[:3])
    iters, inner, piters = 6, 8, 60
    plan = P.BatchSolver(inst, max_iter=iters, n_inner=inner, power_iters=piters,
                         warm_start=False, record_costs=True, tune=False)
    plan.run()
    torch.cuda.synchronize()
    for i, it in enumerate(inst):
        prob, ell, n = it["prob"], it["ell"], it["prob"].n
        banner(f"batch cold-start instance {i} n={n} ell={ell}")
        om = host(it["omega"])
        fl = Floor(prob, om, sv.sketch(prob, om), ell)
        info = plan.info(i)
        assert info["status"] == 0
        xr, cr, tol_x, tol_c = fl.wapg(info["alpha"], iters, inner, warm_start=False)
        check(host(plan.x[i]), xr, tol_x, what="x after 6 iterations")
        check(host(plan.costs[i]), cr, tol_c, what="costs")


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
        check(host(plan.x[i]), xr, TOL["f32"], what="x after 10 iterations")
        check(host(plan.costs[i]), cr, TOL["f32"], what="costs")


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
    om = host(it["omega"])
    fl = Floor(prob, om, sv.sketch(prob, om), it["ell"])
    xr, _, tol_x, _ = fl.wapg(info["alpha"], 5, 5)
    check(host(plan.x[1]), xr, tol_x, what="x of the refilled instance")
    assert torch.equal(plan.x[0], x1[0])


def test_batch_tile_table_and_errors():
    P = need_gpu()
    banner("batch tiles / errors")
    inst = _instances(700, specs=SPECS[:2])
    plan = P.BatchSolver(inst, max_iter=1, n_inner=1, power_iters=2, tune=True)
    tiles = plan.tiles()
    assert tiles and all(t[2] in (8, 16, 32, 64, 128, 256) for t in tiles)
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
        Yref = sv.sketch(prob, om)
        check(host(Y), Yref, TOL["f32"], what="sketch")
        fl = Floor(prob, om, Yref, ell)
        info = plan.info(i)
        check(plan.shat(i, ell), fl.ref["shat"], TOL["f32"], what="shat")
        xr, cr, tol_x, tol_c = fl.wapg(info["alpha"], 4, 5, x0=np.zeros((n1, n2)))
        check(host(plan.x[i]), xr, tol_x, what="x after 4 iterations")
        check(host(plan.costs[i]), cr, tol_c, what="costs")
    for i, it in enumerate(inst):
        it["omega"].copy_(dev(W.omega(it["ell"], it["n1"], it["n2"], 950 + i), "f32"))
    plan.sketch_only()
    torch.cuda.synchronize()
    for i, it in enumerate(inst):
        Y, _ = plan.sketch(i, it["n1"], it["n2"], it["ell"])
        check(host(Y), sv.sketch(it["prob"], host(it["omega"])), TOL["f32"], what="refilled sketch")


# instances of the batched workload's largest sizes: 1024^2 with a 7 x 7 PSF
# (ell = 16) and 768^2 with a 15 x 15 PSF (ell = 8, the 29-tap A^T A stencil)
BIG = [(1024, 7, 1.2, 16, 1e-3), (768, 15, 2.8, 8, 4e-3)]


def test_batch_workload_sizes_match_oracle():
    """Sketch (every column), Nystrom eigenvalues, P^{-1} on a probe, the
    power-method constant and 5 WAPG iterations with 20 dual iterations at
    the batched workload's largest image sizes, each against the oracle's
    own sketch and factorisation."""
    P = need_gpu()
    banner("batch workload sizes 1024^2 / 768^2")
    inst = _instances(1000, specs=BIG)
    iters, inner, piters = 5, 20, 40
    plan = P.BatchSolver(inst, reg=P.REG_TV, max_iter=iters, n_inner=inner,
                         power_iters=piters, record_costs=True, tune=True)
    plan.run()
    torch.cuda.synchronize()
    for i, it in enumerate(inst):
        prob, ell, n = it["prob"], it["ell"], it["prob"].n
        banner(f"batch big instance {i} n={n} ell={ell}")
        Y, U = plan.sketch(i, n, n, ell)
        om = host(it["omega"])
        Yref = sv.sketch(prob, om)
        check(host(Y), Yref, TOL["f32"], what="sketch")
        ref = onys.nystrom(Yref.reshape(ell, -1), om.reshape(ell, -1))
        info = plan.info(i)
        assert info["status"] == 0
        shat = plan.shat(i, ell)
        check(shat, ref["shat"], TOL["f32"], what="shat")
        opc = sv.Precond(ref["U"], ref["shat"], ref["nu"], "sqrt")
        z = W.gaussian((n * n,), 1500 + i)
        check(_host_pinv(z, host(U), shat, info["nu"]), opc.pinv(z), TOL["f32"], what="P^-1 z")
        Lr = sv.lipschitz(prob, opc, host(it["v0"]), piters)
        assert abs(info["L"] - Lr) < TOL["f32"] * Lr
        xr, cr = sv.wapg(prob, opc, info["alpha"], iters, inner=inner)
        check(host(plan.x[i]), xr, TOL["f32"], what="x after 5 iterations")
        check(host(plan.costs[i]), cr, TOL["f32"], what="costs")
