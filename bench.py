"""Time to a 1e-4 relative cost gap: Nystrom-preconditioned WAPG vs plain APG.

One "step" is one whole preconditioned reconstruction on the GPU: the sketch
Y = A^T A Omega (Alg. 1 step 2), the shifted Nystrom factorisation (Alg. 1
steps 3-8), the step size by the power method, and WAPG (Alg. 3) run for the
number of outer iterations that reaches a relative cost gap of 1e-4.  Plain
APG (P = I, with its own power method) is timed the same way beside it.

--rate-sweep K1,K2,... prints instead the constant L_f^P ||x^1 - x*||_P^2 of
WAPG's rate bound for plain APG and each sketch size (x^1 = 0, x* from a long
preconditioned run at the workload's own sketch size): the sketch-size study
of the CT experiments on the synthetic workload.

Inputs are synthetic and seeded (module `workloads`), already resident in
HBM when the timed region starts.  F* is the smallest cost seen over long
untimed runs of both methods; the iteration counts that reach the gap are
found by untimed runs that record the cost, then the timed runs repeat the
solve with exactly that many iterations and no cost recording.

Prints one JSON line.  Usage:
    python bench.py [--steps K] [--warmup W] [--tail sqrt|plain]
                    [--workload batch64|sr512|ct512|fan512|deblur128|irm256]
                    [--no-cpu-baseline] [--no-oracle-err] [--copy-calibration]
                    [--rate-sweep 10,20,50,100]
    python bench.py --workload batch64 --make-fstar [--fstar-range a:b]

The default workload is the batched one (64 deblurring problems of uneven
sizes, one graph launch per solve of the whole batch), the largest of the
benchmark configurations that fits one GPU; it times the batch to the point
where every instance has reached the gap.  Its F* per instance comes from a
stored table of long FP64 runs of both methods (--make-fstar writes it).  The IRM workload (l_1 - l_1 deblurring by
Alg. 2) times its fixed schedule of outer iterations with Nystrom-PCG against
plain CG x-updates.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

GAP = 1e-4
HBM_PEAK_GBS = 8000.0

WORKLOAD_KEYS = {
    "sr512": "sr512_haar_bf16",
    "ct512": "ct512_hs1_f32",
    "fan512": "fan512_tv_f32",
    "deblur128": "deblur128_tv_f64",
    "batch64": "batch64_deblur_f32",
    "irm256": "irm256_l1l1_f32",
}

# The paper's wall time for building the preconditioner (Table II; an RTX
# 3090, 512^2 image, 100 views) where a workload has its geometry, prior and
# sketch size: context only, another machine and another implementation.
PAPER_BUILD_S = {
    "fan512_tv_f32": {"value": 0.09, "unit": "s", "gpu": "RTX 3090", "table": "II",
                      "geometry": "fan beam", "reg": "tv", "K": 20},
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- inputs
class Setup:
    """Operator, measurements and Omega of one workload, on the GPU."""

    def __init__(self, P, torch, wl, seed=0):
        self.wl = wl
        n = wl.n
        self.torch = torch
        tdt = {"f64": torch.float64, "f32": torch.float32}[wl.dtype]
        sdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[wl.sketch_dtype]
        self.tdt, self.sdt = tdt, sdt
        if wl.op in ("ct", "fan"):
            if wl.op == "ct":
                self.op = P.Operator(P.OP_PARALLEL_BEAM, n, n, views=wl.views, bins=wl.bins)
            else:
                self.op = P.Operator(P.OP_FAN_BEAM, n, n, views=wl.views, bins=wl.bins,
                                     fan=wl.fan)
            xt = W.phantom_ellipses(n, seed)
            clean = P.op_forward(self.op, torch.from_numpy(xt).to(tdt).cuda())
            cmax = float(clean.abs().max())
            noise = W.gaussian(tuple(clean.shape), seed)
            y = clean + wl.noise_rel_max * cmax * torch.from_numpy(noise).to(tdt).cuda()
            self.reg, self.loss, self.delta = wl.reg, P.LOSS_LS, 0.0
        else:
            h = W.gaussian_psf(wl.psf_k, wl.psf_sigma)
            xt = W.phantom_blocks(n, seed)
            kind = P.OP_BLUR if wl.op == "blur" else P.OP_BLURDOWN
            plain = P.Operator(kind, n, n, psf=h, factor=wl.factor)
            clean = P.op_forward(plain, torch.from_numpy(xt).to(tdt).cuda())
            noise = W.gaussian(tuple(clean.shape), seed)
            y = clean + wl.noise_sigma * torch.from_numpy(noise).to(tdt).cuda()
            if wl.salt_pepper:
                salt, pepper = W.salt_pepper_masks(tuple(clean.shape), seed, wl.salt_pepper)
                y[torch.from_numpy(salt).cuda()] = 1.0
                y[torch.from_numpy(pepper).cuda()] = 0.0
            levels = 3 if wl.reg == "l1haar3" else 0
            self.op = P.Operator(kind, n, n, psf=h, factor=wl.factor, wavelet_levels=levels)
            self.reg = "l1" if levels else wl.reg
            huber = wl.loss == "huber"
            self.loss = P.LOSS_HUBER if huber else P.LOSS_LS
            self.delta = wl.huber_delta if huber else 0.0
        self.y = y.contiguous()
        self.omega = torch.from_numpy(W.round_dtype(W.omega(wl.ell, n, n, seed), wl.sketch_dtype)) \
            .to(sdt).cuda().contiguous()
        self.v0 = torch.from_numpy(W.gaussian((n, n), seed, stream=7)).to(tdt).cuda().contiguous()
        self.rd = P.reg_desc(self.reg, n, n, n_inner=wl.inner)
        self.Y = torch.empty_like(self.omega)


def run_pc(P, S, iters, power_iters, record_cost, ev=None):
    """Sketch + factor + power method + WAPG for `iters` outer iterations."""
    if ev is not None:
        ev[0].record()
    P.nys_sketch(S.op, S.omega, out=S.Y)
    if ev is not None:
        ev[1].record()
    pc = P.nys_factor(S.omega, S.Y, S.wl.ell, u_dtype=S.tdt, tail=getattr(S, "tail", "sqrt"))
    if ev is not None:
        ev[2].record()
    x, costs, info = P.solve(S.op, S.y, S.rd, S.wl.lam, pc, iters, power_v0=S.v0,
                             power_iters=power_iters, loss=S.loss, delta=S.delta,
                             record_cost=record_cost)
    return x, costs, info, pc


def run_plain(P, S, iters, power_iters, record_cost):
    x, costs, info = P.solve(S.op, S.y, S.rd, S.wl.lam, None, iters, power_v0=S.v0,
                             power_iters=power_iters, loss=S.loss, delta=S.delta,
                             record_cost=record_cost)
    return x, costs, info


def sketch_traffic(wl):
    """HBM bytes per sketch launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken or the
    workload differs."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sketch_sr512_bf16_hbm.json")
    src = os.path.join(ROOT, "paper_2411_08178_amd", "csrc", "sketch_sr.hip")
    if wl.name != "sr512_haar_bf16" or not os.path.exists(path):
        return None
    d = json.load(open(path))
    if hashlib.sha1(open(src, "rb").read()).hexdigest() != d["source_sha1"]:
        return None
    return d["traffic_bytes_per_launch"]


def copy_peak(torch):
    """Measured stream-copy rate (GB/s): an elementwise kernel reading 1 GiB
    and writing 1 GiB, best of 5, events on the launch stream."""
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    stream = torch.cuda.current_stream()
    best = None
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        torch.mul(a, 1.0, out=b)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return round(2 * (1 << 30) / (best * 1e-3) / 1e9, 1)


def first_below(costs, fstar, gap):
    g = (costs - fstar) / abs(fstar)
    idx = np.nonzero(g <= gap)[0]
    return int(idx[0]) + 1 if len(idx) else None


# ---------------------------------------------------------------- CPU leg
def cpu_baseline(wl, k_pc, power_iters, alpha, seed=0):
    """The FP64 oracle timed on a bounded sample of the same workload and
    extrapolated to one preconditioned time-to-gap (seconds)."""
    from threadpoolctl import threadpool_info

    from oracle import nystrom as onys
    from oracle import solver as sv
    prob, _ = sv.problem_from_workload(wl, seed=seed)
    n, ell = wl.n, wl.ell
    om = W.round_dtype(W.omega(ell, n, n, seed), wl.sketch_dtype)
    # sketch: a few columns, scaled to ell; the sample sizes below follow the
    # measured cost of one A^T A application so that the leg stays bounded
    t0 = time.perf_counter()
    prob.phi(om[0])
    t_phi = time.perf_counter() - t0
    ncols = int(min(32, max(1, 6.0 // max(t_phi, 1e-3))))
    t0 = time.perf_counter()
    for k in range(1, ncols + 1):
        prob.phi(om[k % ell])
    t_col = (time.perf_counter() - t0) / ncols
    # factorisation on all ell columns: its cost does not depend on the
    # values, so the sketch of a positive diagonal operator of the same shape
    # stands in for the columns not computed above
    d = 0.01 + 0.24 * np.abs(W.gaussian((n * n,), seed, stream=8))
    Yfull = d[None, :] * om.reshape(ell, -1)
    t0 = time.perf_counter()
    r = onys.nystrom(Yfull, om.reshape(ell, -1))
    t_factor = time.perf_counter() - t0
    pc = sv.Precond(r["U"], r["shat"], r["nu"], "sqrt")
    # power method: a few steps, scaled
    v = W.gaussian((n, n), seed, stream=7)
    pi = int(min(30, max(1, 4.0 // max(t_phi, 1e-3))))
    t0 = time.perf_counter()
    sv.lipschitz(prob, pc, v, pi)
    t_pow = (time.perf_counter() - t0) / pi
    # WAPG: a few outer iterations, scaled
    it = int(min(60, max(1, 8.0 // max(t_phi, 1e-3))))
    t0 = time.perf_counter()
    sv.wapg(prob, pc, alpha, it, inner=wl.inner, record_cost=False)
    t_it = (time.perf_counter() - t0) / it
    total = t_col * ell + t_factor + t_pow * power_iters + t_it * k_pc
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    sample = (f"oracle on {ncols} sketch columns (x{ell}), full Alg. 1 factor, "
              f"{pi} power steps (x{power_iters}), {it} WAPG iterations (x{k_pc}); "
              f"numpy/scipy FP64, BLAS threads {threads}")
    return dict(value=total, unit="s", cores=threads, kind="oracle", sample=sample,
                parts=dict(sketch_per_col_s=t_col, factor_s=t_factor, power_step_s=t_pow,
                           wapg_iter_s=t_it))


# ---------------------------------------------------------------- batch
FSTAR_DIR = os.path.join(ROOT, "bench_fstar")
FSTAR_INNER, FSTAR_ITERS = 200, 1000


def batch_problem(P, torch, s, noise_sigma):
    """Operator, PSF and float32 measurements of one instance of the batched
    workload, formed on the GPU."""
    n = s.n
    h = W.gaussian_psf(s.psf_k, s.psf_sigma)
    op = P.Operator(P.OP_BLUR, n, n, psf=h)
    xt = torch.from_numpy(W.phantom_blocks(n, s.seed)).float().cuda()
    noise = torch.from_numpy(W.gaussian((n, n), s.seed)).float().cuda()
    y = (P.op_forward(op, xt) + noise_sigma * noise).contiguous()
    return op, h, y


class BatchSetup:
    """The 64 deblurring problems of the batched workload, on the GPU."""

    def __init__(self, P, torch, wl, seed=0):
        self.specs = W.batch_instances(wl.count, seed)
        self.items = []
        self.omega_host = []
        for s in self.specs:
            n = s.n
            _, h, y = batch_problem(P, torch, s, wl.noise_sigma)
            om_h = torch.from_numpy(W.omega(s.ell, n, n, s.seed)).float().pin_memory()
            om = om_h.cuda().contiguous()
            v0 = torch.from_numpy(W.gaussian((n, n), s.seed, stream=7)).float().cuda().contiguous()
            self.omega_host.append(om_h)
            self.items.append(dict(psf=h, y=y, lam=s.lam, ell=s.ell, omega=om, v0=v0))
        self.N = [s.n * s.n for s in self.specs]
        self.sketch_bytes = sum(2 * 4 * s.ell * s.n * s.n for s in self.specs)
        self.omega_bytes = sum(4 * s.ell * s.n * s.n for s in self.specs)


def batch_plan(P, B, wl, precondition, iters, power_iters, record, tail="sqrt"):
    return P.BatchSolver(B.items, reg=P.REG_TV, max_iter=iters, n_inner=wl.inner,
                         power_iters=power_iters, precondition=precondition,
                         tail=0 if tail == "sqrt" else 1, record_costs=record, tune=True)


def fstar_path(wl, seed, tail):
    return os.path.join(FSTAR_DIR, f"{wl.name}_seed{seed}.json")


def make_fstar(args, P, torch, wl):
    """F* of every instance of the batched workload: the smallest cost of two
    long FP64 runs, plain APG and Nystrom-preconditioned WAPG (the instance's
    own sketch size, sqrt tail), each with FSTAR_INNER dual iterations per
    prox so that the proximal steps are nearly exact; the two must agree to
    1e-8 relative.  Written to bench_fstar/ (instances a:b with --fstar-range
    merge into an existing table)."""
    specs = W.batch_instances(wl.count, args.seed)
    a, b = (int(v) for v in args.fstar_range.split(":")) if args.fstar_range else (0, len(specs))
    path = args.fstar_out or fstar_path(wl, args.seed, "sqrt")
    table = json.load(open(path)) if os.path.exists(path) else {
        "workload": wl.name, "seed": args.seed, "inner": FSTAR_INNER, "iters": FSTAR_ITERS,
        "dtype": "f64", "methods": ["plain APG", "Nystrom WAPG, sqrt tail"],
        "instances": [None] * len(specs)}
    for i in range(a, b):
        s = specs[i]
        t0 = time.perf_counter()
        op, h, y32 = batch_problem(P, torch, s, wl.noise_sigma)
        y = y32.double().contiguous()
        n = s.n
        rd = P.reg_desc("tv", n, n, n_inner=FSTAR_INNER)
        v0 = torch.from_numpy(W.gaussian((n, n), s.seed, stream=7)).cuda().contiguous()
        _, c_pl, _ = P.solve(op, y, rd, s.lam, None, FSTAR_ITERS, power_v0=v0,
                             power_iters=args.power_iters)
        om = torch.from_numpy(W.omega(s.ell, n, n, s.seed)).cuda().contiguous()
        pc = P.nys_factor(om, P.nys_sketch(op, om), s.ell, u_dtype=torch.float64)
        _, c_pc, _ = P.solve(op, y, rd, s.lam, pc, FSTAR_ITERS, power_v0=v0,
                             power_iters=args.power_iters)
        m_pl, m_pc = float(c_pl.min()), float(c_pc.min())
        fs = min(m_pl, m_pc)
        res = abs(m_pl - m_pc) <= 1e-8 * abs(fs)
        table["instances"][i] = dict(n=n, psf_k=s.psf_k, psf_sigma=s.psf_sigma, lam=s.lam,
                                     ell=s.ell, fstar=fs, min_plain=m_pl, min_precond=m_pc,
                                     resolved=bool(res))
        log(f"instance {i} n={n} ell={s.ell}: F*={fs!r} plain {m_pl!r} precond {m_pc!r} "
            f"agree {abs(m_pl - m_pc) / abs(fs):.2e} ({time.perf_counter() - t0:.1f}s)")
        del pc, om
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        json.dump(table, open(path, "w"), indent=1)
    print(json.dumps({"fstar_table": os.path.relpath(path, ROOT), "done": [a, b]}), flush=True)


def load_fstar(wl, seed, specs):
    """F* per instance from the stored FP64 table, or None (entries that do not
    match the instance draw are rejected)."""
    path = fstar_path(wl, seed, "sqrt")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    out = []
    for s, e in zip(specs, t["instances"]):
        if e is None or e["n"] != s.n or e["ell"] != s.ell or e["psf_k"] != s.psf_k or \
                abs(e["lam"] - s.lam) > 1e-15 * s.lam:
            return None
        out.append(e)
    return out if len(out) == len(specs) else None


def cpu_model():
    """The host CPU's model name and the CPUs this process may use."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def cpu_baseline_batch(wl, B, k_pc, power_iters, seed=0):
    """The FP64 oracle on a bounded sample of the batch (two instances of
    different sizes), extrapolated per pixel to all instances (seconds); once
    with every BLAS thread and once on one core."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import nystrom as onys
    from oracle import solver as sv
    sample = [s for s in B.specs if s.n == 256][:1] + [s for s in B.specs if s.n == 512][:1]

    def measure():
        per_px = dict(sketch_col=[], factor_col=[], power=[], wapg=[])
        for s in sample:
            n = s.n
            h = W.gaussian_psf(s.psf_k, s.psf_sigma)
            prob = sv.Problem("blur", n, None, s.lam, "tv", h=h)
            prob.y = prob.A(W.phantom_blocks(n, s.seed)) + wl.noise_sigma * W.gaussian((n, n), s.seed)
            om = W.round_dtype(W.omega(s.ell, n, n, s.seed), "f32")
            ncols = 8
            t0 = time.perf_counter()
            Y = np.stack([prob.phi(om[k]) for k in range(ncols)])
            per_px["sketch_col"].append((time.perf_counter() - t0) / ncols / (n * n))
            d = 0.01 + 0.24 * np.abs(W.gaussian((n * n,), seed, stream=8))
            Yfull = d[None, :] * om.reshape(s.ell, -1)
            t0 = time.perf_counter()
            r = onys.nystrom(Yfull, om.reshape(s.ell, -1))
            per_px["factor_col"].append((time.perf_counter() - t0) / (n * n * s.ell))
            pc = sv.Precond(r["U"], r["shat"], r["nu"], "sqrt")
            t0 = time.perf_counter()
            sv.lipschitz(prob, pc, W.gaussian((n, n), s.seed, stream=7), 10)
            per_px["power"].append((time.perf_counter() - t0) / 10 / (n * n))
            it = 4
            t0 = time.perf_counter()
            sv.wapg(prob, pc, 0.5, it, inner=wl.inner, record_cost=False)
            per_px["wapg"].append((time.perf_counter() - t0) / it / (n * n))
            del Y
        m = {k: float(np.mean(v)) for k, v in per_px.items()}
        total = 0.0
        for s in B.specs:
            N = s.n * s.n
            total += (m["sketch_col"] * N * s.ell + m["factor_col"] * N * s.ell +
                      m["power"] * N * power_iters + m["wapg"] * N * k_pc)
        return total, m

    total, m = measure()
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    with threadpool_limits(limits=1):
        total1, m1 = measure()
    model, ncpu = cpu_model()
    desc = (f"oracle on instances n={[s.n for s in sample]}: 8 sketch columns, full Alg. 1 "
            f"factor, 10 power steps, 4 WAPG iterations each; per-pixel costs extrapolated to "
            f"all {len(B.specs)} instances ({k_pc} iterations); numpy/scipy FP64, "
            f"BLAS threads {threads}")
    return dict(value=total, unit="s", cores=threads, kind="oracle", sample=desc,
                cpu_model=model, host_cpus=ncpu,
                one_core={"value": total1, "cores": 1,
                          "parts": {k + "_per_px_s": v for k, v in m1.items()}},
                parts={k + "_per_px_s": v for k, v in m.items()})


def oracle_err_batch(P, torch, wl, B, tail, seed=0):
    """Errors of the timed launch configuration against the FP64 oracle on one
    instance of the batch (the smallest): three sketch columns, P^{-1} on a
    probe (both sides factorising their own sketch) and the iterate after six
    WAPG iterations.  The instance runs alone through the same batched solver
    (one graph, same kernels)."""
    from oracle import nystrom as onys
    from oracle import solver as sv
    i = int(np.argmin([s.n * s.n * s.ell * s.psf_k for s in B.specs]))
    s = B.specs[i]
    it = B.items[i]
    n, ell = s.n, s.ell
    plan = P.BatchSolver([it], reg=P.REG_TV, max_iter=6, n_inner=wl.inner, power_iters=60,
                         tail=0 if tail == "sqrt" else 1, record_costs=True, tune=False)
    plan.run()
    torch.cuda.synchronize()
    prob = sv.Problem("blur", n, it["y"].double().cpu().numpy(), s.lam, "tv", h=it["psf"])
    om = it["omega"].double().cpu().numpy()
    Yg, Ug = plan.sketch(0, n, n, ell)
    Yref = sv.sketch(prob, om)
    rel = lambda a, b: float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
    cols = [0, ell // 2, ell - 1]
    e_sk = max(rel(Yg[k].double().cpu().numpy(), Yref[k]) for k in cols)
    r = onys.nystrom(Yref.reshape(ell, -1), om.reshape(ell, -1))
    opc = sv.Precond(r["U"], r["shat"], r["nu"], tail)
    info = plan.info(0)
    shat = plan.shat(0, ell)
    U = Ug.double().cpu().numpy()
    z = W.gaussian((n * n,), seed + 77)
    sK = np.sqrt(shat[-1]) if tail == "sqrt" else shat[-1]
    d = (sK + info["nu"]) / (shat + info["nu"]) - 1.0
    e_pinv = rel(z + U.T @ (d * (U @ z)), opc.pinv(z))
    xr, _ = sv.wapg(prob, opc, info["alpha"], 6, inner=wl.inner)
    e_x = rel(plan.x[0].double().cpu().numpy(), xr)
    return {"instance": i, "n": n, "ell": ell, "psf_k": s.psf_k, "sketch_cols": e_sk,
            "pinv_probe": e_pinv, "x_after_6_iterations": e_x, "norm": "relative 2-norm"}


def main_batch(args, P, torch, wl):
    log(f"workload {wl.name}: {wl.count} instances")
    t0 = time.perf_counter()
    B = BatchSetup(P, torch, wl, args.seed)
    torch.cuda.synchronize()
    log(f"inputs generated in {time.perf_counter() - t0:.1f}s: {sum(B.N)} pixels, "
        f"{sum(s.ell for s in B.specs)} sketch columns, {B.sketch_bytes / 1e9:.2f} GB Omega + Y")
    tail = args.tail
    ref_iters = args.ref_iters
    t0 = time.perf_counter()
    ref_pc = batch_plan(P, B, wl, True, ref_iters, args.power_iters, True, tail)
    ref_pc.run()
    ref_pl = batch_plan(P, B, wl, False, ref_iters, args.power_iters, True, tail)
    ref_pl.run()
    torch.cuda.synchronize()
    c_pc = np.stack([c.cpu().numpy() for c in ref_pc.costs])
    c_pl = np.stack([c.cpu().numpy() for c in ref_pl.costs])
    table = load_fstar(wl, args.seed, B.specs)
    if table is not None:
        fstar = np.array([e["fstar"] for e in table])
        resolved = [bool(e["resolved"]) for e in table]
        fsrc = (f"FP64 runs of both methods, {FSTAR_INNER} dual iterations, {FSTAR_ITERS} "
                f"iterations ({os.path.relpath(fstar_path(wl, args.seed, tail), ROOT)})")
    else:
        fstar = np.minimum(c_pc.min(axis=1), c_pl.min(axis=1))
        resolved = [False] * len(fstar)
        fsrc = f"smallest FP32 cost of the {ref_iters}-iteration reference runs (no FP64 table)"
    # F* is a lower bound of every cost: the FP32 runs may undercut it only by
    # their own cost-evaluation rounding
    undercut = float(np.max((fstar - np.minimum(c_pc.min(axis=1), c_pl.min(axis=1))) / fstar))
    k_pc = [first_below(c_pc[i], fstar[i], GAP) for i in range(len(fstar))]
    k_pl = [first_below(c_pl[i], fstar[i], GAP) for i in range(len(fstar))]
    reached_pc = all(k is not None for k in k_pc)
    reached_pl = all(k is not None for k in k_pl)
    kp = max(k if k is not None else ref_iters for k in k_pc)
    kq = max(k if k is not None else ref_iters for k in k_pl)
    Lpc = [ref_pc.info(i)["L"] for i in range(len(fstar))]
    floor_pc = float(np.max((c_pc[:, -1] - fstar) / fstar))
    floor_pl = float(np.max((c_pl[:, -1] - fstar) / fstar))
    log(f"reference runs ({ref_iters} its) {time.perf_counter() - t0:.1f}s; F* from {fsrc}; "
        f"resolved {sum(resolved)}/{len(resolved)}; largest undercut {undercut:.2e}; "
        f"batch iterations to gap: precond {kp} (all: {reached_pc}), plain {kq} (all: {reached_pl}); "
        f"gap after {ref_iters}: precond {floor_pc:.2e}, plain {floor_pl:.2e}")
    del ref_pc, ref_pl
    stream = torch.cuda.current_stream()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)

    def timed(plan):
        for _ in range(args.warmup):
            plan.run()
        torch.cuda.synchronize()
        t_start.record(stream)
        for _ in range(args.steps):
            plan.run()
        t_end.record(stream)
        torch.cuda.synchronize()
        return t_start.elapsed_time(t_end) / args.steps

    plan_pc = batch_plan(P, B, wl, True, kp, args.power_iters, False, tail)
    ms_pc = timed(plan_pc)
    # roofline: the batched sketch A^T A Omega over all instances (one
    # persistent launch), a burst bracketed by events on the launch stream
    burst = 10
    plan_pc.sketch_only()
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(burst):
        plan_pc.sketch_only()
    t_end.record(stream)
    torch.cuda.synchronize()
    sk_ms = t_start.elapsed_time(t_end) / burst
    tiles = plan_pc.tiles()
    del plan_pc
    plan_pl = batch_plan(P, B, wl, False, kq, args.power_iters, False, tail)
    ms_pl = timed(plan_pl)
    del plan_pl
    # Omega from pinned host memory to HBM (reported beside the value, which
    # starts with every input resident in HBM)
    t_start.record(stream)
    for it, om_h in zip(B.items, B.omega_host):
        it["omega"].copy_(om_h, non_blocking=True)
    t_end.record(stream)
    torch.cuda.synchronize()
    up_ms = t_start.elapsed_time(t_end)
    log(f"preconditioned {ms_pc:.1f} ms ({kp} its), plain {ms_pl:.1f} ms ({kq} its); "
        f"batched sketch {sk_ms * 1e3:.1f} us; Omega upload {up_ms:.1f} ms")
    achieved = B.sketch_bytes / (sk_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": batch_sketch_traffic(wl, args.seed),
            "kernel": "bstream_kernel: batched sketch A^T A Omega, all instances, one launch",
            "bytes_per_launch": B.sketch_bytes, "avg_launch_us": round(sk_ms * 1e3, 2)}
    roof["measured_copy_peak"] = copy_peak(torch)
    roof["frac_of_copy_peak"] = round(achieved / roof["measured_copy_peak"], 4)
    out = {
        "metric": "time to 1e-4 rel. cost gap, Nystrom-precond WAPG (sketch+factor+step+solve)",
        "value": round(ms_pc / 1e3, 6),
        "gap_reached": {"precond": reached_pc, "plain": reached_pl},
        "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_pc, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "instances": wl.count,
                   "sizes": sorted(set(s.n for s in B.specs)), "pixels": int(sum(B.N)),
                   "ell_total": int(sum(s.ell for s in B.specs)), "solver_dtype": "f32",
                   "factor_dtype": "f64", "reg": "tv", "inner": wl.inner, "tail": tail,
                   "power_iters": args.power_iters, "seed": args.seed, "tiles": tiles},
        "plain_apg_s": round(ms_pl / 1e3, 6),
        "speedup_vs_plain": round(ms_pl / ms_pc, 4),
        "omega_upload_s": round(up_ms / 1e3, 6),
        "value_with_omega_upload_s": round((ms_pc + up_ms) / 1e3, 6),
        "iters_to_gap": {"precond": kp, "plain": kq, "reference_iters": ref_iters,
                         "precond_per_instance_median": float(np.median(
                             [k if k is not None else ref_iters for k in k_pc])),
                         "plain_per_instance_median": float(np.median(
                             [k if k is not None else ref_iters for k in k_pl]))},
        "fstar": {"source": fsrc, "resolved": int(sum(resolved)), "instances": len(resolved),
                  "tolerance": 1e-8, "largest_undercut": undercut,
                  "gap_after_reference": {"precond": floor_pc, "plain": floor_pl}},
        "L_precond_range": [float(min(Lpc)), float(max(Lpc))],
        "roofline": roof,
    }
    if not args.no_oracle_err:
        t0 = time.perf_counter()
        out["oracle_err"] = oracle_err_batch(P, torch, wl, B, tail, args.seed)
        log(f"oracle error leg took {time.perf_counter() - t0:.1f}s")
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline_batch(wl, B, kp, args.power_iters, args.seed)
        log(f"cpu baseline leg took {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


def code_digest(path):
    """sha1 of a C++ source without its // comments and blank lines: changes
    to the code (not to its comments) change it."""
    import hashlib
    import re
    lines = []
    for line in open(path, encoding="utf-8"):
        code = re.sub(r"//.*$", "", line).rstrip()
        if code:
            lines.append(code)
    return hashlib.sha1("\n".join(lines).encode()).hexdigest()


def batch_sketch_traffic(wl, seed):
    """HBM bytes of one batched sketch launch from the committed rocprofv3
    counter summary, or None when the stencil source's code changed since it
    was taken or the workload differs."""
    path = os.path.join(ROOT, "profiles", "bstream_batch64_hbm.json")
    src = os.path.join(ROOT, "paper_2411_08178_amd", "csrc", "batch.hip")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("workload") != wl.name or d.get("seed") != seed or \
            code_digest(src) != d.get("source_code_sha1"):
        return None
    return d["traffic_bytes_per_launch"]


# ---------------------------------------------------------------- IRM
def lp_objective_gpu(P, torch, op, x, y, lam, p, q, eps):
    """Smoothed l_p - l_q objective of x (A x on the GPU, sums in FP64)."""
    r = (P.op_forward(op, x) - y).double()
    xd = x.double()
    g1 = torch.zeros_like(xd)
    g2 = torch.zeros_like(xd)
    g1[1:, :] = xd[1:, :] - xd[:-1, :]
    g2[:, 1:] = xd[:, 1:] - xd[:, :-1]
    f = float(((r * r + eps) ** (p / 2)).sum()) / p
    g = float(((g1 * g1 + eps) ** (q / 2)).sum() + ((g2 * g2 + eps) ** (q / 2)).sum()) / q
    return f + lam * g


def cpu_baseline_irm(wl, h, y_host, its_pc, seed=0):
    """The FP64 oracle on a bounded sample (the sketch of Phi_1, Alg. 1, a few
    PCG steps), extrapolated to the GPU run's step counts (seconds)."""
    from threadpoolctl import threadpool_info

    from oracle import irm as oi
    from oracle import nystrom as onys
    from oracle import operators as ops
    n, ell, eps = wl.n, wl.ell, wl.smooth_eps
    A = lambda v: ops.blur(v, h)
    At = lambda v: ops.blur_adjoint(v, h)
    x = np.zeros((n, n))
    wf = oi.weights(A(x) - y_host, 1.0, eps)
    wg = oi.weights(ops.grad(x), 1.0, eps)
    phi = lambda v: (At(wf * A(v.reshape(n, n))) +
                     wl.lam * ops.grad_adjoint(wg * ops.grad(v.reshape(n, n)))).reshape(-1)
    om = W.round_dtype(W.omega(ell, n, n, seed), "f32")
    ncols = 8
    t0 = time.perf_counter()
    Y = np.stack([phi(om[k]) for k in range(ncols)])
    t_col = (time.perf_counter() - t0) / ncols
    Yfull = np.concatenate([Y, (0.5 + W.gaussian((ell - ncols, 1), seed, 9) ** 2) *
                            om[ncols:].reshape(ell - ncols, -1)])
    t0 = time.perf_counter()
    r = onys.nystrom(Yfull, om.reshape(ell, -1))
    t_fac = time.perf_counter() - t0
    b = At(wf * y_host).reshape(-1)
    pinv = lambda v: onys.pinv_apply(v, r["U"], r["shat"], r["nu"], "plain")
    steps = 30
    t0 = time.perf_counter()
    oi.pcg(phi, b, np.zeros(n * n), 1e-30, steps, pinv)
    t_step = (time.perf_counter() - t0) / steps
    total = len(its_pc) * (t_col * ell + t_fac) + sum(its_pc) * t_step
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return dict(value=total, unit="s", cores=threads, kind="oracle",
                sample=(f"oracle: {ncols} sketch columns of Phi_1 (x{ell}), Alg. 1 on a full-size "
                        f"stand-in, {steps} PCG steps; extrapolated to {len(its_pc)} outer "
                        f"iterations and {sum(its_pc)} PCG steps; numpy/scipy FP64, BLAS threads "
                        f"{threads}"),
                parts=dict(sketch_col_s=t_col, factor_s=t_fac, pcg_step_s=t_step))


def main_irm(args, P, torch, wl):
    n = wl.n
    h = W.gaussian_psf(wl.psf_k, wl.psf_sigma)
    op = P.Operator(P.OP_BLUR, n, n, psf=h)
    xt = torch.from_numpy(W.phantom_blocks(n, args.seed)).float().cuda()
    y = P.op_forward(op, xt)
    salt, pepper = W.salt_pepper_masks((n, n), args.seed, wl.salt_pepper)
    y[torch.from_numpy(salt).cuda()] = 1.0
    y[torch.from_numpy(pepper).cuda()] = 0.0
    y = y.contiguous()
    om = torch.from_numpy(W.omega(wl.ell, n, n, args.seed)).float().cuda().contiguous()
    eps, p, q, tol, outer = wl.smooth_eps, args.irm_p, 1.0, 1e-4, wl.outer
    log(f"workload {wl.name}: n={n} ell={wl.ell} p={p} outer={outer} PCG tol={tol}")
    stream = torch.cuda.current_stream()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)

    def run(omega):
        return P.irm_solve(op, y, wl.lam, p=p, q=q, eps=eps, max_outer=outer, max_cg=20000,
                           cg_tol=tol, omega=omega)

    def timed(omega):
        for _ in range(args.warmup):
            run(omega)
        torch.cuda.synchronize()
        t_start.record(stream)
        for _ in range(args.steps):
            x, its = run(omega)
        t_end.record(stream)
        torch.cuda.synchronize()
        return t_start.elapsed_time(t_end) / args.steps, x, its

    ms_pc, x_pc, its_pc = timed(om)
    ms_cg, x_cg, its_cg = timed(None)
    f_pc = lp_objective_gpu(P, torch, op, x_pc, y, wl.lam, p, q, eps)
    f_cg = lp_objective_gpu(P, torch, op, x_cg, y, wl.lam, p, q, eps)
    log(f"PCG {ms_pc:.1f} ms ({sum(its_pc)} steps), CG {ms_cg:.1f} ms ({sum(its_cg)} steps); "
        f"objective {f_pc:.8g} vs {f_cg:.8g}")
    # roofline: one P^{-1} application (two passes over U, ell x N FP32)
    Yb = P.nys_sketch(op, om)
    pc = P.nys_factor(om, Yb, wl.ell, u_dtype=torch.float32, tail="plain")
    v = torch.randn(n, n, device="cuda")
    out = torch.empty_like(v)
    P.nys_apply(pc, v, out=out)
    torch.cuda.synchronize()
    burst = 50
    t_start.record(stream)
    for _ in range(burst):
        P.nys_apply(pc, v, out=out)
    t_end.record(stream)
    torch.cuda.synchronize()
    ap_ms = t_start.elapsed_time(t_end) / burst
    ap_bytes = 2 * 4 * wl.ell * n * n + 3 * 4 * n * n
    achieved = ap_bytes / (ap_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "P^-1 application (U^T v, then v + U c; U is ell x N FP32)",
            "bytes_per_launch": ap_bytes, "avg_launch_us": round(ap_ms * 1e3, 2)}
    roof["measured_copy_peak"] = copy_peak(torch)
    roof["frac_of_copy_peak"] = round(achieved / roof["measured_copy_peak"], 4)
    out_j = {
        "metric": "IRM wall time (Alg. 2, fixed outer iterations, CG tol 1e-4): Nystrom-PCG vs CG",
        "value": round(ms_pc / 1e3, 6),
        "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_pc, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": n, "ell": wl.ell, "p": p, "q": q, "eps": eps,
                   "lambda": wl.lam, "outer": outer, "cg_tol": tol, "psf": [wl.psf_k, wl.psf_sigma],
                   "salt_pepper": wl.salt_pepper, "seed": args.seed, "tail": "plain"},
        "plain_cg_s": round(ms_cg / 1e3, 6),
        "speedup_vs_plain": round(ms_cg / ms_pc, 4),
        "saved_time": round((ms_cg - ms_pc) / ms_cg, 4),
        "cg_steps": {"pcg_total": int(sum(its_pc)), "cg_total": int(sum(its_cg)),
                     "pcg": its_pc, "cg": its_cg},
        "objective": {"pcg": f_pc, "cg": f_cg},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out_j["cpu_baseline"] = cpu_baseline_irm(wl, h, y.double().cpu().numpy(), its_pc, args.seed)
        log(f"cpu baseline leg took {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out_j), flush=True)


# ---------------------------------------------------------------- main
def main_rate_sweep(args, P, torch, wl):
    """The rate constant against the sketch size (one JSON line)."""
    S = Setup(P, torch, wl, args.seed)
    S.tail = args.tail
    t0 = time.perf_counter()
    x_star, c, _, _ = run_pc(P, S, args.ref_iters, args.power_iters, True)
    torch.cuda.synchronize()
    log(f"x* from {args.ref_iters} preconditioned iterations in {time.perf_counter() - t0:.1f}s, "
        f"F = {float(c[-1]):.10g}")
    rows = []
    n = wl.n
    for K in [0] + [int(k) for k in args.rate_sweep.split(",") if k]:
        pc = None
        if K:
            om = torch.from_numpy(W.round_dtype(W.omega(K, n, n, args.seed), wl.sketch_dtype)) \
                .to(S.sdt).cuda().contiguous()
            Y = P.nys_sketch(S.op, om)
            pc = P.nys_factor(om, Y, K, u_dtype=S.tdt, tail=args.tail)
        r = P.rate_constant(S.op, S.y, S.rd, wl.lam, pc, x_star, power_iters=args.power_iters,
                            power_v0=S.v0, loss=S.loss, delta=S.delta)
        rows.append({"K": K, "L": r["L"], "pdist2": r["pdist2"], "value": r["value"]})
        log(f"K={K}: L={r['L']:.6g} ||x*||_P^2={r['pdist2']:.6g} constant={r['value']:.6g}")
        del pc
    print(json.dumps({"metric": "L_f^P ||x^1 - x*||_P^2 vs sketch size (x^1 = 0)",
                      "workload": wl.name, "tail": args.tail, "x_star_iters": args.ref_iters,
                      "power_iters": args.power_iters, "rows": rows}), flush=True)


def main_ell_sweep(args, P, torch, wl):
    """Time to the 1e-4 gap against the sketch size K (one JSON line): for
    plain APG and each K, an untimed reference run of args.ref_iters
    iterations, F* = the smallest cost of all of them, then a timed run of
    exactly the iterations that reach the gap (sketch + factorisation + power
    method + WAPG, as the headline metric times them)."""
    S = Setup(P, torch, wl, args.seed)
    S.tail = args.tail
    n = wl.n
    Ks = [0] + [int(k) for k in args.ell_sweep.split(",") if k]

    def one(K, iters, record):
        if K == 0:
            return P.solve(S.op, S.y, S.rd, wl.lam, None, iters, power_v0=S.v0,
                           power_iters=args.power_iters, loss=S.loss, delta=S.delta,
                           record_cost=record)
        om = torch.from_numpy(W.round_dtype(W.omega(K, n, n, args.seed), wl.sketch_dtype)) \
            .to(S.sdt).cuda().contiguous()
        Y = P.nys_sketch(S.op, om)
        pc = P.nys_factor(om, Y, K, u_dtype=S.tdt, tail=args.tail)
        return P.solve(S.op, S.y, S.rd, wl.lam, pc, iters, power_v0=S.v0,
                       power_iters=args.power_iters, loss=S.loss, delta=S.delta,
                       record_cost=record)

    costs, Ls = {}, {}
    for K in Ks:
        t0 = time.perf_counter()
        _, c, info = one(K, args.ref_iters, True)
        torch.cuda.synchronize()
        costs[K] = c.cpu().numpy()
        Ls[K] = info["L"]
        log(f"K={K}: reference {args.ref_iters} its in {time.perf_counter() - t0:.1f}s, "
            f"end cost {costs[K][-1]:.10g}, L={Ls[K]:.6g}")
    fstar = float(min(c.min() for c in costs.values()))
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for K in Ks:
        k = first_below(costs[K], fstar, GAP)
        row = {"K": K, "iters_to_gap": k, "L": Ls[K]}
        if k is not None:
            one(K, k, False)
            torch.cuda.synchronize()
            e0.record(stream)
            one(K, k, False)
            e1.record(stream)
            torch.cuda.synchronize()
            row["time_to_gap_s"] = round(e0.elapsed_time(e1) / 1e3, 6)
        else:
            row["gap_after_reference"] = float((costs[K][-1] - fstar) / fstar)
        rows.append(row)
        log(f"K={K}: {row}")
    print(json.dumps({"metric": "time to 1e-4 rel. cost gap vs sketch size (K = 0: plain APG)",
                      "workload": wl.name, "tail": args.tail, "reference_iters": args.ref_iters,
                      "fstar": fstar, "power_iters": args.power_iters, "rows": rows}), flush=True)


def sketch_burst(args, P, torch, wl):
    """Inputs of the workload, then args.sketch_burst back-to-back sketch
    launches bracketed by events (a profiler run's subject)."""
    stream = torch.cuda.current_stream()
    if wl.count > 1:
        B = BatchSetup(P, torch, wl, args.seed)
        plan = batch_plan(P, B, wl, True, 1, 1, False)
        run, nbytes = plan.sketch_only, B.sketch_bytes
    else:
        S = Setup(P, torch, wl, args.seed)
        run = lambda: P.nys_sketch(S.op, S.omega, out=S.Y)  # noqa: E731
        nbytes = 2 * wl.ell * S.op.N * S.omega.element_size()
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.sketch_burst):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.sketch_burst
    print(json.dumps({"workload": wl.name, "sketch_launches": args.sketch_burst + 1,
                      "avg_sketch_us": round(ms * 1e3, 2), "bytes_per_launch": nbytes,
                      "GB_per_s": round(nbytes / (ms * 1e-3) / 1e9, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch64", choices=sorted(WORKLOAD_KEYS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--power-iters", type=int, default=100)
    ap.add_argument("--rate-sweep", default="",
                    help="comma-separated sketch sizes: print the rate constant per size")
    ap.add_argument("--ell-sweep", default="",
                    help="comma-separated sketch sizes: print the time to the gap per size")
    ap.add_argument("--ref-iters", type=int, default=20000,
                    help="iterations of the untimed F* runs of both methods")
    ap.add_argument("--tail", default="sqrt", choices=["sqrt", "plain"],
                    help="s_K in P: its square root (the paper's heuristic) or itself")
    ap.add_argument("--irm-p", type=float, default=1.0,
                    help="data-term exponent p of the IRM workload (the paper runs 0.5 ... 1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-err", action="store_true",
                    help="skip the FP64-oracle error leg")
    ap.add_argument("--make-fstar", action="store_true",
                    help="batched workload: compute the FP64 F* table (long runs of both methods)")
    ap.add_argument("--fstar-out", default="",
                    help="path of the F* table to write (--make-fstar; default bench_fstar/)")
    ap.add_argument("--fstar-range", default="",
                    help="a:b -- instances of the F* table to compute (--make-fstar)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--sketch-burst", type=int, default=0,
                    help="only build the workload's inputs and run its sketch this many times "
                         "(kernel traces and counters of the sketch kernel)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2411_08178_amd as P
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    P.lib()

    if args.copy_calibration:
        # a plain elementwise kernel of known traffic: reads 1 GiB, writes 1 GiB
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4, "launches": 3}))
        return

    wl = W.workload(WORKLOAD_KEYS[args.workload])
    if args.sketch_burst > 0:
        return sketch_burst(args, P, torch, wl)
    if wl.count > 1:
        if args.make_fstar:
            return make_fstar(args, P, torch, wl)
        if args.ref_iters == 20000:
            args.ref_iters = 300
        return main_batch(args, P, torch, wl)
    if wl.name.startswith("irm"):
        return main_irm(args, P, torch, wl)
    if args.rate_sweep:
        return main_rate_sweep(args, P, torch, wl)
    if args.ell_sweep:
        return main_ell_sweep(args, P, torch, wl)
    log(f"workload {wl.name}: n={wl.n} ell={wl.ell} sketch={wl.sketch_dtype} solver={wl.dtype}")
    S = Setup(P, torch, wl, args.seed)
    torch.cuda.synchronize()

    # ---- F* and iteration counts (untimed)
    ref_iters = args.ref_iters
    S.tail = args.tail
    t0 = time.perf_counter()
    _, c_pc, info_pc, pc_ref = run_pc(P, S, ref_iters, args.power_iters, True)
    _, c_pl, info_pl = run_plain(P, S, ref_iters, args.power_iters, True)
    torch.cuda.synchronize()
    c_pc, c_pl = c_pc.cpu().numpy(), c_pl.cpu().numpy()
    fstar = float(min(c_pc.min(), c_pl.min()))
    k_pc = first_below(c_pc, fstar, GAP)
    k_pl = first_below(c_pl, fstar, GAP)
    pcinfo = pc_ref.info()
    log(f"reference runs {ref_iters} its in {time.perf_counter() - t0:.1f}s; F*={fstar:.10g} "
        f"(pc end {c_pc[-1]:.10g}, plain end {c_pl[-1]:.10g}); k_pc={k_pc} k_plain={k_pl}; "
        f"L_pc={info_pc['L']:.6g} L_plain={info_pl['L']:.6g}; nu={pcinfo['nu']:.3e} "
        f"shat[0]={pcinfo['shat'][0]:.6g} shat[-1]={pcinfo['shat'][pcinfo['k_eff'] - 1]:.6g}")
    del pc_ref
    fstar_resolved = abs(c_pc.min() - c_pl.min()) <= 1e-6 * abs(fstar)
    kp = k_pc if k_pc is not None else ref_iters
    kq = k_pl if k_pl is not None else ref_iters

    # ---- timed: preconditioned
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        run_pc(P, S, kp, args.power_iters, False)
    torch.cuda.synchronize()
    sk_ms = []
    pcs = []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for s in range(args.steps):
        _, _, _, pc = run_pc(P, S, kp, args.power_iters, False, ev=ev[3 * s:3 * s + 3])
        pcs.append(pc)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_pc = t_start.elapsed_time(t_end) / args.steps
    sk_ms = [ev[3 * s].elapsed_time(ev[3 * s + 1]) for s in range(args.steps)]
    build_ms = [ev[3 * s].elapsed_time(ev[3 * s + 2]) for s in range(args.steps)]
    del pcs

    # ---- timed: plain APG
    for _ in range(args.warmup):
        run_plain(P, S, kq, args.power_iters, False)
    torch.cuda.synchronize()
    t_start.record(stream)
    for s in range(args.steps):
        run_plain(P, S, kq, args.power_iters, False)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_pl = t_start.elapsed_time(t_end) / args.steps
    log(f"preconditioned {ms_pc:.3f} ms ({kp} its), plain {ms_pl:.3f} ms ({kq} its)")

    # ---- roofline of the sketch kernel (algorithmic bytes: Omega in, Y out).
    # Back-to-back launches bracketed by events on the launch stream, so the
    # interval holds kernel time only (no host launch gaps).
    burst = 20
    P.nys_sketch(S.op, S.omega, out=S.Y)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(burst):
        P.nys_sketch(S.op, S.omega, out=S.Y)
    t_end.record(stream)
    torch.cuda.synchronize()
    esz = S.omega.element_size()
    sk_bytes = 2 * wl.ell * S.op.N * esz
    sk_avg_ms = t_start.elapsed_time(t_end) / burst
    achieved = sk_bytes / (sk_avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": sketch_traffic(wl),
            "kernel": "sketch (A^T A Omega)", "bytes_per_launch": sk_bytes,
            "avg_launch_us": round(sk_avg_ms * 1e3, 2),
            "sketch_in_step_us": round(float(np.mean(sk_ms)) * 1e3, 2)}
    roof["measured_copy_peak"] = copy_peak(torch)
    roof["frac_of_copy_peak"] = round(achieved / roof["measured_copy_peak"], 4)

    out = {
        "metric": "time to 1e-4 rel. cost gap, Nystrom-precond WAPG (sketch+factor+step+solve)",
        # when the preconditioned run does not reach the gap within the
        # reference iterations, the time of those iterations (a lower bound)
        "value": round(ms_pc / 1e3, 6),
        "gap_reached": {"precond": k_pc is not None, "plain": k_pl is not None},
        "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_pc, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl.dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "ell": wl.ell, "sketch_dtype": wl.sketch_dtype,
                   "solver_dtype": wl.dtype, "factor_dtype": "f64", "reg": wl.reg,
                   "loss": wl.loss, "lambda": wl.lam, "power_iters": args.power_iters,
                   "tail": args.tail, "seed": args.seed},
        "plain_apg_s": round(ms_pl / 1e3, 6),
        "speedup_vs_plain": round(ms_pl / ms_pc, 4),
        "iters_to_gap": {"precond": k_pc, "plain": k_pl, "reference_iters": ref_iters},
        "fstar": fstar, "fstar_resolved": bool(fstar_resolved),
        "L": {"precond": info_pc["L"], "plain": info_pl["L"]},
        "roofline": roof,
        # building the preconditioner (sketch + factorisation) inside the
        # timed steps, from the stream's events
        "precond_build_s": round(float(np.mean(build_ms)) / 1e3, 6),
    }
    if wl.name in PAPER_BUILD_S:
        out["paper_precond_build_s"] = PAPER_BUILD_S[wl.name]
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(wl, kp, args.power_iters, info_pc["alpha"], args.seed)
        log(f"cpu baseline leg took {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
