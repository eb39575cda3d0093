"""Writes tests/golden/sketch_rule_workloads.json: the effective dimension
d_eff(mu) and the sketch size 2 ceil(1.5 d_eff + 1) of Thm. 2 (Sec. II) for
the Phi = A^T A of the benchmark workloads, over mu = 1e-1 ... 1e-4 times
the largest eigenvalue.  Spectra: closed form for the periodic blur and the
blur followed by 2x decimation (full size); dense eigendecompositions of the
parallel-beam operator on a 64 x 64 stand-in of the CT workload (the views
and bins scaled by 1/8: 90 views, 92 bins), because the 512 x 512 operator
has no closed-form spectrum.  Calls only oracle/ and the input recipes.

    python -m oracle.sketch_rule_table
"""
from __future__ import annotations

import json
import os

import numpy as np

import workloads as W
from oracle import operators as ops
from oracle import sketchsize as sz

MU_REL = (1e-1, 1e-2, 1e-3, 1e-4)
OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests",
                   "golden", "sketch_rule_workloads.json")


def row(name, eigs, note):
    eigs = np.sort(np.clip(np.asarray(eigs, np.float64).ravel(), 0.0, None))[::-1]
    top = float(eigs[0])
    out = {"workload": name, "N": int(eigs.size), "lambda_max": top, "spectrum": note, "rows": []}
    for r in MU_REL:
        d = sz.deff_from_eigs(eigs, r * top)
        out["rows"].append({"mu_over_lambda_max": r, "d_eff": d, "K_rule": sz.sketch_size_rule(d)})
    # the workload's own sketch size: the mu at which the rule gives it
    return out


def table():
    rows = []
    wl = W.workload("deblur128_tv_f64")
    rows.append(row(wl.name, sz.blur_eigs(W.gaussian_psf(wl.psf_k, wl.psf_sigma), wl.n, wl.n),
                    "closed form: |DFT(h)|^2"))
    wl = W.workload("sr512_haar_bf16")
    rows.append(row(wl.name, sz.blurdown_eigs(W.gaussian_psf(wl.psf_k, wl.psf_sigma), wl.n, wl.n,
                                              wl.factor),
                    "closed form: four-alias symbol of A A^T (the nonzero eigenvalues)"))
    for s in W.batch_instances(64, 0)[:8]:
        rows.append(row(f"batch64_deblur_f32 instance seed {s.seed} ({s.n}^2, k {s.psf_k})",
                        sz.blur_eigs(W.gaussian_psf(s.psf_k, s.psf_sigma), s.n, s.n),
                        "closed form: |DFT(h)|^2"))
    n, views, bins = 64, 90, 92
    Phi = sz.dense_phi(lambda x: ops.joseph(x, views, bins), lambda p: ops.joseph_adjoint(p, n), n, n)
    rows.append(row(f"ct512_hs1_f32 stand-in ({n}^2, {views} views, {bins} bins)",
                    np.linalg.eigvalsh(Phi), "dense eigendecomposition"))
    return rows


if __name__ == "__main__":
    t = table()
    with open(OUT, "w") as f:
        json.dump({"source": "oracle/sketch_rule_table.py", "theorem": "Thm. 2 (Sec. II)",
                   "mu_over_lambda_max": list(MU_REL), "workloads": t}, f, indent=1)
    for r in t:
        print(r["workload"], [(x["mu_over_lambda_max"], round(x["d_eff"], 1), x["K_rule"])
                              for x in r["rows"]])
