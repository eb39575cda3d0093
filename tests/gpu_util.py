"""Helpers shared by the GPU parity tests (host-side marshalling only)."""
import os
import sys

import numpy as np
import pytest
import torch

import workloads as W

# stated tolerances: FP64 steps, FP32 steps, BF16 sketches (and whatever is
# computed from BF16 inputs)
TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 2e-3}
# element-wise bound of results rounded to bfloat16 once: its unit roundoff
# 2^-8 relative to each value (so at most 2^-8 max|ref|), plus FP32 accumulation
BF16_ELEM = 2.0 ** -8 + 1e-5
TDT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_08178_amd as P
    P.lib()  # raises loudly if the HIP library is missing
    return P


def dev(a, dt="f64"):
    """Round a float64 array to dtype dt and move it to the GPU."""
    r = W.round_dtype(np.asarray(a, np.float64), dt)
    return torch.from_numpy(r).to(TDT[dt]).cuda().contiguous()


def host(t):
    return t.detach().float().cpu().double().numpy() if t.dtype == torch.bfloat16 \
        else t.detach().cpu().double().numpy()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def elem(a, b):
    """max |a - b| / max |b|: the element-wise companion of rel()."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


def check(got, want, tol, elem_tol=None, what=""):
    """Asserts rel(got, want) <= tol and max|got - want| <= elem_tol max|want|
    (elem_tol defaults to tol), after printing both measured errors."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    et = tol if elem_tol is None else elem_tol
    r, e = rel(got, want), elem(got, want)
    name = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0].split("::")[-1]
    print(f"[parity] {name} {what}: rel {r:.2e} (tol {tol:.0e}) elem {e:.2e} (tol {et:.0e})",
          flush=True)
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    assert r <= tol, f"{what}: rel {r:.3e} > {tol:.1e}"
    assert e <= et, f"{what}: elem {e:.3e} > {et:.1e}"
    return r, e


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()
