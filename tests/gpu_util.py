"""Helpers shared by the GPU parity tests (host-side marshalling only)."""
import sys

import numpy as np
import pytest
import torch

import workloads as W

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 2e-3}
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


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()
