"""ctypes binding of libnys (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(HERE, "libnys.so")

F64, F32, BF16 = 0, 1, 2
OP_BLUR, OP_BLURDOWN, OP_PARALLEL_BEAM, OP_IDENTITY, OP_FAN_BEAM = 0, 1, 2, 3, 4
REG_TV, REG_TV_ANISO, REG_HS1, REG_L1, REG_HS2, REG_HSINF = 0, 1, 2, 3, 4, 5
LOSS_LS, LOSS_HUBER = 0, 1
REG_NAMES = {"tv": REG_TV, "tv_aniso": REG_TV_ANISO, "hs1": REG_HS1, "l1": REG_L1,
             "hs2": REG_HS2, "hsinf": REG_HSINF}

_STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "ENOTPD", 4: "ENOTFINITE",
           5: "ENOCONV", 6: "EHIP"}


class NysError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class OpDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n1", C.c_int32), ("n2", C.c_int32),
                ("psf_size", C.c_int32), ("psf", C.POINTER(C.c_double)),
                ("factor", C.c_int32), ("n_views", C.c_int32), ("n_bins", C.c_int32),
                ("wavelet_levels", C.c_int32), ("wavelet", C.c_int32),
                ("fan_src", C.c_double), ("fan_det", C.c_double), ("fan_du", C.c_double)]


class FactorOpts(C.Structure):
    _fields_ = [("nu_mode", C.c_int32), ("tail", C.c_int32), ("mu", C.c_double),
                ("max_escalations", C.c_int32), ("u_dtype", C.c_int32)]


class RegDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n1", C.c_int32), ("n2", C.c_int32),
                ("lnorm2", C.c_double), ("n_inner", C.c_int32), ("max_newton", C.c_int32),
                ("newton_tol", C.c_double), ("box", C.c_int32), ("lo", C.c_double),
                ("hi", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("op", C.c_void_p), ("loss", C.c_int32), ("delta", C.c_double),
                ("reg", RegDesc), ("lam", C.c_double), ("y", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("alpha", C.c_double), ("safety", C.c_double),
                ("power_iters", C.c_int32), ("power_v0", C.c_void_p),
                ("warm_start", C.c_int32)]


class UnrollOpts(C.Structure):
    _fields_ = [("n_outer", C.c_int32), ("n_inner", C.c_int32), ("alpha", C.c_double)]


class IrmOpts(C.Structure):
    _fields_ = [("p", C.c_double), ("q", C.c_double), ("eps", C.c_double),
                ("max_outer", C.c_int32), ("outer_tol", C.c_double), ("max_cg", C.c_int32),
                ("cg_tol", C.c_double), ("nu_mode", C.c_int32), ("tail", C.c_int32),
                ("mu", C.c_double)]


class BatchItem(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("psf_k", C.c_int32),
                ("psf", C.POINTER(C.c_double)), ("ell", C.c_int32), ("lam", C.c_double),
                ("y", C.c_void_p), ("omega", C.c_void_p), ("v0", C.c_void_p),
                ("x", C.c_void_p), ("costs", C.c_void_p)]


class BatchOpts(C.Structure):
    _fields_ = [("reg", C.c_int32), ("max_iter", C.c_int32), ("n_inner", C.c_int32),
                ("power_iters", C.c_int32), ("precondition", C.c_int32),
                ("warm_start", C.c_int32), ("nu_mode", C.c_int32), ("tail", C.c_int32),
                ("mu", C.c_double), ("safety", C.c_double), ("tune", C.c_int32)]


_lib = None


def lib():
    """Load libnys.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise NysError(6, f"{library_path} is missing: build it with "
                              "`python -m paper_2411_08178_amd.build`")
        L = C.CDLL(library_path)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "nys_op_create": [C.POINTER(OpDesc), C.POINTER(vp)],
            "nys_op_shape": [vp, C.POINTER(i64), C.POINTER(i64)],
            "nys_op_workspace_size": [vp, i32, i64, C.POINTER(C.c_size_t)],
            "nys_sketch_workspace_size": [vp, i32, i64, C.POINTER(C.c_size_t)],
            "nys_factor_workspace_size": [i64, i64, C.POINTER(C.c_size_t)],
            "nys_apply_workspace_size": [vp, i64, C.POINTER(C.c_size_t)],
            "nys_pnorm2_workspace_size": [vp, i64, i32, C.POINTER(C.c_size_t)],
            "nys_prox_workspace_size": [C.POINTER(RegDesc), vp, i32, C.POINTER(C.c_size_t)],
            "nys_workspace_size": [C.POINTER(Problem), vp, i32, C.POINTER(C.c_size_t)],
            "nys_cost_workspace_size": [C.POINTER(Problem), i32, C.POINTER(C.c_size_t)],
            "irm_workspace_size": [C.POINTER(Problem), i32, i64, C.POINTER(C.c_size_t)],
            "op_forward": [vp, i32, vp, vp, i64, vp, C.c_size_t, vp],
            "op_adjoint": [vp, i32, vp, vp, i64, vp, C.c_size_t, vp],
            "nys_sketch": [vp, i32, vp, vp, i64, vp, C.c_size_t, vp],
            "nys_factor": [vp, vp, i32, i64, i64, C.POINTER(FactorOpts), vp, C.c_size_t,
                           C.POINTER(vp), vp],
            "nys_pc_info": [vp, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(i32), C.POINTER(i32), vp],
            "nys_pc_u": [vp, C.POINTER(vp), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                         C.POINTER(i32)],
            "nys_pc_diag": [vp, C.POINTER(dbl), i32, vp],
            "nys_pc_copy_u": [vp, vp, vp],
            "nys_apply": [vp, i32, i32, vp, vp, i64, vp, C.c_size_t, vp],
            "nys_pnorm2": [vp, i64, i32, i32, vp, vp, vp, vp, C.c_size_t, vp],
            "prox_weighted": [C.POINTER(RegDesc), dbl, vp, i32, vp, vp, vp, vp, C.c_size_t, vp],
            "nys_prox_state_bytes": [C.POINTER(RegDesc), vp, i32, C.POINTER(C.c_size_t)],
            "solve": [C.POINTER(Problem), vp, i32, C.POINTER(SolveOpts), vp, vp,
                      C.POINTER(dbl), vp, C.c_size_t, vp],
            "nys_cost": [C.POINTER(Problem), i32, vp, vp, vp, C.c_size_t, vp],
            "nys_solve_plan_create": [C.POINTER(Problem), vp, i32, C.POINTER(SolveOpts), vp, vp,
                                      vp, C.c_size_t, vp, C.POINTER(dbl), C.POINTER(vp)],
            "nys_solve_plan_run": [vp, vp],
            "nys_unrolled_workspace": [C.POINTER(Problem), vp, i32, C.POINTER(UnrollOpts), i32,
                                       C.POINTER(C.c_size_t)],
            "unrolled_forward": [C.POINTER(Problem), vp, i32, C.POINTER(UnrollOpts), i32, vp,
                                 C.POINTER(dbl), vp, vp, C.c_size_t, vp],
            "unrolled_backward": [C.POINTER(Problem), vp, i32, C.POINTER(UnrollOpts), i32, vp,
                                  C.POINTER(dbl), vp, vp, C.POINTER(dbl), vp, C.c_size_t, vp],
            "irm_solve": [C.POINTER(Problem), i32, C.POINTER(IrmOpts), vp, i64, vp, vp,
                          C.POINTER(i32), C.POINTER(i32), C.POINTER(dbl), vp, C.c_size_t, vp],
            "batch_solve_create": [C.POINTER(BatchItem), i32, C.POINTER(BatchOpts),
                                   C.POINTER(vp), vp],
            "batch_solve_run": [vp, vp],
            "batch_solve_sketch": [vp, vp],
            "batch_solve_info": [vp, i32, C.POINTER(dbl), vp],
            "batch_solve_shat": [vp, i32, C.POINTER(dbl), vp],
            "batch_solve_buffers": [vp, i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(i64)],
            "batch_solve_copy": [vp, i32, i32, vp, vp],
            "batch_solve_tiles": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), i32,
                                  C.POINTER(i32)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.nys_op_destroy.argtypes = [vp]
        L.nys_op_destroy.restype = None
        L.nys_pc_destroy.argtypes = [vp]
        L.nys_pc_destroy.restype = None
        L.batch_solve_destroy.argtypes = [vp]
        L.batch_solve_destroy.restype = None
        L.nys_solve_plan_destroy.argtypes = [vp]
        L.nys_solve_plan_destroy.restype = None
        L.nys_last_error.restype = C.c_char_p
        L.nys_version.restype = C.c_char_p
        _lib = L
    return _lib


def version() -> str:
    return lib().nys_version().decode()


def _check(status: int):
    if status != 0:
        raise NysError(status, lib().nys_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_DT = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}


def _dt(t: torch.Tensor) -> int:
    if t.dtype not in _DT:
        raise NysError(1, f"unsupported dtype {t.dtype}")
    return _DT[t.dtype]


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise NysError(1, "tensors must be contiguous CUDA (HIP) tensors")
    return C.c_void_p(t.data_ptr())


def _workspace(query, *args):
    """A device workspace of the size the library's query returns: (tensor or
    None, pointer, bytes).  Allocated by torch on the current stream (the
    library allocates nothing per call); 256-byte aligned."""
    nb = C.c_size_t()
    _check(query(*args, C.byref(nb)))
    if nb.value == 0:
        return None, None, 0
    t = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    off = (-t.data_ptr()) % 256
    return t, C.c_void_p(t.data_ptr() + off), nb.value


class Operator:
    """Handle of an operator A (optionally composed with Haar synthesis)."""

    def __init__(self, kind: int, n1: int, n2: int, psf=None, factor: int = 1,
                 views: int = 0, bins: int = 0, wavelet_levels: int = 0, wavelet: str = "haar",
                 fan=None):
        """fan = (source radius, detector radius, bin spacing) in pixels (OP_FAN_BEAM)."""
        d = OpDesc()
        d.kind, d.n1, d.n2 = kind, n1, n2
        self._psf = None
        if psf is not None:
            self._psf = np.ascontiguousarray(psf, dtype=np.float64)
            d.psf_size = self._psf.shape[0]
            d.psf = self._psf.ctypes.data_as(C.POINTER(C.c_double))
        d.factor, d.n_views, d.n_bins, d.wavelet_levels = factor, views, bins, wavelet_levels
        d.wavelet = {"haar": 0, "db4": 1}[wavelet]
        if fan is not None:
            d.fan_src, d.fan_det, d.fan_du = (float(v) for v in fan)
        h = C.c_void_p()
        _check(lib().nys_op_create(C.byref(d), C.byref(h)))
        self.handle = h
        N, M = C.c_int64(), C.c_int64()
        _check(lib().nys_op_shape(h, C.byref(N), C.byref(M)))
        self.N, self.M = N.value, M.value
        self.n1, self.n2 = n1, n2
        self.kind = kind
        self.views, self.bins, self.factor = views, bins, factor

    @property
    def meas_shape(self):
        if self.kind in (OP_PARALLEL_BEAM, OP_FAN_BEAM):
            return (self.views, self.bins)
        if self.kind == OP_BLURDOWN:
            return (self.n1 // self.factor, self.n2 // self.factor)
        return (self.n1, self.n2)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.nys_op_destroy(self.handle)
            self.handle = None


def _ncols(t: torch.Tensor, per: int) -> int:
    if t.numel() % per:
        raise NysError(1, f"tensor of {t.numel()} elements is not a stack of {per}")
    return t.numel() // per


def op_forward(op: Operator, x: torch.Tensor, out: Optional[torch.Tensor] = None):
    n = _ncols(x, op.N)
    lead = x.shape[:-2] if x.dim() >= 2 and x.shape[-2:] == (op.n1, op.n2) else (n,)
    if out is None:
        out = torch.empty(tuple(lead) + op.meas_shape, dtype=x.dtype, device=x.device)
    ws, wp, wb = _workspace(lib().nys_op_workspace_size, op.handle, _dt(x), n)
    _check(lib().op_forward(op.handle, _dt(x), _ptr(x), _ptr(out), n, wp, wb, _stream()))
    return out


def op_adjoint(op: Operator, y: torch.Tensor, out: Optional[torch.Tensor] = None):
    n = _ncols(y, op.M)
    lead = y.shape[:-2] if y.dim() >= 2 else (n,)
    if out is None:
        out = torch.empty(tuple(lead) + (op.n1, op.n2), dtype=y.dtype, device=y.device)
    ws, wp, wb = _workspace(lib().nys_op_workspace_size, op.handle, _dt(y), n)
    _check(lib().op_adjoint(op.handle, _dt(y), _ptr(y), _ptr(out), n, wp, wb, _stream()))
    return out


def nys_sketch(op: Operator, omega: torch.Tensor, out: Optional[torch.Tensor] = None):
    ell = _ncols(omega, op.N)
    if out is None:
        out = torch.empty_like(omega)
    ws, wp, wb = _workspace(lib().nys_sketch_workspace_size, op.handle, _dt(omega), ell)
    _check(lib().nys_sketch(op.handle, _dt(omega), _ptr(omega), _ptr(out), ell, wp, wb,
                            _stream()))
    return out


class Preconditioner:
    """Handle of the Nystrom preconditioner (U, spectrum, coefficients)."""

    def __init__(self, handle, N, ell, u_dtype):
        self.handle, self.N, self.ell = handle, N, ell
        self.u_dtype = torch.float64 if u_dtype == F64 else torch.float32

    def info(self):
        shat = (C.c_double * self.ell)()
        nu = C.c_double()
        keff = C.c_int32()
        st = C.c_int32()
        _check(lib().nys_pc_info(self.handle, shat, C.byref(nu), C.byref(keff), C.byref(st),
                                 _stream()))
        return dict(shat=np.array(shat[:]), nu=nu.value, k_eff=keff.value, status=st.value)

    def diag(self):
        out = (C.c_double * 16)()
        _check(lib().nys_pc_diag(self.handle, out, 16, _stream()))
        v = list(out)
        return dict(nu=v[0], s_tail=v[1], mu=v[2], pinv_norm=v[3], k_eff=int(v[4]),
                    status=int(v[5]), escalations=int(v[6]), sweeps_shift=int(v[7]),
                    sweeps_eig=int(v[8]), stamps=v[9:16])

    def U(self) -> torch.Tensor:
        out = torch.empty((self.ell, self.N), dtype=self.u_dtype, device="cuda")
        _check(lib().nys_pc_copy_u(self.handle, _ptr(out), _stream()))
        return out

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.nys_pc_destroy(self.handle)
            self.handle = None


def nys_factor(omega: torch.Tensor, Y: torch.Tensor, ell: int, nu_mode: int = 0,
               tail: str = "sqrt", mu: float = -1.0, max_escalations: int = 6,
               u_dtype: torch.dtype = torch.float32) -> Preconditioner:
    if omega.shape != Y.shape or omega.dtype != Y.dtype:
        raise NysError(1, "omega and Y must have the same shape and dtype")
    N = omega.numel() // ell
    o = FactorOpts(nu_mode, 0 if tail == "sqrt" else 1, mu, max_escalations, _DT[u_dtype])
    h = C.c_void_p()
    ws, wp, wb = _workspace(lib().nys_factor_workspace_size, N, ell)
    _check(lib().nys_factor(_ptr(omega), _ptr(Y), _dt(omega), N, ell, C.byref(o), wp, wb,
                            C.byref(h), _stream()))
    return Preconditioner(h, N, ell, _DT[u_dtype])


def nys_apply(pc: Preconditioner, v: torch.Tensor, inverse: bool = True,
              out: Optional[torch.Tensor] = None):
    n = _ncols(v, pc.N)
    if out is None:
        out = torch.empty_like(v)
    ws, wp, wb = _workspace(lib().nys_apply_workspace_size, pc.handle, n)
    _check(lib().nys_apply(pc.handle, 1 if inverse else 0, _dt(v), _ptr(v), _ptr(out), n,
                           wp, wb, _stream()))
    return out


def pnorm2(pc: Optional[Preconditioner], a: torch.Tensor, b: Optional[torch.Tensor] = None,
           inverse: bool = False) -> float:
    """(a - b)^T P (a - b) (P^{-1} with inverse; P = I without a pc), FP64."""
    n = a.numel()
    if b is not None and (b.shape != a.shape or b.dtype != a.dtype):
        raise ValueError("pnorm2: a and b must share shape and dtype")
    out = torch.empty(1, dtype=torch.float64, device=a.device)
    h = pc.handle if pc is not None else None
    ws, wp, wb = _workspace(lib().nys_pnorm2_workspace_size, h, n, _dt(a))
    _check(lib().nys_pnorm2(h, n, 1 if inverse else 0, _dt(a), _ptr(a),
                            _ptr(b) if b is not None else None, _ptr(out), wp, wb, _stream()))
    return float(out.item())


def rate_constant(op, y, reg, lam, pc: Optional[Preconditioner], x_star: torch.Tensor,
                  x1: Optional[torch.Tensor] = None, power_iters: int = 100,
                  power_v0: Optional[torch.Tensor] = None, loss: int = 0, delta: float = 0.0):
    """L_f^P ||x^1 - x*||_P^2, the constant of WAPG's rate bound (the cost gap
    after k iterations is at most twice it over (k + 1)^2).  x^1 is the
    start (zero by default, as the solver starts); L_f^P from the solver's
    power method; returns dict(L, pdist2, value)."""
    _, _, info = solve(op, y, reg, lam, pc, 1, power_v0=power_v0, power_iters=power_iters,
                       loss=loss, delta=delta, record_cost=False)
    d2 = pnorm2(pc, x_star.contiguous(), x1.contiguous() if x1 is not None else None)
    return dict(L=info["L"], pdist2=d2, value=info["L"] * d2)


def reg_desc(kind, n1, n2, n_inner=20, lnorm2=0.0, max_newton=0, newton_tol=0.0,
             box=None) -> RegDesc:
    """box = (lo, hi) restricts x to C = {lo <= x <= hi} (TV and Hessian kinds)."""
    if isinstance(kind, str):
        kind = REG_NAMES[kind]
    lo, hi = box if box is not None else (0.0, 0.0)
    return RegDesc(kind, n1, n2, lnorm2, n_inner, max_newton, newton_tol,
                   1 if box is not None else 0, float(lo), float(hi))


def prox_state(reg: RegDesc, pc: Optional[Preconditioner], dtype) -> Optional[torch.Tensor]:
    """Zero-initialised warm-start state for prox_weighted."""
    nb = C.c_size_t()
    _check(lib().nys_prox_state_bytes(C.byref(reg), pc.handle if pc else None, _DT[dtype],
                                      C.byref(nb)))
    if nb.value == 0:
        return None
    return torch.zeros(nb.value, dtype=torch.uint8, device="cuda")


def prox_weighted(reg: RegDesc, lam_bar: float, pc: Optional[Preconditioner], s: torch.Tensor,
                  state: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None):
    if out is None:
        out = torch.empty_like(s)
    h = pc.handle if pc else None
    ws, wp, wb = _workspace(lib().nys_prox_workspace_size, C.byref(reg), h, _dt(s))
    _check(lib().prox_weighted(C.byref(reg), lam_bar, h, _dt(s), _ptr(s), _ptr(out), _ptr(state),
                               wp, wb, _stream()))
    return out


def _problem(op: Operator, y: torch.Tensor, reg: RegDesc, lam: float, loss: int, delta: float):
    p = Problem()
    p.op = op.handle
    p.loss, p.delta, p.reg, p.lam = loss, delta, reg, lam
    p.y = y.data_ptr()
    return p


def solve(op: Operator, y: torch.Tensor, reg: RegDesc, lam: float, pc: Optional[Preconditioner],
          max_iter: int, alpha: float = -1.0, power_v0: Optional[torch.Tensor] = None,
          power_iters: int = 100, safety: float = 1.01, loss: int = LOSS_LS, delta: float = 0.0,
          warm_start: bool = True, record_cost: bool = True):
    """WAPG (plain APG when pc is None).  Returns (x, costs or None, info)."""
    p = _problem(op, y, reg, lam, loss, delta)
    o = SolveOpts(max_iter, alpha, safety, power_iters,
                  power_v0.data_ptr() if power_v0 is not None else None,
                  1 if warm_start else 0)
    x = torch.empty((op.n1, op.n2), dtype=y.dtype, device=y.device)
    costs = torch.empty(max(max_iter, 1), dtype=torch.float64, device=y.device) if record_cost else None
    info = (C.c_double * 8)()
    h = pc.handle if pc else None
    ws, wp, wb = _workspace(lib().nys_workspace_size, C.byref(p), h, _dt(y))
    _check(lib().solve(C.byref(p), h, _dt(y), C.byref(o), _ptr(x), _ptr(costs), info, wp, wb,
                       _stream()))
    return x, costs, dict(alpha=info[0], L=info[1], status=int(info[2]))


class SolvePlan:
    """`solve` captured once as HIP graphs (nys_solve_plan_*): run() replays
    the whole fixed-count iteration on the current stream with no host work
    inside the loop, into the tensors x and costs it owns (like its inputs,
    they keep their addresses while the plan lives)."""

    def __init__(self, op: Operator, y: torch.Tensor, reg: RegDesc, lam: float,
                 pc: Optional[Preconditioner], max_iter: int, alpha: float = -1.0,
                 power_v0: Optional[torch.Tensor] = None, power_iters: int = 100,
                 safety: float = 1.01, loss: int = LOSS_LS, delta: float = 0.0,
                 warm_start: bool = True, record_cost: bool = True):
        self.handle = None
        self._keep = (op, y, pc, power_v0)
        self._p = _problem(op, y, reg, lam, loss, delta)
        o = SolveOpts(max_iter, alpha, safety, power_iters,
                      power_v0.data_ptr() if power_v0 is not None else None,
                      1 if warm_start else 0)
        self.x = torch.empty((op.n1, op.n2), dtype=y.dtype, device=y.device)
        self.costs = (torch.empty(max(max_iter, 1), dtype=torch.float64, device=y.device)
                      if record_cost else None)
        h = pc.handle if pc else None
        self._ws, wp, wb = _workspace(lib().nys_workspace_size, C.byref(self._p), h, _dt(y))
        self._ws_ptr = wp.value if wp is not None else 0
        info = (C.c_double * 8)()
        out = C.c_void_p()
        _check(lib().nys_solve_plan_create(C.byref(self._p), h, _dt(y), C.byref(o), _ptr(self.x),
                                           _ptr(self.costs), wp, wb, _stream(), info,
                                           C.byref(out)))
        self.handle = out.value
        self.info = dict(alpha=info[0], L=info[1])

    def run(self):
        _check(lib().nys_solve_plan_run(self.handle, _stream()))
        return self.x, self.costs

    def status(self) -> int:
        """The status of the last run (synchronises): the first device status
        word (NYS_ENOTFINITE), else the second (NYS_ENOCONV: an l1 prox that
        did not converge within its captured trials)."""
        if self._ws is None:
            return 0
        off = self._ws_ptr - self._ws.data_ptr()
        w = self._ws[off:off + 8].view(torch.int32).tolist()
        return int(w[0] or w[1])

    def __del__(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize()
            lib().nys_solve_plan_destroy(self.handle)
            self.handle = None


def nys_cost(op: Operator, y: torch.Tensor, reg: RegDesc, lam: float, x: torch.Tensor,
             loss: int = LOSS_LS, delta: float = 0.0) -> torch.Tensor:
    p = _problem(op, y, reg, lam, loss, delta)
    out = torch.empty(1, dtype=torch.float64, device=x.device)
    ws, wp, wb = _workspace(lib().nys_cost_workspace_size, C.byref(p), _dt(x))
    _check(lib().nys_cost(C.byref(p), _dt(x), _ptr(x), _ptr(out), wp, wb, _stream()))
    return out


# ---------------------------------------------------------------- autograd
class OpForwardFn(torch.autograd.Function):
    """y = A x; the backward applies the hand-written adjoint kernel A^T."""

    @staticmethod
    def forward(ctx, x, op):
        ctx.op = op
        return op_forward(op, x.contiguous())

    @staticmethod
    def backward(ctx, gy):
        return op_adjoint(ctx.op, gy.contiguous()), None


class OpAdjointFn(torch.autograd.Function):
    """x = A^T y; the backward applies A."""

    @staticmethod
    def forward(ctx, y, op):
        ctx.op = op
        return op_adjoint(op, y.contiguous())

    @staticmethod
    def backward(ctx, gx):
        return op_forward(ctx.op, gx.contiguous()), None


class PinvFn(torch.autograd.Function):
    """P^{-1} v; P^{-1} is symmetric, so the backward applies it again."""

    @staticmethod
    def forward(ctx, v, pc):
        ctx.pc = pc
        return nys_apply(pc, v.contiguous(), inverse=True)

    @staticmethod
    def backward(ctx, g):
        return nys_apply(ctx.pc, g.contiguous(), inverse=True), None


class UnrolledWAPGFn(torch.autograd.Function):
    """K unrolled WAPG iterations with the P-weighted TV prox (`unrolled_forward`
    / `unrolled_backward` of the C ABI); gradients w.r.t. y and lambda."""

    @staticmethod
    def forward(ctx, y, lam, op, reg, pc, n_outer, n_inner, alpha):
        batch = y.shape[0]
        y = y.contiguous()
        lam_h = lam.detach().to("cpu", torch.float64).contiguous()
        p = _problem(op, y, reg, 1.0, LOSS_LS, 0.0)
        o = UnrollOpts(n_outer, n_inner, alpha)
        nb = C.c_size_t()
        _check(lib().nys_unrolled_workspace(C.byref(p), pc.handle if pc else None, _dt(y),
                                            C.byref(o), batch, C.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device=y.device)
        if ws.data_ptr() % 256:
            raise NysError(1, "unrolled workspace is not 256-byte aligned")
        x = torch.empty((batch, op.n1, op.n2), dtype=y.dtype, device=y.device)
        lam_p = lam_h.numpy().ctypes.data_as(C.POINTER(C.c_double))
        _check(lib().unrolled_forward(C.byref(p), pc.handle if pc else None, _dt(y), C.byref(o),
                                      batch, _ptr(y), lam_p, _ptr(x), _ptr(ws), nb.value,
                                      _stream()))
        ctx.save_for_backward(y)
        ctx.args = (op, reg, pc, o, lam_h, ws, lam.dtype, lam.device)
        return x

    @staticmethod
    def backward(ctx, gx):
        (y,) = ctx.saved_tensors
        op, reg, pc, o, lam_h, ws, ldt, ldev = ctx.args
        batch = y.shape[0]
        p = _problem(op, y, reg, 1.0, LOSS_LS, 0.0)
        gy = torch.empty_like(y)
        glam = (C.c_double * batch)()
        lam_p = lam_h.numpy().ctypes.data_as(C.POINTER(C.c_double))
        _check(lib().unrolled_backward(C.byref(p), pc.handle if pc else None, _dt(y), C.byref(o),
                                       batch, _ptr(y), lam_p, _ptr(gx.contiguous()), _ptr(gy),
                                       glam, _ptr(ws), ws.numel(), _stream()))
        gl = torch.tensor(list(glam), dtype=ldt, device=ldev)
        return gy, gl, None, None, None, None, None, None


def unrolled_wapg(op: Operator, y: torch.Tensor, lam: torch.Tensor, reg: RegDesc,
                  pc: Optional[Preconditioner], n_outer: int, n_inner: int, alpha: float):
    """x (batch, n1, n2) = unrolled WAPG on y (batch, *meas_shape) with weights
    lam (batch,); differentiable w.r.t. y and lam."""
    return UnrolledWAPGFn.apply(y, lam, op, reg, pc, n_outer, n_inner, alpha)


class BatchSolver:
    """Plan of many periodic-blur reconstructions solved in one graph launch.

    items: list of dicts with keys psf (k x k numpy float64, separable),
    y (n1 x n2 float32 CUDA tensor), lam, v0 (n1 x n2 float32), and, when
    precondition is true, ell and omega (ell x n1 x n2 float32).  Outputs
    x[i] (float32) and, with record_costs, costs[i] (float64, max_iter).
    The plan keeps references to every tensor it reads or writes.
    """

    def __init__(self, items, reg: int = REG_TV, max_iter: int = 100, n_inner: int = 20,
                 power_iters: int = 100, precondition: bool = True, warm_start: bool = True,
                 nu_mode: int = 0, tail: int = 0, mu: float = -1.0, safety: float = 1.01,
                 tune: bool = True, record_costs: bool = False):
        self.handle = None
        self._keep = []
        self.x, self.costs = [], []
        arr = (BatchItem * len(items))()
        for i, it in enumerate(items):
            y = it["y"]
            n1, n2 = y.shape
            psf = np.ascontiguousarray(it["psf"], dtype=np.float64)
            x = torch.empty_like(y)
            c = (torch.zeros(max_iter, dtype=torch.float64, device=y.device)
                 if record_costs else None)
            om = it.get("omega") if precondition else None
            self._keep += [psf, y, it["v0"], x, c, om]
            self.x.append(x)
            self.costs.append(c)
            arr[i].n1, arr[i].n2 = n1, n2
            arr[i].psf_k = psf.shape[0]
            arr[i].psf = psf.ctypes.data_as(C.POINTER(C.c_double))
            arr[i].ell = int(it.get("ell", 0)) if precondition else 0
            arr[i].lam = float(it["lam"])
            arr[i].y = _ptr(y)
            arr[i].omega = _ptr(om)
            arr[i].v0 = _ptr(it["v0"])
            arr[i].x = _ptr(x)
            arr[i].costs = _ptr(c)
        o = BatchOpts(reg, max_iter, n_inner, power_iters, int(precondition), int(warm_start),
                      nu_mode, tail, mu, safety, int(tune))
        h = C.c_void_p()
        _check(lib().batch_solve_create(arr, len(items), C.byref(o), C.byref(h), _stream()))
        self.handle = h
        self.count = len(items)

    def run(self):
        _check(lib().batch_solve_run(self.handle, _stream()))
        return self.x

    def sketch_only(self):
        """Enqueue only the sketches of every instance (first step of run)."""
        _check(lib().batch_solve_sketch(self.handle, _stream()))

    def info(self, i: int):
        out = (C.c_double * 6)()
        _check(lib().batch_solve_info(self.handle, i, out, _stream()))
        return dict(alpha=out[0], L=out[1], pinv_norm=out[2], nu=out[3], status=int(out[4]),
                    k_eff=int(out[5]))

    def shat(self, i: int, ell: int):
        out = (C.c_double * ell)()
        _check(lib().batch_solve_shat(self.handle, i, out, _stream()))
        return np.array(out[:], dtype=np.float64)

    def sketch(self, i: int, n1: int, n2: int, ell: int):
        """(Y, U) of instance i copied out: ell x n1 x n2 and ell x N, float32."""
        dev = self.x[i].device
        Y = torch.empty(ell, n1, n2, dtype=torch.float32, device=dev)
        U = torch.empty(ell, n1 * n2, dtype=torch.float32, device=dev)
        _check(lib().batch_solve_copy(self.handle, i, 0, _ptr(Y), _stream()))
        _check(lib().batch_solve_copy(self.handle, i, 1, _ptr(U), _stream()))
        return Y, U

    def tiles(self):
        cap = 64
        a, b, c = (C.c_int32 * cap)(), (C.c_int32 * cap)(), (C.c_int32 * cap)()
        n = C.c_int32()
        _check(lib().batch_solve_tiles(self.handle, a, b, c, cap, C.byref(n)))
        return [(a[i], b[i], c[i]) for i in range(min(n.value, cap))]

    def __del__(self):
        if self.handle is not None and _lib is not None:
            _lib.batch_solve_destroy(self.handle)
            self.handle = None


def irm_solve(op: Operator, y: torch.Tensor, lam: float, p: float = 1.0, q: float = 1.0,
              eps: float = 1e-6, max_outer: int = 20, outer_tol: float = 0.0,
              max_cg: int = 1000, cg_tol: float = 1e-4, omega: Optional[torch.Tensor] = None,
              x0: Optional[torch.Tensor] = None, tail: str = "plain", mu: float = -1.0,
              nu_mode: int = 0, return_info: bool = False):
    """l_p - l_q reconstruction by Alg. 2 (CG, or Nystrom-PCG when omega is
    given).  Returns (x, cg_iterations_per_outer_iteration)."""
    dt = _dt(y)
    n1, n2 = op.n1, op.n2
    x = torch.empty((n1, n2), dtype=y.dtype, device=y.device)
    rd = reg_desc("tv_aniso", n1, n2)
    prob = _problem(op, y, rd, lam, LOSS_LS, 0.0)
    o = IrmOpts(p, q, eps, max_outer, outer_tol, max_cg, cg_tol, nu_mode,
                0 if tail == "sqrt" else 1, mu)
    its = (C.c_int32 * max_outer)()
    info = (C.c_double * (3 * max_outer))()
    done = C.c_int32()
    ell = 0 if omega is None else omega.shape[0]
    ws, wp, wb = _workspace(lib().irm_workspace_size, C.byref(prob), dt, ell)
    _check(lib().irm_solve(C.byref(prob), dt, C.byref(o), _ptr(omega), ell, _ptr(x0), _ptr(x),
                           its, C.byref(done), info, wp, wb, _stream()))
    if return_info:
        fac = [dict(status=int(info[3 * i]), k_eff=int(info[3 * i + 1]), nu=info[3 * i + 2])
               for i in range(done.value)] if ell else []
        return x, [its[i] for i in range(done.value)], fac
    return x, [its[i] for i in range(done.value)]
