"""MI355X (gfx950) Nystrom-preconditioned image reconstruction.

Thin Python binding over the C ABI in include/nys.h (libnys.so, built by
`paper_2411_08178_amd.build`).  Torch tensors provide device memory and the
current stream; every step of the computation runs in the HIP library.  The
binding raises if the library is missing: there is no CPU fallback.
"""
from ._binding import (  # noqa: F401
    NysError, lib, library_path, Operator, Preconditioner, RegDesc,
    op_forward, op_adjoint, nys_sketch, nys_factor, nys_apply, pnorm2, rate_constant,
    prox_weighted, prox_state, reg_desc, solve, SolvePlan, nys_cost, version,
    F64, F32, BF16, OP_BLUR, OP_BLURDOWN, OP_PARALLEL_BEAM, OP_IDENTITY, OP_FAN_BEAM,
    REG_TV, REG_TV_ANISO, REG_HS1, REG_L1, REG_HS2, REG_HSINF, REG_NAMES, LOSS_LS, LOSS_HUBER,
    OpForwardFn, OpAdjointFn, PinvFn, UnrolledWAPGFn, unrolled_wapg, BatchSolver,
    irm_solve,
)
