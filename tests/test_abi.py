"""The C-ABI library loads on the CPU and exports every symbol nys.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nys.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:nys_status|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["op_forward", "op_adjoint", "nys_sketch", "nys_factor", "nys_apply",
                     "prox_weighted", "solve"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2411_08178_amd as P
    lib = ctypes.CDLL(P.library_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert P.version().startswith("nys-mi355x")


def test_host_side_argument_errors_without_a_device():
    """Argument checks and size queries run on the host: they answer without a
    GPU and never enqueue anything."""
    import paper_2411_08178_amd as P
    lib = ctypes.CDLL(P.library_path)
    lib.nys_last_error.restype = ctypes.c_char_p
    nb = ctypes.c_size_t()
    # Alg. 1 scratch: Gram partials, the 2 ell x 2 ell Gram, 5 ell^2 + ell matrices
    assert lib.nys_factor_workspace_size(ctypes.c_int64(16384), ctypes.c_int64(32),
                                         ctypes.byref(nb)) == 0
    assert nb.value >= 8 * (64 * 64 + 5 * 32 * 32 + 32)
    assert lib.nys_factor_workspace_size(ctypes.c_int64(16384), ctypes.c_int64(129),
                                         ctypes.byref(nb)) == 1           # ell > 128
    assert b"bad argument" in lib.nys_last_error()
    # a null operator handle is refused before any device work
    assert lib.op_forward(None, 1, None, None, ctypes.c_int64(1), None, ctypes.c_size_t(0),
                          None) == 1
    assert lib.nys_sketch(None, 1, None, None, ctypes.c_int64(1), None, ctypes.c_size_t(0),
                          None) == 1
