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
