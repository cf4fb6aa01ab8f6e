"""The C-ABI library loads and exports every function include/dalia.h
declares (no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dalia.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(
        r"^\s*(?:dl_status|void|int32_t|size_t|const char\*)\s+(\w+)\s*\(",
        src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("bta_assemble", "bta_factor", "bta_solve", "bta_selinv",
                 "fobj_eval", "dl_model_create", "dl_ws_create"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2507_06938_amd import build as B
    if not os.path.exists(B.LIB):
        B.build(verbose=False)
    lib = ctypes.CDLL(B.LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.dl_theta_dim(1) == 4 and lib.dl_theta_dim(3) == 15
