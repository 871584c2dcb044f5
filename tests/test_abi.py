"""The C-ABI library loads and exports every entry point the header declares (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "stkkt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = "\n".join(l for l in text.splitlines() if "typedef" not in l)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if not n.startswith("STKKT")))


def test_header_declares_the_method_calls():
    names = declared_functions()
    for n in ["kkt_assemble", "kkt_matvec", "ras_setup", "ras_apply", "coarse_setup", "kkt_solve"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1508_06103_amd as st
    lib = ctypes.CDLL(st.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) <= set(st.EXPORTED)


def test_error_path_without_gpu():
    """A NULL problem is rejected before any device call, with a message."""
    import paper_1508_06103_amd as st
    h = ctypes.c_void_p()
    rc = st._lib.kkt_assemble(None, None, None, ctypes.byref(h), None)
    assert rc == st.EINVAL
    assert b"NULL" in st._lib.kkt_last_error()
