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


def test_header_is_plain_c(tmp_path):
    """The boundary header compiles as C99 and as C++ with no HIP or torch
    headers, and its structs have the layout the binding marshals."""
    import shutil
    import subprocess
    import paper_1508_06103_amd as st
    src = tmp_path / "abi.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "stkkt.h"\n'
                   "int main(void) {\n"
                   '  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(kkt_problem_t), offsetof(kkt_problem_t, regularization),\n'
                   "         sizeof(ras_params_t), sizeof(coarse_params_t), sizeof(solve_params_t), sizeof(kkt_stats_t),\n"
                   "         sizeof(server_params_t));\n"
                   "  return 0;\n}\n")
    inc = os.path.join(ROOT, "include")
    cc = shutil.which("gcc") or shutil.which("cc")
    exe = tmp_path / "abi"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), "-o", str(exe)], check=True)
    cxx = shutil.which("g++")
    if cxx:
        subprocess.run([cxx, "-x", "c++", "-std=c++17", "-Wall", "-Werror", "-fsyntax-only", "-I", inc, str(src)],
                       check=True)
    sizes = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(st._Problem), st._Problem.regularization.offset, ctypes.sizeof(st._RasParams),
            ctypes.sizeof(st._CoarseParams), ctypes.sizeof(st._SolveParams), ctypes.sizeof(st._Stats),
            ctypes.sizeof(st._ServerParams)]
    assert sizes == want
