"""The C-ABI boundary without a GPU: the library loads, exports every function
that include/wd.h declares, the Python binding carries the same names, and the
pure host-side entry points (sizes, status strings, parameter defaults) agree
with the layout the header documents."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wd.h")
LIB = os.path.join(ROOT, "paper_0710_2442_amd", "libwd.so")


def declared_functions():
    s = open(HEADER).read()
    s = re.sub(r"/\*.*?\*/", "", s, flags=re.S)
    s = re.sub(r"//[^\n]*", "", s)
    return sorted(set(re.findall(r"\b(wd_[a-z0-9_]+)\s*\(", s)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libwd.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("wd_dslash", "wd_solve", "wd_gauge_create", "wd_solve_batch", "wd_ptc_train_step",
                 "wd_tune_dslash", "wd_dslash_mrhs", "wd_last_error"):
        assert must in names
    assert len(names) >= 30


def test_library_exports_every_declared_function(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_exports_are_unmangled_c_symbols():
    out = os.popen(f"nm -D --defined-only {LIB}").read()
    defined = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in declared_functions():
        assert n in defined, n


def test_python_binding_has_the_same_names():
    import paper_0710_2442_amd as wd
    missing = [n for n in declared_functions() if not callable(getattr(wd, n, None))]
    assert not missing, missing


def _dims(d):
    return (ctypes.c_int * 4)(*d)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (8, 8, 8, 8), (6, 4, 6, 10), (32, 32, 32, 64), (24, 24, 24, 48)])
def test_sizes_follow_the_documented_layout(lib, dims):
    lib.wd_vh_pad.restype = ctypes.c_size_t
    lib.wd_field_bytes.restype = ctypes.c_size_t
    lib.wd_field_bytes.argtypes = [ctypes.c_int * 4, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    vpad = lib.wd_vh_pad(_dims(dims))
    assert vpad % 256 == 0 and vh <= vpad < vh + 256
    per_site = {0: 192, 1: 96, 2: 52, 3: 48}  # F64, F32, F16 (+scale), BF16
    for prec, b in per_site.items():
        half = lib.wd_field_bytes(_dims(dims), prec, 1, 0)
        assert half == b * vpad
        assert lib.wd_field_bytes(_dims(dims), prec, 1, 2) == 2 * half
        assert lib.wd_field_bytes(_dims(dims), prec, 12, 1) == 12 * half


def test_status_strings_and_defaults(lib):
    lib.wd_status_string.restype = ctypes.c_char_p
    msgs = [lib.wd_status_string(code) for code in (0, 1, -1, -2, -3, -4, -5, -6)]
    assert all(msgs) and len(set(msgs)) == len(msgs)
    import paper_0710_2442_amd as wd
    p = wd.wd_solve_params_default()
    assert p.struct_size == ctypes.sizeof(p)
    assert p.max_iter > 0 and p.check_every > 0


def test_a_c99_program_compiles_links_and_calls_the_library(tmp_path):
    """The header is plain C99 (no C++ in it) and a C program links against
    libwd.so and calls its host-side entry points."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_wd.c"
    src.write_text(
        '#include <stdio.h>\n#include "wd.h"\n'
        "int main(void) {\n"
        "  int dims[4] = {8, 8, 8, 8};\n"
        "  wd_solve_params p;\n"
        "  wd_solve_params_default(&p);\n"
        "  printf(\"%zu %zu %d %d %s\\n\", wd_field_bytes(dims, WD_F64, 1, WD_FULL), p.struct_size, p.solver,\n"
        "         (int)wd_dslash(NULL, NULL, NULL, 0.1, dims, WD_FULL), wd_status_string(WD_ERR_ARG));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "use_wd"
    lib_dir = os.path.dirname(LIB)
    cc = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.dirname(HEADER),
                         str(src), "-L", lib_dir, "-lwd", f"-Wl,-rpath,{lib_dir}", "-o", str(exe)],
                        capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    nbytes, size, solver, rc, msg = run.stdout.split(maxsplit=4)
    import paper_0710_2442_amd as wd
    assert int(nbytes) == wd.wd_field_bytes((8, 8, 8, 8), "f64")
    assert int(size) == wd.wd_solve_params_default().struct_size and int(solver) == wd.WD_SOLVER_CG
    assert int(rc) == -1 and msg.strip()
