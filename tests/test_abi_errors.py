"""Argument errors at the C-ABI, without a GPU: every entry point that takes
a handle returns an error status for a NULL handle, and wd_gauge_create and
the size queries reject bad arguments before any device call.  The other
arguments are NULL or zero, so an entry point that touched them before
checking would crash the test process."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wd.h")
# WD_LIB: test another build of the library (e.g. one with host AddressSanitizer)
LIB = os.environ.get("WD_LIB") or os.path.join(ROOT, "paper_0710_2442_amd", "libwd.so")
WD_OK, WD_ERR_ARG, WD_ERR_DIMS, WD_ERR_PREC = 0, -1, -2, -3


def prototypes():
    """(return type, name, [parameter types]) of every function wd.h declares."""
    s = open(HEADER).read()
    s = re.sub(r"/\*.*?\*/", "", s, flags=re.S)
    out = []
    for ret, name, params in re.findall(r"\n\s*([a-z_ ]+?\s*\**)\s*\b(wd_[a-z0-9_]+)\s*\(([^)]*)\)\s*;", s):
        ps = [p.strip() for p in params.replace("\n", " ").split(",") if p.strip() and p.strip() != "void"]
        out.append((ret.strip(), name, ps))
    return out


def ctype_of(param):
    if "*" in param or "[" in param:
        return ctypes.c_void_p
    if "double" in param:
        return ctypes.c_double
    if "size_t" in param:
        return ctypes.c_size_t
    if "unsigned long long" in param:
        return ctypes.c_ulonglong
    return ctypes.c_int


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libwd.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    L.wd_last_error.restype = ctypes.c_char_p
    if os.environ.get("WD_LIB"):
        # the sanitized copy must really run under the sanitizer runtime
        maps = open("/proc/self/maps").read()
        assert "libclang_rt.asan" in maps and os.path.basename(LIB) in maps
    return L


HANDLE_FUNCS = [(n, ps) for r, n, ps in prototypes()
                if ps and re.search(r"\bwd_(gauge|ptc)\s*\*", ps[0]) and not n.endswith("_destroy")]


def test_the_header_parse_finds_the_handle_functions():
    names = [n for n, _ in HANDLE_FUNCS]
    for must in ("wd_dslash", "wd_solve", "wd_dslash_mrhs", "wd_ptc_train_step", "wd_tune_dslash", "wd_solve_batch"):
        assert must in names
    assert len(names) >= 25


@pytest.mark.parametrize("name,params", HANDLE_FUNCS, ids=[n for n, _ in HANDLE_FUNCS])
def test_null_handle_is_an_error(lib, name, params):
    f = getattr(lib, name)
    f.restype = ctypes.c_int
    f.argtypes = [ctype_of(p) for p in params]
    args = [t(0) if t is not ctypes.c_void_p else None for t in f.argtypes]
    rc = f(*args)
    assert rc == WD_ERR_ARG, (name, rc)
    assert lib.wd_last_error()


@pytest.mark.parametrize("name", ["wd_gauge_destroy", "wd_ptc_destroy"])
def test_destroying_null_is_a_no_op(lib, name):
    f = getattr(lib, name)
    f.argtypes = [ctypes.c_void_p]
    assert f(None) == WD_OK


def _dims(d):
    return (ctypes.c_int * 4)(*d) if d is not None else None


@pytest.mark.parametrize("U,dims,tbc,prec,want", [
    (None, (4, 4, 4, 4), -1, 0, WD_ERR_ARG),          # no links
    (True, None, -1, 0, WD_ERR_ARG),                  # no dims
    (True, (4, 3, 4, 4), -1, 0, WD_ERR_DIMS),         # odd extent
    (True, (4, 4, 0, 4), -1, 0, WD_ERR_DIMS),         # empty extent
    (True, (4, 4, 4, -2), -1, 0, WD_ERR_DIMS),        # negative extent
    (True, (2048, 2048, 2048, 2), -1, 0, WD_ERR_DIMS),  # more than 2^30 sites per parity
    (True, (4, 4, 4, 4), 0, 0, WD_ERR_ARG),           # time boundary neither +1 nor -1
    (True, (4, 4, 4, 4), -1, 7, WD_ERR_PREC),         # unknown precision
])
def test_gauge_create_rejects_bad_arguments(lib, U, dims, tbc, prec, want):
    f = lib.wd_gauge_create
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_void_p)]
    links = (ctypes.c_double * 8)() if U else None  # never read: the arguments fail first
    out = ctypes.c_void_p(12345)
    rc = f(links, _dims(dims), tbc, prec, None, ctypes.byref(out))
    assert rc == want, (rc, lib.wd_last_error())
    assert out.value is None  # *out is cleared on failure
    assert f(links, _dims((4, 4, 4, 4)), -1, 0, None, None) == WD_ERR_ARG  # no place for the handle


@pytest.mark.parametrize("dims", [None, (4, 3, 4, 4), (4, 4, 0, 4), (2, 2, 2, -2)])
def test_size_queries_return_zero_for_bad_dims(lib, dims):
    for fn, extra in ((lib.wd_vh_pad, ()), (lib.wd_field_bytes, (0, 1, 2)), (lib.wd_halo_face_bytes, (0,))):
        fn.restype = ctypes.c_size_t
        assert fn(_dims(dims), *extra) == 0, fn.__name__


def test_size_queries_reject_bad_precision_count_and_parity(lib):
    lib.wd_field_bytes.restype = ctypes.c_size_t
    d = _dims((4, 4, 4, 4))
    assert lib.wd_field_bytes(d, 4, 1, 0) == 0
    assert lib.wd_field_bytes(d, 0, 0, 0) == 0
    assert lib.wd_field_bytes(d, 0, 1, 3) == 0
    lib.wd_halo_face_bytes.restype = ctypes.c_size_t
    assert lib.wd_halo_face_bytes(d, 3) == 0  # faces are FP64 or FP32


def test_micro_benchmarks_reject_bad_sizes_before_the_device(lib):
    f = lib.wd_micro_stream
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_size_t, ctypes.c_int,
                  ctypes.c_void_p]
    sec = ctypes.c_double(math.nan)
    assert f(0, 9, 0, 1, 1 << 20, 1, ctypes.addressof(sec)) == WD_ERR_ARG
    assert f(0, 1, 0, 1, 15, 1, ctypes.addressof(sec)) == WD_ERR_ARG
    assert f(0, 1, 0, 1, 1 << 20, 1, None) == WD_ERR_ARG
    r = lib.wd_micro_resident
    r.restype = ctypes.c_int
    r.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    assert r(0, (1 << 20) + 16, 1, 1, ctypes.addressof(sec)) == WD_ERR_ARG   # not whole MiB
    assert r(0, 1 << 19, 1, 1, ctypes.addressof(sec)) == WD_ERR_ARG          # below 1 MiB
    assert r(0, 1 << 20, 0, 1, ctypes.addressof(sec)) == WD_ERR_ARG          # no pass
    assert r(0, 1 << 20, 1, 101, ctypes.addressof(sec)) == WD_ERR_ARG        # too many launches
    assert r(0, 1 << 20, 1, 1, None) == WD_ERR_ARG


def test_error_paths_under_host_address_sanitizer(tmp_path):
    """This file's tests again, against a host-sanitized copy of the library
    (every host source built with -fsanitize=address, device code left out;
    built here, a few seconds), in a child process with the compiler's ASan
    runtime preloaded: no sanitizer report, every test passes."""
    import importlib.util
    import subprocess
    import sys

    if os.environ.get("WD_LIB"):
        pytest.skip("already running against another build")
    import torch

    if torch.cuda.is_available():
        pytest.skip("the host-only sanitized copy carries no device code: run on a machine without a GPU")
    spec = importlib.util.spec_from_file_location("_wd_build", os.path.join(ROOT, "paper_0710_2442_amd", "build.py"))
    B = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(B)
    rt = B.asan_runtime()
    assert rt is not None, "the compiler's ASan runtime is missing"
    lib = B.build(asan=True, out_dir=str(tmp_path))
    env = dict(os.environ, WD_LIB=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", os.path.abspath(__file__)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout[-3000:] + p.stderr[-3000:]
    assert "AddressSanitizer" not in p.stderr
    assert " passed" in p.stdout
