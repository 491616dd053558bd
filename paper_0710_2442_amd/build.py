"""Build libwd.so (HIP for gfx950) in-tree.

Every ``csrc/*.hip`` file is compiled for gfx950 with hipcc; ``csrc/*.cpp``
(host-only C++) is compiled by hipcc as plain C++.  Objects go to
``_build/`` at the repository root and the shared library is written next to
this file, where the Python binding loads it.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libwd.so")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep packed-FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every fused multiply-add is written out (fma) in the sources, so a
    # kernel's rounding never depends on how the compiler schedules it: the
    # multi-RHS, batched and single-RHS hops agree bit for bit
    "-ffp-contract=off",
    # matrix-core results in ordinary VGPRs (no accumulator-register copies)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I", os.path.join(ROOT, "include"),
]
CXX_FLAGS = ["-x", "c++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
             "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include")]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


# Host AddressSanitizer build (--asan): the host side of every source is
# compiled with -fsanitize=address and the device side is not compiled at all
# (--offload-host-only), so the copy checks the C-ABI's host code (argument
# checks, error paths, bookkeeping) on a machine without a GPU and builds in
# seconds; its kernels cannot run.
ASAN_BUILD = os.path.join(ROOT, "_build_asan")
ASAN_LIB = os.path.join(ASAN_BUILD, "libwd_asan.so")
ASAN_FLAGS = ["--offload-host-only", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
              "-fno-omit-frame-pointer"]


def _compile(src, asan=False, out_dir=None):
    obj = os.path.join(out_dir or (ASAN_BUILD if asan else BUILD), os.path.basename(src) + ".o")
    flags = HIP_FLAGS if src.endswith(".hip") else CXX_FLAGS
    if asan:
        flags = flags + (ASAN_FLAGS if src.endswith(".hip") else ASAN_FLAGS[1:])
    cmd = [_hipcc(), *flags, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{err}")
    return obj, err


def build(verbose=False, jobs=None, asan=False, out_dir=None):
    """Build libwd.so (asan: the host-sanitized, host-only copy libwd_asan.so
    in out_dir, default _build_asan/, for the CPU tests of the C-ABI; load it
    with the compiler's ASan runtime preloaded)."""
    out_dir = out_dir or (ASAN_BUILD if asan else BUILD)
    lib = os.path.join(out_dir, "libwd_asan.so") if asan else LIB
    os.makedirs(out_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda src: _compile(src, asan, out_dir), srcs))
    for obj, err in results:
        if verbose and err:
            print(err, file=sys.stderr)
    objs = [o for o, _ in results]
    if asan:
        objs.append(_empty_fatbins(objs, out_dir))
    tmp = lib + ".tmp"
    link = ["-Xarch_host", "-fsanitize=address", "-shared-libasan"] if asan else []
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *link, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


def _empty_fatbins(objs, out_dir):
    """The host-only objects refer to one device-code bundle per source
    (__hip_fatbin_<id>).  Define each as a clang offload bundle with no
    entries, so the copy loads and registers no device code."""
    names = set()
    for o in objs:
        r = subprocess.run(["nm", "-u", o], capture_output=True, text=True, check=True)
        names.update(l.split()[-1] for l in r.stdout.splitlines() if "__hip_fatbin_" in l)
    src = os.path.join(out_dir, "empty_fatbins.c")
    with open(src, "w") as f:
        for n in sorted(names):
            f.write('const char %s[32] __attribute__((aligned(4096))) = "__CLANG_OFFLOAD_BUNDLE__";\n' % n)
    obj = src + ".o"
    subprocess.run(["gcc", "-c", "-fPIC", src, "-o", obj], check=True)
    return obj


def asan_runtime():
    """Path of the compiler's AddressSanitizer runtime (to preload), or None."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


if __name__ == "__main__":
    print(build(verbose=True, asan="--asan" in sys.argv[1:]))
