"""Build libori.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_1602_04691_amd.build [--jobs N] [--incremental]

Compiles the FFT pass kernels once per supported padded length L
(``csrc/passes.hip`` with ``-DORI_L=<L>``), the multi-problem passes of the
short lengths (``csrc/multi_passes.hip``), the auxiliary kernels and the
host runtime, and links ``paper_1602_04691_amd/libori.so``.
"""

import argparse
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libori.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no automatic a * b + c contraction: the fused operations are written
    # out (cx.h), so a body rounds the same in every kernel that runs it
    "-ffp-contract=off",
    "-I", INCLUDE, "-I", CSRC,
]


def supported_lengths():
    text = open(os.path.join(CSRC, "plan.h")).read()
    m = re.search(r"#define ORI_FOR_EACH_L\(X\)(.*?)\n\n", text, re.S)
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def _sources():
    units = [(os.path.join(CSRC, "passes.hip"), f"passes_L{L}.o", [f"-DORI_L={L}"])
             for L in supported_lengths()]
    units.append((os.path.join(CSRC, "multi_passes.hip"), "multi_passes.o", []))
    units.append((os.path.join(CSRC, "aux.hip"), "aux.o", []))
    units.append((os.path.join(CSRC, "physics.hip"), "physics.o", []))
    units.append((os.path.join(CSRC, "ori_api.cpp"), "ori_api.o", ["-x", "hip"]))
    return units


def _deps_mtime(src):
    """Newest of the unit's source and every header it may include."""
    return max([os.path.getmtime(src)] + [os.path.getmtime(os.path.join(d, f))
                                          for d in (CSRC, INCLUDE) for f in os.listdir(d)
                                          if f.endswith((".h", ".inc"))])


def _compile(unit, incremental):
    src, obj, extra = unit
    out = os.path.join(BUILD, obj)
    if incremental and os.path.exists(out) and os.path.getmtime(out) >= _deps_mtime(src):
        return out, ""
    cmd = [HIPCC] + FLAGS + extra + ["-c", src, "-o", out]
    p = subprocess.run(cmd, capture_output=True, text=True)
    log = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{log}")
    return out, log


def build(jobs=None, incremental=False, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or int(os.environ.get("MAX_JOBS", "0") or 0) or min(16, os.cpu_count() or 4)
    units = _sources()
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(u, incremental), units))
    objs = [o for o, _ in results]
    for _, log in results:
        if verbose and log.strip():
            print(log)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{p.stdout}{p.stderr}")
    os.replace(tmp, LIB)
    _build_c_smoke()
    _build_sanitized(objs)
    return LIB


# a C program that uses the C ABI without Python (tests/c/ori_abi_smoke.c)
C_SMOKE_SRC = os.path.join(ROOT, "tests", "c", "ori_abi_smoke.c")
C_SMOKE_BIN = os.path.join(ROOT, "tests", "c", "ori_abi_smoke")


def _build_c_smoke():
    if not os.path.exists(C_SMOKE_SRC):
        return
    cmd = [HIPCC, "-x", "hip", f"--offload-arch={ARCH}", "-O2", "-I", INCLUDE, C_SMOKE_SRC, "-o", C_SMOKE_BIN,
           "-L", PKG, "-lori", "-Wl,-rpath,$ORIGIN/../../paper_1602_04691_amd"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{p.stdout}{p.stderr}")


# The runtime's host code under AddressSanitizer and UBSan (device code is
# not instrumented: every -fsanitize= applies to the host pass only), linked
# with the same kernel objects, and two C programs against it: the host-only
# paths of the ABI (runs without a GPU) and the C ABI smoke program.
ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libori_asan.so")
C_HOST_PATHS_SRC = os.path.join(ROOT, "tests", "c", "ori_host_paths.c")
C_HOST_PATHS_ASAN = os.path.join(ROOT, "tests", "c", "ori_host_paths_asan")
C_SMOKE_ASAN = os.path.join(ROOT, "tests", "c", "ori_abi_smoke_asan")
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime_dir():
    # the directory of the compiler's own libclang_rt.asan-x86_64.so
    p = subprocess.run([HIPCC, "--print-resource-dir"], capture_output=True, text=True)
    res = p.stdout.strip().splitlines()[-1] if p.returncode == 0 and p.stdout.strip() else ""
    d = os.path.join(res, "lib", "linux")
    return d if res and os.path.exists(os.path.join(d, "libclang_rt.asan-x86_64.so")) else None


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{p.stdout}{p.stderr}")


def _build_sanitized(objs):
    rt = asan_runtime_dir()
    if rt is None:
        return None
    os.makedirs(ASAN_DIR, exist_ok=True)
    src = os.path.join(CSRC, "ori_api.cpp")
    obj = os.path.join(ASAN_DIR, "ori_api.o")
    _run([HIPCC, "-x", "hip", f"--offload-arch={ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", INCLUDE, "-I", CSRC]
         + SANITIZE + ["-c", src, "-o", obj])
    kernels = [o for o in objs if os.path.basename(o) != "ori_api.o"]
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + SANITIZE + ["-shared-libasan", "-o", ASAN_LIB, obj]
         + kernels + [f"-Wl,-rpath,{rt}"])
    for src, out in ((C_HOST_PATHS_SRC, C_HOST_PATHS_ASAN), (C_SMOKE_SRC, C_SMOKE_ASAN)):
        _run([HIPCC, "-x", "hip", f"--offload-arch={ARCH}", "-O1", "-g", "-I", INCLUDE] + SANITIZE
             + ["-shared-libasan", src, "-o", out, "-L", ASAN_DIR, "-lori_asan", f"-Wl,-rpath,{rt}",
                "-Wl,-rpath,$ORIGIN/../../paper_1602_04691_amd/_build/asan"])
    return ASAN_LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.incremental, a.verbose))


if __name__ == "__main__":
    sys.exit(main())
