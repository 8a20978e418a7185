"""Build libdfx.so (host core + gfx950 kernels) in-tree with hipcc.

`python -m paper_2406_18109_amd.build` or `build()`; compiles every source
each call (objects in parallel) and links paper_2406_18109_amd/libdfx.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libdfx.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function", "-pthread"]
# Device code: no packed FP32 instructions, IEEE-rounded fp32 divide/sqrt,
# denormals kept.
# Uniform (wave-wide) control flow, such as the op-list dispatch, is left
# unstructured: structurising it adds flow blocks to every interpreted op.
DEVICE = ["--offload-arch=" + ARCH, "-fhip-fp32-correctly-rounded-divide-sqrt",
          "-fno-gpu-flush-denormals-to-zero", "-mllvm", "-structurizecfg-skip-uniform-regions=true",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SOURCES = [
    ("core.cpp", False),
    ("serve.cpp", False),
    ("batch.cpp", False),
    ("kernels.hip", True),
    ("vm_tier0.hip", True),
    ("vm_tier1.hip", True),
    ("vm_tier2.hip", True),
    ("vm_tier3.hip", True),
    ("serve.hip", True),
    ("batch.hip", True),
]


def _compile(src: str, device: bool) -> str:
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON
    if device:
        cmd += DEVICE + ["-x", "hip"]
    else:
        cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compile failed: " + src)
    return obj


def build(verbose: bool = False) -> str:
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "-pthread", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


# Host code with AddressSanitizer and UndefinedBehaviorSanitizer, for the
# CPU tests of the host logic (analysis-only contexts): the host sources are
# compiled by g++ and linked with the kernel objects of the last build().
# Python is not instrumented, so the runtime must be preloaded
# (sanitizer_env).  Output: _build/libdfx_san.so.
SAN_OUT = os.path.join(BUILD, "libdfx_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def build_sanitized() -> str:
    kernels = [os.path.join(BUILD, src + ".o") for src, device in SOURCES if device]
    if not all(os.path.exists(k) for k in kernels):
        build()
    objs = []
    for src, device in SOURCES:
        if device:
            continue
        obj = os.path.join(BUILD, src + ".san.o")
        cmd = (["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off", "-pthread", "-D__HIP_PLATFORM_AMD__",
                "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")] + SAN_FLAGS +
               ["-c", os.path.join(CSRC, src), "-o", obj])
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("sanitizer compile failed: " + src)
        objs.append(obj)
    cmd = (["g++", "-shared", "-fPIC", "-pthread"] + SAN_FLAGS + ["-o", SAN_OUT] + objs + kernels +
           ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("sanitizer link failed")
    return SAN_OUT


def sanitizer_env() -> dict:
    """Environment that loads the sanitizer build into an uninstrumented Python."""
    rt = []
    for name in ("libasan.so", "libubsan.so"):
        path = subprocess.run(["g++", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
        if not os.path.isabs(path):
            raise RuntimeError("sanitizer runtime not found: " + name)
        rt.append(path)
    env = dict(os.environ)
    env.update(DFX_LIB=SAN_OUT, LD_PRELOAD=" ".join(rt), ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return env


if __name__ == "__main__":
    build(verbose=True)
