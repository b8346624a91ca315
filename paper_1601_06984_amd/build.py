"""Builds libmlbm.so in-tree: host plan builder (g++) + HIP kernels for
gfx950 (hipcc), linked into one shared library."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libmlbm.so")

HIP_SOURCES = ["sim.hip", "adjoint.hip"]
CXX_SOURCES = ["plan.cpp"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd):
    r = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link ``lib/libmlbm.so``;
    returns its path."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = []
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-c", src, "-o", obj],
                     obj))
    for src in HIP_SOURCES:
        if not os.path.exists(os.path.join(CSRC, src)):
            continue
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(([hipcc] + HIPCC_FLAGS + ["-c", src, "-o", obj], obj))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_sanitized_host(out_dir: str) -> str:
    """A variant of the library whose host plan builder is compiled with
    AddressSanitizer and UndefinedBehaviorSanitizer (g++; the device code and
    the HIP host objects are the normal build's, so build() must have run).
    Returns the path of the shared library; load it with the sanitizer
    runtime preloaded (see sanitizer_env)."""
    objs = [os.path.join(BUILD, src + ".o") for src in HIP_SOURCES]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError("build() first: missing " + ", ".join(missing))
    os.makedirs(out_dir, exist_ok=True)
    plan_o = os.path.join(out_dir, "plan_sanitized.o")
    lib = os.path.join(out_dir, "libmlbm_sanitized.so")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-std=c++17", "-fPIC", "-pthread"]
    _run(["g++"] + flags + ["-c", "plan.cpp", "-o", plan_o])
    _run(["g++", "-shared", "-fsanitize=address,undefined", "-pthread", plan_o] + objs +
         ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", lib])
    return lib


def sanitizer_env(lib: str, log_dir: str) -> dict:
    """Environment for a process that loads the sanitized library: the ASan
    runtime first, then libstdc++ (so that ASan finds the C++ exception
    runtime a Python process loads late), reports written under log_dir."""
    def rt(name):
        return subprocess.run(["g++", "-print-file-name=" + name], capture_output=True,
                              text=True, check=True).stdout.strip()
    env = dict(os.environ)
    env["MLBM_LIBRARY"] = lib
    env["LD_PRELOAD"] = rt("libasan.so") + " " + rt("libstdc++.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:log_path=" + os.path.join(log_dir, "asan")
    env["UBSAN_OPTIONS"] = ("halt_on_error=1:print_stacktrace=1:log_path=" +
                            os.path.join(log_dir, "ubsan"))
    return env


if __name__ == "__main__":
    build(verbose=True)
