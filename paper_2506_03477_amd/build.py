"""Build libchi0.so (and the synthetic-input GPU generator) for gfx950 with
hipcc, in-tree.  ``python -m paper_2506_03477_amd.build``."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libchi0.so")
SYNTH_SRC = os.path.join(ROOT, "synth", "csrc", "synth_gen.hip")
SYNTH_LIB = os.path.join(ROOT, "synth", "libsynth_gen.so")

SAN_LIB = os.path.join(BUILD, "libchi0_hostsan.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code (some of their
# forms are unreliable on the target boxes); hipcc still emits ordinary FP32.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-Wno-unused-value"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def _sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def build(verbose: bool = False, jobs: int = 8, save_temps: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    objs = []
    cmds = []
    for s in srcs:
        o = os.path.join(BUILD, os.path.basename(s) + ".o")
        objs.append(o)
        cmd = [HIPCC] + COMMON + ["-c", s, "-o", o]
        if s.endswith(".cpp"):
            cmd = [HIPCC, "-x", "hip"] + COMMON + ["-c", s, "-o", o]
        if save_temps:
            cmd.insert(1, "-save-temps=obj")
        cmds.append(cmd)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    tmp = SYNTH_LIB + ".tmp"
    _run([HIPCC] + COMMON + ["-shared", "-o", tmp, SYNTH_SRC])
    os.replace(tmp, SYNTH_LIB)
    return LIB


# AddressSanitizer and UndefinedBehaviorSanitizer on host code only: every
# -fsanitize= sits behind -Xarch_host, so the device code is built as usual.
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def asan_runtime() -> str:
    """Path of the ASan runtime the sanitized library needs first in the
    process (LD_PRELOAD) when it is loaded into an unsanitized program."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    return _run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"]).strip()


def build_host_sanitized() -> str:
    """libchi0 with the host layer (api.cpp: validation, planner, tile model,
    error paths) built with ASan + UBSan, linked with the kernels' objects
    of the last build(), as _build/libchi0_hostsan.so.  For CPU tests of the
    host-only entry points: load it with the runtime of asan_runtime()
    preloaded and CHI0_LIB pointing at it."""
    if not all(os.path.exists(os.path.join(BUILD, os.path.basename(s) + ".o"))
               for s in _sources()):
        build()
    objs = []
    for s in _sources():
        o = os.path.join(BUILD, os.path.basename(s) + ".o")
        if s.endswith(".cpp"):
            o = os.path.join(BUILD, os.path.basename(s) + ".hostsan.o")
            _run([HIPCC, "-x", "hip"] + COMMON + HOST_SAN + ["-c", s, "-o", o])
        objs.append(o)
    tmp = SAN_LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + HOST_SAN + ["-o", tmp] + objs)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    print(build(verbose=True, save_temps="--save-temps" in sys.argv))
