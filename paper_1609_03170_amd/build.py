"""Compile the HIP sources of the library into paper_1609_03170_amd/libopengrape.so.

gfx950 only.  Every HIP translation unit is built with packed-FP32
instruction selection disabled (-packed-fp32-ops off) and without automatic
floating-point contraction (-ffp-contract=off): the device code writes its
fused multiply-adds explicitly, so an operation rounds the same way in every
kernel that performs it."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libopengrape.so")
SOURCES = [os.path.join(HERE, "csrc", "og_api.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off",
    "-I", os.path.join(ROOT, "include"),
]


# Host-code checks: the library's sources with AddressSanitizer and
# UndefinedBehaviorSanitizer on the host side only (each -fsanitize= follows
# -Xarch_host, so no device code is instrumented), linked with the host-side
# ABI driver tests/host/sanitize_abi.cpp into one executable.
SAN_DRIVER = os.path.join(ROOT, "tests", "host", "sanitize_abi.cpp")
SAN_EXE = os.path.join(ROOT, "tests", "host", "sanitize_abi")
SAN_FLAGS = [
    "--offload-arch=gfx950",
    "-O1",
    "-g",
    "-std=c++17",
    "-fno-omit-frame-pointer",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off",
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-I", os.path.join(ROOT, "include"),
]


def _lib_cmd(verbose):
    cmd = [HIPCC] + FLAGS + ["-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    return cmd


def _san_cmds(verbose):
    obj = SAN_EXE + ".og.o"
    cmds = [[HIPCC, "-c"] + SAN_FLAGS + ["-o", obj] + SOURCES,
            [HIPCC] + SAN_FLAGS + ["-o", SAN_EXE + ".tmp", obj, SAN_DRIVER]]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    return cmds


def _wait(proc, what):
    out, err = proc.communicate()
    if proc.returncode != 0:
        sys.stderr.write(out + err)
        raise RuntimeError("hipcc failed building " + what)


def build(verbose: bool = False, sanitized: bool = False) -> str:
    """Build libopengrape.so; with sanitized=True also the host-sanitizer
    executable, compiled at the same time in a second process."""
    p_lib = subprocess.Popen(_lib_cmd(verbose), stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    if sanitized:
        build_sanitized(verbose)
    _wait(p_lib, "libopengrape.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_sanitized(verbose: bool = False) -> str:
    compile_cmd, link_cmd = _san_cmds(verbose)
    for cmd, what in ((compile_cmd, "the sanitized host object"), (link_cmd, "the sanitizer driver")):
        _wait(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True), what)
    os.remove(SAN_EXE + ".og.o")
    os.replace(SAN_EXE + ".tmp", SAN_EXE)
    return SAN_EXE


def sanitized_stale() -> bool:
    """True when the sanitizer executable is missing or older than a source."""
    if not os.path.exists(SAN_EXE):
        return True
    t = os.path.getmtime(SAN_EXE)
    srcs = SOURCES + [SAN_DRIVER, os.path.join(HERE, "csrc", "og_device.h"),
                      os.path.join(ROOT, "include", "opengrape.h")]
    return any(os.path.getmtime(s) > t for s in srcs)


if __name__ == "__main__":
    print(build(verbose=True))
