"""Compile the HIP library for gfx950 into paper_2505_04155_amd/_build/libamppcg.so."""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libamppcg.so")
SOURCES = ["amp_pcg.hip"]
HEADERS = ["amp_controller.hpp", "amp_device.hpp", "amp_kernels.hpp", "amp_cheb.hpp", "amp_fv.hpp",
           "amp_batch.hpp", "amp_hex.hpp", "amp_hexsolve.hpp", "amp_pmg.hpp"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return [
        "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions are kept out of every kernel
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # one rounding per operation, as the precision model prescribes
        "-ffp-contract=off",
        # leading pointer/int kernel arguments arrive in SGPRs at launch
        "-mllvm", "-amdgpu-kernarg-preload-count=16",
        "-fno-gpu-rdc", "-Wall", "-Wno-unused-result",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def sources_mtime() -> float:
    paths = [os.path.join(CSRC, f) for f in SOURCES + HEADERS]
    paths.append(os.path.join(ROOT, "include", "amp_pcg.h"))
    paths.append(os.path.abspath(__file__))
    return max(os.path.getmtime(p) for p in paths)


KERNEL_HEADERS = ["amp_controller.hpp", "amp_device.hpp", "amp_kernels.hpp", "amp_cheb.hpp"]


def _code_only(text: str) -> str:
    """C++ source without comments and blank space (string literals in these
    headers hold no comment markers)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_digest() -> str:
    """SHA-256 over the code of the sources that define the iteration kernels
    (device headers, comments and layout ignored) and the compiler flags:
    names the kernel build a stored measurement of those kernels belongs to."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_HEADERS:
        with open(os.path.join(CSRC, f), encoding="utf-8") as fh:
            h.update(f.encode() + b"\0" + _code_only(fh.read()).encode())
    h.update(" ".join(f for f in flags() if not f.startswith("/")).encode())
    return h.hexdigest()[:16]


def is_stale() -> bool:
    return not os.path.exists(LIB) or os.path.getmtime(LIB) < sources_mtime()


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + flags() + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
