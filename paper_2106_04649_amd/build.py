"""Build libmk.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_2106_04649_amd.build            # libmk.so
    python -m paper_2106_04649_amd.build --asan     # _build/asan/libmk_asan.so
    python -m paper_2106_04649_amd.build --device-checks   # libmk_checked.so

Each source compiles on its own (in parallel) and the objects are linked
into ``paper_2106_04649_amd/libmk.so``.  The build always recompiles.  The
sanitizer build instruments the host code with AddressSanitizer and
UndefinedBehaviorSanitizer, for the host-side checks in tests/.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmk.so")
SOURCES = ["k_contract.hip", "k_mfma.hip", "k_quant.hip", "k_trace.hip", "k_net.hip", "k_tail.hip", "mk_api.hip",
           "mk_net_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libmk.so")


def common_flags():
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        # packed FP32 instructions stay off: plain scalar/vector FP32 only
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-I", INCLUDE,
        "-I", CSRC,
    ]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *common_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def build_sanitized(verbose: bool = False) -> str:
    """The library with AddressSanitizer and UndefinedBehaviorSanitizer on its
    host code (device code unchanged in kind, built at -O1 with debug info):
    ``_build/asan/libmk_asan.so``, for host-side checks without a GPU.  The
    sanitizer flags apply to the host compilation only."""
    out = os.path.join(BUILD, "asan")
    os.makedirs(out, exist_ok=True)
    host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    flags = [f if f != "-O3" else "-O1" for f in common_flags()] + ["-g"] + host

    def one(src: str) -> str:
        obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(one, SOURCES))
    lib = os.path.join(out, "libmk_asan.so")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", lib]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    if verbose:
        print(f"built {lib}")
    return lib


CHECKED_LIB = os.path.join(HERE, "libmk_checked.so")


def build_checked(verbose: bool = False) -> str:
    """The library with its device-side bounds checks compiled in
    (-DMK_DEVICE_CHECKS, otherwise the normal flags): every kernel compares
    the end of each range it addresses with the allocation behind the
    pointer and records failures for mk_device_checks().  In-tree as
    ``libmk_checked.so`` beside ``libmk.so``."""
    out = os.path.join(BUILD, "checked")
    os.makedirs(out, exist_ok=True)
    flags = common_flags() + ["-DMK_DEVICE_CHECKS"]

    def one(src: str) -> str:
        obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = CHECKED_LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, CHECKED_LIB)
    if verbose:
        print(f"built {CHECKED_LIB}")
    return CHECKED_LIB


if __name__ == "__main__":
    try:
        if "--asan" in sys.argv[1:]:
            build_sanitized(verbose=True)
        elif "--device-checks" in sys.argv[1:]:
            build_checked(verbose=True)
        else:
            build(verbose=True)
    except RuntimeError as exc:
        print(exc, file=sys.stderr)
        sys.exit(1)
