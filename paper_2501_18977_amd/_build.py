"""Builds the gfx950 HIP library ``libbbfc.so`` in-tree with hipcc."""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbbfc.so")
SOURCES = ["bbfc_api.cpp", "bbfc_kernels.hip", "bbfc_batch.hip", "bbfc_server.cpp", "bbfc_probe.hip", "bbfc_bulk.hip", "bbfc_ordered.hip"]
HEADERS = ["bbfc_common.hpp", "bbfc_internal.hpp", "bbfc_tile.hpp"]
ARCH = os.environ.get("BBFC_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-fno-strict-aliasing",
    "-ffp-contract=off",
    "-Wall",
    "-Wno-unused-command-line-argument",
    # packed FP32 instructions stay off in every gfx950 object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    env = os.environ.get("HIPCC")
    if env:
        return env
    found = shutil.which("hipcc")
    return found or "/opt/rocm/bin/hipcc"


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(extra_flags: list[str] | None = None, out: str | None = None, verbose: bool = False) -> str:
    """Compile every source (in parallel) and link ``libbbfc.so``; always rebuilds."""
    from concurrent.futures import ThreadPoolExecutor

    out = out or LIB
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [hipcc(), *HIP_FLAGS, *(extra_flags or []), "-I", os.path.join(ROOT, "include")]
    compile_flags = [f for f in common if f != "-shared"]

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [*compile_flags, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, sources()))
    tmp = out + ".tmp"
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, out)
    return out


# Host code under AddressSanitizer and UndefinedBehaviorSanitizer (device
# code is not instrumented: each flag applies to the host pass only).
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
HOST_SANITIZED = ["bbfc_api.cpp", "bbfc_server.cpp"]
SAN_LIB = os.path.join(HERE, "_build", "libbbfc_hostsan.so")


def build_host_sanitized() -> str:
    """libbbfc_hostsan.so: the library with the host code of the C ABI and
    the server (the sources whose host logic runs without a device) built
    with sanitizers, linked with the other objects of the regular build
    (which must exist: build() makes them). Loaded through BBFC_LIBRARY by
    the CPU tests, with the compiler's ASan runtime preloaded."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    flags = [hipcc(), *[f for f in HIP_FLAGS if f not in ("-shared", "-O3")], "-O1", "-g", *HOST_SANITIZE,
             "-I", os.path.join(ROOT, "include")]

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, src + ".hostsan.o")
        subprocess.run([*flags, "-c", "-o", obj, os.path.join(CSRC, src)], check=True)
        return obj

    others = [os.path.join(objdir, s + ".o") for s in SOURCES if s not in HOST_SANITIZED]
    missing = [o for o in others if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"regular objects missing ({missing[0]}): run build() first")
    with ThreadPoolExecutor(max_workers=2) as ex:
        objs = list(ex.map(compile_one, HOST_SANITIZED))
    tmp = SAN_LIB + ".tmp"
    subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *others], check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "bbfc.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build(verbose=True))
