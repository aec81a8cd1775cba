"""Build libsfrom.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1604_06750_amd.build  (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsfrom.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")
ARCH = os.environ.get("SFROM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "cartesian.cpp", "elastic.cpp", "general.cpp", "offline.hip", "wide.hip", "online.hip", "fine.hip", "surrogate.hip"]

COMMON = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-pragmas",
    f"-I{os.path.join(os.path.dirname(HERE), 'include')}",
]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def _stale(src: str, obj: str) -> bool:
    """Object older than its source or any header of the library."""
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src), os.path.join(CSRC, "sfrom_internal.h"),
            os.path.join(os.path.dirname(HERE), "include", "sfrom.h"), __file__]
    return os.path.getmtime(obj) < max(os.path.getmtime(d) for d in deps)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    if incremental and not _stale(src, obj):
        return obj
    lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
    cmd = [_hipcc(), *lang, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compile every source (or, with ``incremental``, only those whose
    object is older than the source or the headers) and link libsfrom.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


# Host sanitizers: AddressSanitizer and UndefinedBehaviorSanitizer on the
# host code only (each flag behind -Xarch_host; device code is compiled as
# usual). The library is loaded with the ASan runtime preloaded
# (asan_runtime()) and SFROM_LIBRARY pointing at it, and exercised through
# host-only handles.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_DIR = os.path.join(BUILD_DIR, "sanitize")


def asan_runtime() -> str:
    r = subprocess.run([_hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


def build_sanitized(verbose: bool = True) -> str:
    """libsfrom.so with host ASan + UBSan in _build/sanitize/ (rebuilt when
    a source or header is newer than it)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    out = os.path.join(SAN_DIR, "libsfrom.so")
    deps = [os.path.join(CSRC, x) for x in SOURCES] + [os.path.join(CSRC, "sfrom_internal.h"),
                                                       os.path.join(os.path.dirname(HERE), "include", "sfrom.h"),
                                                       __file__]
    if os.path.exists(out) and os.path.getmtime(out) >= max(os.path.getmtime(d) for d in deps):
        return out

    def comp(src):
        obj = os.path.join(SAN_DIR, os.path.basename(src) + ".o")
        cmd = [_hipcc(), "-x", "hip", *COMMON, *SANITIZE, "-g", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(comp, SOURCES))
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *SANITIZE, "-shared-libsan", *objs,
           "-o", out + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(out + ".tmp", out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)
