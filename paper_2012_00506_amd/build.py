"""Build the HIP library ``libfeastband.so`` for gfx950 (in-tree).

Every ``csrc/*.hip`` file is compiled by hipcc to an object under
``_build/`` and linked into ``libfeastband.so`` next to this file.

``sanitize=True`` (``--asan``) builds ``libfeastband_asan.so`` under
``_build_asan/`` instead: the host code with AddressSanitizer and
UndefinedBehaviorSanitizer (device code is compiled as usual and is never
run from it); it is loaded in place of the library by setting
FEASTBAND_LIB, with the clang ASan runtime preloaded, for the host-side
checks of the C ABI.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfeastband.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("FEASTBAND_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-Wno-unused-result",
    "-I" + os.path.join(HERE, "..", "include"),
]
LDFLAGS = ["-shared", f"--offload-arch={ARCH}"]
# host-only sanitizers: each -fsanitize= applies to the host pass alone
SAN_FLAGS = [
    "-O1", "-g", "-fno-omit-frame-pointer",
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
]
SAN_LDFLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-shared-libasan"]
OUT_SAN = os.path.join(HERE, "libfeastband_asan.so")
BUILD_SAN = os.path.join(HERE, "_build_asan")


def asan_runtime() -> str | None:
    """The clang ASan runtime that a process loading the sanitized library
    must preload, or None."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, force: bool = True, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD_SAN if sanitize else BUILD, os.path.basename(src)[:-4] + ".o")
    if not force and os.path.exists(obj):
        deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
        deps.append(os.path.join(HERE, "..", "include", "feastband.h"))
        if os.path.getmtime(obj) > max(os.path.getmtime(d) for d in deps):
            return obj
    flags = [f for f in CFLAGS if f != "-O3"] + SAN_FLAGS if sanitize else CFLAGS
    cmd = [HIPCC, *flags, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False, force: bool = True, sanitize: bool = False) -> str:
    """Compile all sources and link the shared library; returns its path.
    force=False recompiles only sources older than their object files'
    dependencies (the source, the internal headers and the C ABI header)."""
    os.makedirs(BUILD_SAN if sanitize else BUILD, exist_ok=True)
    out = OUT_SAN if sanitize else OUT
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, sanitize), srcs))
    tmp = out + ".tmp"
    cmd = [HIPCC, *LDFLAGS, *(SAN_LDFLAGS if sanitize else []), *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True, force="--incremental" not in sys.argv, sanitize="--asan" in sys.argv)
    sys.exit(0)
