"""Compile the HIP/C++ sources into ``librsai.so`` (gfx950) next to this file.

Every source is compiled in parallel to an object file with hipcc, then linked
into one shared library. Flags: wave64 gfx950 code, -O3, and packed-FP32 code
generation disabled (``-target-feature -packed-fp32-ops``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librsai.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["rsai_tier.hip", "rsai_tier0h.hip", "rsai_tier2.hip", "rsai_wide.hip", "rsai_big.hip", "rsai_prep.hip", "rsai_backward.hip", "rsai_krylov.hip", "rsai_noalloc.hip", "rsai_match.hip", "rsai_detsum.hip", "rsai_host.cpp"]
ARCH = os.environ.get("RSAI_ARCH", "gfx950")


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include")]


# per-source flags: the register-block QR loops of the tier kernels and of the adjoint's
# refactorising kernel must unroll completely (constant register indices), which
# exceeds the default threshold; unrolled, the adjoint's block leaves scratch memory
# (the 512x512 adjoint with every factor recomputed: 6.2 -> 4.9 ms)
_UNROLL = ["-mllvm", "-pragma-unroll-threshold=262144"]
SOURCE_FLAGS = {"rsai_tier.hip": _UNROLL, "rsai_tier0h.hip": _UNROLL, "rsai_tier2.hip": _UNROLL,
                "rsai_backward.hip": _UNROLL}


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None) -> str:
    """Compile all sources and link ``librsai.so`` (or ``out``). Returns the library path."""
    bdir = BUILD_DIR if out is None else BUILD_DIR + "_" + os.path.basename(out).replace(".so", "")
    os.makedirs(bdir, exist_ok=True)
    hipcc = _hipcc()
    extra = list(extra or [])

    def compile_one(src):
        obj = os.path.join(bdir, src + ".o")
        cmd = [hipcc] + flags() + SOURCE_FLAGS.get(src, []) + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    target = LIB if out is None else out
    tmp = target + f".tmp{os.getpid()}"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(verbose=True))
