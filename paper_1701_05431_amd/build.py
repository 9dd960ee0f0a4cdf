"""Build the gfx950 shared library ``libfvm.so`` from ``csrc/*.hip`` in place.

    python -m paper_1701_05431_amd.build

hipcc cross-compiles for gfx950 (no GPU needed). Packed-FP32 instructions are
disabled for every HIP source.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfvm.so")
SOURCES = ["fvm_api.hip", "fvm_kernels.hip", "fvm_batch.hip", "fvm_adjoint.hip",
           "fvm_output.hip", "fvm_maxent.hip", "fvm_adjoint_spray.hip", "fvm_resident.hip"]
ARCH = os.environ.get("FVM_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def flags(extra=()):
    # no automatic FMA contraction: the kernels write their fused
    # multiply-adds explicitly, so every inlined copy of a flux rounds the
    # same way and results do not depend on the tiling
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(HERE, "..", "include"), *extra]


def _jobs() -> int:
    """Parallel compiles: MAX_JOBS if set, else the usable cores, at most 16."""
    env = os.environ.get("MAX_JOBS")
    if env and env.isdigit() and int(env) > 0:
        return min(int(env), 16)
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def build(verbose: bool = False, extra=(), out: str = LIB) -> str:
    """Compiles every source (extra: additional hipcc flags) and links `out`."""
    with tempfile.TemporaryDirectory(prefix="fvm_build_") as tmpdir:
        objs, cmds = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, src.replace(".hip", ".o"))
            cmds.append([HIPCC, *flags(extra), "-c", os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
        if verbose:
            for cmd in cmds:
                print(" ".join(cmd), flush=True)
        with ThreadPoolExecutor(max_workers=_jobs()) as ex:
            for r in ex.map(lambda c: subprocess.run(c, check=True), cmds):
                pass
        tmp = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
