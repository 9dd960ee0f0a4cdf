"""The device code of the fused step's wave strips, run on the CPU.

tests/emu/strip_emu.cpp compiles the kernels' strip functions as plain C++
(64 host threads in lockstep per wave) under AddressSanitizer, with every
buffer exactly as large as the C ABI's contract. For each model, boundary,
storage layout, lane layout and a set of widths, heights and tile shapes
(exact fits, ragged last strips and rows, workgroups wider than the grid),
it checks (periodic, transmissive and Dirichlet boundaries; the spray's
transport-only strip, which gets no gas velocity at all) that no access
leaves the buffers, that every cell of the grid is
written once a full sweep of tiles has run, that padding columns are never
written, and that a uniform state is left bitwise unchanged.
"""
import itertools
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emu")
CLANG = "/opt/rocm/llvm/bin/clang++"

# (nx, ny, ld, rows, waves per workgroup)
SHAPES = [(1, 5, 2, 2, 1), (129, 9, 130, 4, 2), (300, 7, 304, 3, 8), (128, 6, 128, 64, 1)]


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if not os.path.exists(CLANG) or shutil.which("true") is None:
        pytest.skip("needs the ROCm clang++ for a host build")
    out = str(tmp_path_factory.mktemp("emu") / "strip_emu")
    cmd = [CLANG, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-ffp-contract=off", "-I", os.path.join(EMU, "shim"),
           os.path.join(EMU, "strip_emu.cpp"), "-o", out, "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def test_strips_stay_in_bounds_and_cover_the_grid(emu):
    cases = []
    for model, bc, layout, cpl in itertools.product((0, 1, 2, 3), (0, 1, 2), (0, 1), (1, 2)):
        if model == 3 and bc == 2:
            continue  # the transport-only spray strip has no Dirichlet variant
        for nx, ny, ld, rows, wpb in SHAPES:
            cases.append((model, bc, nx, ny, ld, layout, cpl, rows, wpb))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")

    def run(c):
        r = subprocess.run([emu, *map(str, c)], capture_output=True, text=True, env=env,
                           timeout=600)
        return c, r.returncode, r.stdout + r.stderr[-2000:]

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(run, cases))
    bad = [(c, out) for c, rc, out in results if rc != 0]
    assert not bad, bad[:3]
