"""The adjoint kernel's wave strips run on the CPU.

tests/emu/adjoint_emu.cpp compiles the device code of both adjoint strip
layouts (62 columns with one cell per lane; 128 with two) as plain C++, 64
host threads in lockstep per wave, under AddressSanitizer, with every buffer
exactly as large as the C ABI's contract. For advection and Euler, periodic,
transmissive and Dirichlet boundaries, both storage layouts and a set of
widths, heights and row blocks (exact fits, ragged last strips, grids
narrower than a strip), it checks that no access leaves the buffers, that
every cell is written and no padding column touched, and that the two
layouts give the same multipliers bit for bit. For a few of the shapes the
multipliers are also compared with the oracle's adjoint step.
"""
import itertools
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import fv as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emu")
CLANG = "/opt/rocm/llvm/bin/clang++"

# (nx, ny, ld, rows)
SHAPES = [(1, 5, 2, 2), (2, 7, 2, 3), (130, 9, 130, 4), (257, 6, 258, 64), (128, 6, 128, 5),
          (300, 5, 304, 2)]


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if not os.path.exists(CLANG) or shutil.which("true") is None:
        pytest.skip("needs the ROCm clang++ for a host build")
    out = str(tmp_path_factory.mktemp("adjemu") / "adjoint_emu")
    cmd = [CLANG, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-ffp-contract=off", "-I", os.path.join(EMU, "shim"),
           os.path.join(EMU, "adjoint_emu.cpp"), "-o", out, "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def test_adjoint_strips_in_bounds_and_layouts_agree(emu):
    cases = [(model, bc, nx, ny, ld, layout, rows)
             for model, bc, layout in itertools.product((0, 1), (0, 1, 2), (0, 1))
             for nx, ny, ld, rows in SHAPES]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")

    def run(c):
        r = subprocess.run([emu, *map(str, c)], capture_output=True, text=True, env=env,
                           timeout=600)
        return c, r.returncode, r.stdout + r.stderr[-2000:]

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(run, cases))
    bad = [(c, out) for c, rc, out in results if rc != 0]
    assert not bad, bad[:3]


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("bc", [0, 1, 2])
def test_adjoint_strips_match_the_oracle(emu, tmp_path, model, bc):
    nx, ny, ld, rows = 130, 9, 130, 4
    out = str(tmp_path / "adj.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([emu, str(model), str(bc), str(nx), str(ny), str(ld), "0", str(rows), out],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    nv = 1 if model == 0 else 4
    raw = np.fromfile(out, dtype=np.float64)
    n = nv * ny * nx
    W, lam, got = (raw[k * n:(k + 1) * n].reshape(nv, ny, nx) for k in range(3))
    ghost = np.zeros((4, 6))
    ghost[:, :nv] = raw[3 * n:].reshape(4, nv)
    P = orc.params(model, nx, ny, bc=bc, gamma=1.4, ax=0.7, ay=-0.4, ghost=ghost)
    ref = orc.adjoint_step(P, W, 1e-3, lam)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale
