"""The spray adjoint's device code, built for the host (tests/emu/
spray_adjoint_emu.cpp) and run tile by tile under AddressSanitizer on
buffers exactly as large as the ABI contract (LDS included): no access
outside them, no padding column written, and the values equal the oracle's
adjoint step (relative L-inf 1e-12) for every boundary condition and both
layouts, on grids with ragged tiles in both directions."""
import math
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import fv as orc
from paper_1701_05431_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emu")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if not os.path.exists(CLANG) or shutil.which("true") is None:
        pytest.skip("needs the ROCm clang++ for a host build")
    out = str(tmp_path_factory.mktemp("sadjemu") / "spray_adjoint_emu")
    # FVM_EMU_DEFINES: extra -D flags, e.g. another tile shape
    # ("-DFVM_SADJ_COLS=62 -DFVM_SADJ_ROWS=6")
    extra = os.environ.get("FVM_EMU_DEFINES", "").split()
    cmd = [CLANG, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-ffp-contract=off", *extra, "-I", os.path.join(EMU, "shim"),
           os.path.join(EMU, "spray_adjoint_emu.cpp"), "-o", out, "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _ghosts():
    g = []
    for k, (u, v) in enumerate([(0.3, -0.2), (-0.4, 0.1), (0.2, 0.35), (-0.1, -0.3)]):
        m = inputs.lognormal_moments(1.0 + 0.1 * k, math.log(0.2), 0.3)
        g.append([m[0], m[1], m[2], m[3], m[2] * u, m[2] * v])
    return np.array(g)


def _case(nx, ny, seed):
    W, ug = inputs.spray_state(nx, ny, seed)
    rng = np.random.default_rng(seed + 50)
    W = W.copy()
    W[:4] *= 1.0 + 0.02 * rng.standard_normal((4, ny, nx))
    W[4:] += 0.1 * W[2] * rng.standard_normal((2, ny, nx))
    if nx >= 7 and ny >= 4:
        W[:, 1:3, 2:5] = 0.0   # vacuum cells next to droplets
    lam = rng.standard_normal((6, ny, nx))
    return W, ug, lam


# (nx, ny, pitch)
SHAPES = [(1, 1, 1), (1, 5, 2), (2, 3, 2), (7, 4, 8), (65, 9, 72), (130, 17, 130),
          (64, 8, 64)]


def test_spray_adjoint_cells_in_bounds_and_equal_the_oracle(emu, tmp_path):
    ghost = _ghosts()
    cases = []
    for bc in (0, 1, 2):
        for layout in (0, 1):
            for k, (nx, ny, pitch) in enumerate(SHAPES):
                for theta in (0.1, math.inf):
                    cases.append((bc, layout, nx, ny, pitch, theta, 10 * k + bc))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")

    def run(c):
        bc, layout, nx, ny, pitch, theta, seed = c
        W, ug, lam = _case(nx, ny, seed)
        K, s_eps, dt, lx, ly = 0.7, 0.01, 0.02, 1.0, 0.8
        tag = "_".join(map(str, c)).replace("inf", "i")
        fin, fout = str(tmp_path / f"in_{tag}"), str(tmp_path / f"out_{tag}")
        np.concatenate([W.ravel(), lam.ravel(), ug.ravel(), ghost.ravel()]).tofile(fin)
        it = 0.0 if math.isinf(theta) else 1.0 / theta
        args = [emu, bc, nx, ny, pitch, layout, lx, ly, repr(dt), K, repr(it), s_eps, fin, fout]
        r = subprocess.run(list(map(str, args)), capture_output=True, text=True, env=env,
                           timeout=300)
        if r.returncode != 0:
            return c, r.stdout + r.stderr[-2000:]
        got = np.fromfile(fout).reshape(6, ny, nx)
        P = orc.params(orc.SPRAY, nx, ny, bc=bc, lx=lx, ly=ly, K=K, theta=theta, s_eps=s_eps,
                       ghost=ghost if bc == 2 else None)
        ref = orc.adjoint_step(P, W, dt, lam, ug)
        err = max(np.max(np.abs(got[v] - ref[v])) / max(np.max(np.abs(ref[v])), 1e-300)
                  for v in range(6))
        return c, None if err <= 1e-12 else f"rel Linf {err:.3e}"

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(run, cases))
    bad = [(c, msg) for c, msg in results if msg]
    assert not bad, bad[:3]
