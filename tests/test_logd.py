"""The kernels' FP64 logarithm (fvm_models.hpp, logd: argument reduction to
[sqrt(1/2), sqrt(2)) and the atanh series) and reciprocal square root
(rroot), built for the host through the CPU shim, against the C library:
logd within 2 ulps of log over log-uniform arguments from 1e-300 to 1e300,
arguments near 1, both sides of the reduction's switch at sqrt(1/2), powers
of two and subnormals; rroot within 1 ulp of 1/sqrt over 1e-300 to 1e300.
Both run once with exact hardware estimates and once with estimates off by
1e-7 relative (the refinement steps must recover full precision)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emu")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module", params=["0.0", "1e-7"])
def emu(tmp_path_factory, request):
    if not os.path.exists(CLANG) or shutil.which("true") is None:
        pytest.skip("needs the ROCm clang++ for a host build")
    out = str(tmp_path_factory.mktemp("logd") / "logd_emu")
    cmd = [CLANG, "-std=c++20", "-O1", "-ffp-contract=off", "-I", os.path.join(EMU, "shim"),
           f"-DFVM_EMU_EST_ERR={request.param}", os.path.join(EMU, "logd_emu.cpp"), "-o", out,
           "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def run_emu(emu, fn, x):
    inp = "\n".join(float(v).hex() for v in x) + "\n"
    r = subprocess.run([emu, fn], input=inp, capture_output=True, text=True, check=True,
                       timeout=300)
    pairs = [ln.split() for ln in r.stdout.splitlines()]
    back = np.array([float.fromhex(a) for a, _ in pairs])
    assert np.array_equal(back, x)
    return np.array([float.fromhex(b) for _, b in pairs])


def test_rroot_within_one_ulp(emu):
    rng = np.random.default_rng(11)
    x = np.concatenate([np.exp(rng.uniform(np.log(1e-300), np.log(1e300), 20000)),
                        2.0 ** np.arange(-996, 996, 7, dtype=np.float64),
                        6.283185307179586 * np.exp(rng.uniform(np.log(1e-8), np.log(1e2), 5000))])
    got = run_emu(emu, "rroot", x)
    ref = 1.0 / np.sqrt(x.astype(np.longdouble))
    ulp = np.abs(got.astype(np.longdouble) - ref) / np.spacing(np.abs(ref.astype(np.float64)))
    worst = int(np.argmax(ulp))
    assert ulp.max() <= 1.0, (float(x[worst]).hex(), got[worst], float(ref[worst]), float(ulp.max()))


def test_logd_within_two_ulps(emu):
    rng = np.random.default_rng(7)
    xs = [np.exp(rng.uniform(np.log(1e-300), np.log(1e300), 20000)),
          1.0 + rng.uniform(-1e-3, 1e-3, 5000),
          1.0 + rng.uniform(-1e-12, 1e-12, 2000),
          np.sqrt(0.5) * (1.0 + rng.uniform(-1e-9, 1e-9, 2000)),
          np.sqrt(2.0) * (1.0 + rng.uniform(-1e-9, 1e-9, 2000)),
          2.0 ** np.arange(-1070, 1020, 7, dtype=np.float64),
          np.array([1e-310, 4.9e-324, 2.2250738585072014e-308, 1.7976931348623157e308,
                    0.5, 1.0, 2.0, 0.7071067811865476, 0.7071067811865475])]
    x = np.concatenate(xs)
    x = x[np.isfinite(x) & (x > 0)]
    got = run_emu(emu, "logd", x)
    ref = np.log(x)
    ulp = np.abs(got - ref) / np.spacing(np.abs(ref))
    ulp[ref == 0.0] = np.abs(got[ref == 0.0]) / np.spacing(0.0)
    worst = int(np.argmax(ulp))
    assert ulp.max() <= 2.0, (float(x[worst]).hex(), got[worst], ref[worst], ulp.max())
