"""The binary64 exponential the kernels use for the Gaussian weight
(vegas_math.hpp), built for the host from the same header and checked against
the C library's exp (through numpy): within 3 ulp wherever the result is a
normal number, exact at 0, and the right limits (0 far below, infinity above
709.8)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_09341_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def exp_f64(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    exe = str(tmp_path_factory.mktemp("exp") / "exp_test")
    subprocess.run([HIPCC, "-O2", "-I" + CSRC, os.path.join(ROOT, "tests", "helpers",
                                                              "exp_test.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(x):
        x = np.asarray(x, dtype=np.float64)
        out = subprocess.run([exe], input="\n".join(repr(float(v)) for v in x), text=True,
                             check=True, capture_output=True).stdout.split()
        got = np.array(out, dtype=np.float64).reshape(-1, 2)
        assert np.array_equal(got[:, 0], x)
        return got[:, 1]
    return run


def _ulp_error(y, ref):
    return np.abs(y - ref) / np.spacing(np.abs(ref))


def test_exp_within_3_ulp(exp_f64):
    rng = np.random.default_rng(7)
    x = np.concatenate([
        rng.uniform(-708.0, 709.0, 20_000),       # the whole normal range
        rng.uniform(-40.0, 5.0, 20_000),          # where Gaussian weights live
        rng.uniform(-1e-3, 1e-3, 2_000),          # e^x near 1
        np.log(2.0) * np.arange(-1000, 1001) / 2,  # reduction boundaries n +- 1/2
        np.array([1e-300, -1e-300, 1.0, -1.0, 0.5, 700.0, -700.0]),
    ])
    y, ref = exp_f64(x), np.exp(x)
    normal = np.abs(ref) >= np.finfo(np.float64).tiny
    assert normal.sum() > 0.99 * x.size
    assert _ulp_error(y[normal], ref[normal]).max() <= 3.0


def test_exp_special_values(exp_f64):
    x = [0.0, -0.0, -745.5, -800.0, -1100.0, -1e5, -1e300, -np.inf, 709.78, 709.79, 1e5]
    y = exp_f64(x)
    assert y[0] == 1.0 and y[1] == 1.0
    assert np.all(y[2:8] == 0.0)
    assert np.isfinite(y[8]) and abs(y[8] / np.exp(709.78) - 1) < 1e-15
    assert np.all(np.isinf(y[9:])) and np.all(y[9:] > 0)


def test_exp_subnormal_results(exp_f64):
    """Below -708.4 the result loses precision gradually; the error stays
    within a few units of the smallest subnormal."""
    x = np.linspace(-744.0, -708.5, 3001)
    y, ref = exp_f64(x), np.exp(x)
    assert np.all(np.abs(y - ref) <= 4 * np.maximum(np.spacing(ref), 5e-324))
