"""The binary64 functions the kernels use (vegas_math.hpp), built for the
host from the same header and checked against the C library through numpy:
exp within 3 ulp wherever the result is a normal number, exact at 0, with the
right limits (0 far below, infinity above 709.8); log within 2 ulp over the
whole positive range, subnormals included, exact at 1; x^a as e^(a ln x)
within a few ulp of ln x times |a ln x|, as the refinement uses it; sin and
cos of 2 pi u within 2 ulp of 40-digit values over [0, 1], quarter and eighth
turns included."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_09341_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def mathf(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    exe = str(tmp_path_factory.mktemp("math") / "math_test")
    subprocess.run([HIPCC, "-O2", "-I" + CSRC, os.path.join(ROOT, "tests", "helpers",
                                                              "math_test.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(op, x, a=None):
        x = np.asarray(x, dtype=np.float64)
        if a is None:
            lines = [f"{op} {float(v)!r}" for v in x]
        else:
            lines = [f"{op} {float(v)!r} {float(w)!r}" for v, w in zip(x, np.broadcast_to(a, x.shape))]
        out = subprocess.run([exe], input="\n".join(lines), text=True, check=True,
                             capture_output=True).stdout.split()
        return np.array(out, dtype=np.float64)
    return run


@pytest.fixture(scope="module")
def exp_f64(mathf):
    return lambda x: mathf("e", x)


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


def test_log_within_2_ulp(mathf):
    rng = np.random.default_rng(9)
    x = np.concatenate([
        np.exp(rng.uniform(-700.0, 700.0, 20_000)),             # the normal range
        1.0 + rng.uniform(-1e-3, 1e-3, 5_000),                   # ln x near 0
        rng.uniform(0.0, 1.0, 5_000),                             # where p_i lives
        np.ldexp(rng.uniform(0.5, 1.0, 2_000), rng.integers(-1074, -1022, 2_000)),  # subnormal
        np.array([np.finfo(np.float64).max, np.finfo(np.float64).tiny, 5e-324, 2.0, 0.5]),
    ])
    x = x[x > 0]
    y, ref = mathf("l", x), np.log(x)
    assert mathf("l", [1.0])[0] == 0.0
    nz = ref != 0
    assert _ulp_error(y[nz], ref[nz]).max() <= 2.0


def test_pow_pos_as_the_refinement_uses_it(mathf):
    """r = ((1 - p)/(-ln p))^alpha for p in (0, 1) and alpha in [0, 2]: within
    8 ulp of ln q times |alpha ln q| (plus exp's 3 ulp) of the C library's
    pow; alpha = 0 gives exactly 1."""
    rng = np.random.default_rng(10)
    p = np.concatenate([rng.uniform(0.0, 1.0, 10_000), np.exp(-rng.uniform(0.0, 700.0, 5_000))])
    p = p[(p > 0) & (p < 1)]
    q = (1.0 - p) / -np.log(p)
    alpha = rng.uniform(0.0, 2.0, q.size)
    y, ref = mathf("p", q, alpha), np.power(q, alpha)
    bound = 8.0 * np.abs(alpha * np.log(q)) + 3.0
    assert np.all(_ulp_error(y, ref) <= bound)
    assert np.all(mathf("p", q[:100], 0.0) == 1.0)


def test_sincos_turns_within_2_ulp(mathf):
    import mpmath
    mpmath.mp.dps = 40
    rng = np.random.default_rng(11)
    u = np.concatenate([
        rng.uniform(0.0, 1.0, 4_000),
        np.arange(0, 9) / 8.0,                                   # quarter and eighth turns
        np.arange(0, 9) / 8.0 + 1e-9, np.arange(1, 9) / 8.0 - 1e-9,
        0.5 + rng.uniform(-1e-6, 1e-6, 200), 1.0 - rng.uniform(0.0, 1e-6, 200),
        rng.uniform(0.0, 1e-12, 100),
    ])
    u = u[(u >= 0) & (u <= 1)]
    two_pi = 2 * mpmath.pi
    ref_s = np.array([float(mpmath.sin(two_pi * mpmath.mpf(float(v)))) for v in u])
    ref_c = np.array([float(mpmath.cos(two_pi * mpmath.mpf(float(v)))) for v in u])
    s, c = mathf("s", u), mathf("c", u)
    for y, ref in ((s, ref_s), (c, ref_c)):
        # zeros of sin and cos at whole quarter turns (the 40-digit reference
        # reads about 1e-41 there, the rounding of its own pi)
        exact0 = np.abs(ref) < 1e-30
        assert np.all(np.abs(y[exact0]) <= 1e-300)
        assert _ulp_error(y[~exact0], ref[~exact0]).max() <= 2.0
    # the identities hold to rounding
    assert np.max(np.abs(s * s + c * c - 1.0)) < 4e-16
