"""Pins for the oracle's random source (step O2): Philox4x32-10.

The oracle's Philox is written from Salmon et al. (SC'11). It is checked here
against two independent implementations compiled from their source headers
(PyTorch's ATen engine and rocRAND's engine), and its output words are checked
for uniformity.
"""
import os
import subprocess

import numpy as np
import pytest
from scipy import stats

from paper_2010_09341_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def refs_exe(tmp_path_factory):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    out = str(tmp_path_factory.mktemp("philox") / "philox_refs")
    subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + inc,
                    "-I/opt/rocm/include", os.path.join(HERE, "helpers", "philox_refs.cpp"),
                    "-o", out], check=True)
    return out


def _refs(exe, c, k):
    lines = "\n".join(" ".join(str(int(v)) for v in list(ci) + list(ki)) for ci, ki in zip(c, k))
    res = subprocess.run([exe], input=lines + "\n", capture_output=True, text=True, check=True)
    arr = np.array([[int(v) for v in ln.split()] for ln in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    return arr[:, :4].astype(np.uint32), arr[:, 4:].astype(np.uint32)


def test_philox_matches_aten_and_rocrand(orc, refs_exe):
    rng = np.random.default_rng(1234)
    c, k = W.random_philox_inputs(rng, 20000)
    # a block of small counters with c1 < 2^30 so rocRAND's element offset fits
    c[2:10000, 1] &= (1 << 30) - 1
    aten, roc = _refs(refs_exe, c, k)
    mine = np.stack([orc.philox4x32_10(ci, ki) for ci, ki in zip(c, k)])
    assert np.array_equal(mine, aten)
    ok = c[:, 1] < (1 << 30)
    assert ok.sum() > 9000
    assert np.array_equal(mine[ok], roc[ok])


def test_philox_counter_words_all_matter(orc):
    """Flipping any single input bit changes about half of the 128 output bits."""
    base_c = np.array([5, 0, 3, 1], dtype=np.uint32)
    base_k = np.array([7, 9], dtype=np.uint32)
    ref = orc.philox4x32_10(base_c, base_k)
    flips = []
    for word in range(6):
        for bit in (0, 13, 31):
            c = base_c.copy()
            k = base_k.copy()
            if word < 4:
                c[word] ^= np.uint32(1 << bit)
            else:
                k[word - 4] ^= np.uint32(1 << bit)
            out = orc.philox4x32_10(c, k)
            flips.append(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(out, ref)))
    assert min(flips) > 40 and max(flips) < 90


def test_philox_words_uniform(orc):
    """Chi-square test of the top 8 bits and per-bit balance over 4e5 words."""
    x, k, _ = orc.points(orc.uniform_grid(4, 256), seed=99, t=0, first=0, count=100_000)
    # on the uniform 256-bin grid, the bin index is the top 8 bits of the word
    counts = np.bincount(k.ravel(), minlength=256)
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    p = stats.chi2.sf(chi2, 255)
    assert 1e-4 < p < 1 - 1e-4
