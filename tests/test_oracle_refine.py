"""Pins for the oracle's grid refinement (step O7).

Identities (constant histogram, alpha = 0, two bins), invariants (outer edges,
monotonicity, equal compressed mass per new bin checked in 40-digit
arithmetic), a hand-worked three-bin case, and the classic property that a
separable integrand's grid converges towards the equal-integral quantiles of
its one-dimensional factor.
"""
import math

import mpmath
import numpy as np
import pytest

from paper_2010_09341_amd import workloads as W


def test_constant_histogram_is_identity(orc):
    rng = np.random.default_rng(1)
    e = W.random_grid(rng, 3, 12)
    new = orc.refine(e, np.full((3, 12), 4.5), 1.5)
    assert np.allclose(new, e, rtol=0, atol=1e-15)


def test_alpha_zero_is_identity(orc):
    rng = np.random.default_rng(2)
    e = W.random_grid(rng, 2, 30)
    h = W.random_hist(rng, 2, 30)
    new = orc.refine(e, h, 0.0)
    assert np.allclose(new, e, rtol=0, atol=1e-15)


def test_two_bins_is_identity(orc):
    """With two bins the smoothed values are equal, whatever the histogram."""
    e = np.array([[0.0, 0.3, 1.0]])
    new = orc.refine(e, np.array([[1.0, 100.0]]), 1.5)
    assert np.allclose(new, e, rtol=0, atol=1e-16)


def test_empty_histogram_leaves_grid(orc):
    rng = np.random.default_rng(3)
    e = W.random_grid(rng, 2, 8)
    h = W.random_hist(rng, 2, 8)
    h[1] = 0.0
    new = orc.refine(e, h, 1.5)
    assert np.array_equal(new[1], e[1])
    assert not np.allclose(new[0], e[0])


def test_hand_worked_three_bins(orc):
    """h = (0, 0, 1) on the uniform 3-bin grid, alpha = 1:
    smoothed s = (0, 1/3, 1/2), p = (0, 2/5, 3/5),
    r = (0, (3/5)/ln(5/2), (2/5)/ln(5/3)), delta = (r1 + r2)/3.
    r1 = 0.65480..., r2 = 0.78304..., delta = 0.47928..., so edge 1 falls in
    bin 1 at fraction delta/r1 and edge 2 in bin 2 at (2 delta - r1)/r2."""
    r1 = 0.6 / math.log(2.5)
    r2 = 0.4 / math.log(5 / 3)
    delta = (r1 + r2) / 3
    assert delta < r1 < 2 * delta < r1 + r2
    e1 = 1 / 3 + (delta / r1) / 3
    e2 = 2 / 3 + ((2 * delta - r1) / r2) / 3
    new = orc.refine(orc.uniform_grid(1, 3), np.array([[0.0, 0.0, 1.0]]), 1.0)
    assert np.allclose(new[0], [0.0, e1, e2, 1.0], rtol=0, atol=1e-15)


def _compressed_mass_check(e_old, h, alpha, e_new):
    """Recompute, in 40-digit arithmetic, the compressed weights r and check
    that every new bin holds C_nb/nb of the piecewise-uniform r density."""
    mpmath.mp.dps = 40
    nb = len(h)
    hh = [mpmath.mpf(float(v)) for v in h]
    s = [(hh[0] + hh[1]) / 2] + [(hh[i - 1] + hh[i] + hh[i + 1]) / 3 for i in range(1, nb - 1)] \
        + [(hh[nb - 2] + hh[nb - 1]) / 2]
    S = sum(s)
    r = []
    for v in s:
        p = v / S
        r.append(mpmath.mpf(0) if p == 0 else ((1 - p) / (-mpmath.log(p))) ** alpha)
    R = sum(r)
    eo = [mpmath.mpf(float(v)) for v in e_old]

    def cdf(x):
        x = mpmath.mpf(float(x))
        acc = mpmath.mpf(0)
        for k in range(nb):
            if x >= eo[k + 1]:
                acc += r[k]
            elif x > eo[k]:
                acc += r[k] * (x - eo[k]) / (eo[k + 1] - eo[k])
        return acc

    for j in range(1, nb):
        assert abs(cdf(e_new[j]) - j * R / nb) < 1e-12 * R


@pytest.mark.parametrize("alpha,zeros", [(1.5, 0.0), (1.5, 0.3), (0.5, 0.1), (2.0, 0.0)])
def test_equal_compressed_mass(orc, alpha, zeros):
    rng = np.random.default_rng(int(alpha * 10) + int(zeros * 100))
    dim, nb = 2, 25
    e = W.random_grid(rng, dim, nb)
    h = W.random_hist(rng, dim, nb, zeros=zeros)
    new = orc.refine(e, h, alpha)
    for d in range(dim):
        assert new[d, 0] == 0.0 and new[d, -1] == 1.0
        assert np.all(np.diff(new[d]) > 0)
        _compressed_mass_check(e[d], h[d], alpha, new[d])


def test_refinement_concentrates_on_peak(orc):
    """A separable peaked integrand pulls the edges towards its peak: after a
    few iterations the central bins of a Gaussian are much narrower than the
    outer ones, and symmetric about the centre."""
    dim, nb = 2, 20
    I_t, s_t, e, _ = orc.run(dim, nb, W.F_GAUSS, [0.1], 50_000, seed=1, n_iter=8, alpha=1.5)
    widths = np.diff(e, axis=1)
    for d in range(dim):
        assert widths[d, nb // 2] < 0.3 * widths[d, 0]
        # the grid is roughly symmetric about 0.5
        assert np.allclose(e[d], 1 - e[d][::-1], atol=0.02)
