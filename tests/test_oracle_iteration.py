"""Pins for one oracle iteration (O5, O6) and whole runs (O7, O8) against
brute force, closed forms and statistics."""
import math

import numpy as np
import pytest

from paper_2010_09341_amd import workloads as W

ERF5_4 = 0.99999999999385016  # erf(5)^4, the 4-D Gaussian with a = 0.1 (mpmath, 30 digits)


def test_moments_match_two_pass_brute_force(orc):
    rng = np.random.default_rng(1)
    e = W.random_grid(rng, 3, 11)
    n = 5000
    I, s, h, bad = orc.iterate(e, W.F_GAUSS, [0.2, 0.3, 0.5, 0.7], n, seed=9, t=2)
    w = orc.weights(e, W.F_GAUSS, [0.2, 0.3, 0.5, 0.7], seed=9, t=2, first=0, count=n)
    mean = np.mean(w)
    var = np.sum((w - mean) ** 2) / n / (n - 1)
    assert bad == 0
    assert abs(I - mean) <= 1e-13 * abs(mean)
    assert abs(s - math.sqrt(var)) <= 1e-10 * math.sqrt(var)


def test_histogram_matches_bincount(orc):
    rng = np.random.default_rng(2)
    dim, nb, n = 4, 9, 4000
    e = W.random_grid(rng, dim, nb)
    I, s, h, _ = orc.iterate(e, W.F_SUM, None, n, seed=1, t=0)
    w = orc.weights(e, W.F_SUM, None, seed=1, t=0, first=0, count=n)
    _, k, _ = orc.points(e, seed=1, t=0, first=0, count=n)
    for d in range(dim):
        ref = np.bincount(k[:, d], weights=w * w, minlength=nb)
        assert np.allclose(h[d], ref, rtol=1e-13, atol=0)
        assert abs(h[d].sum() - np.sum(w * w)) <= 1e-13 * np.sum(w * w)


def test_const_on_uniform_grid(orc):
    for dim, nb in ((1, 2), (5, 50), (16, 50)):
        e = orc.uniform_grid(dim, nb)
        I, s, h, _ = orc.iterate(e, W.F_CONST, None, 3000, seed=0, t=0)
        assert abs(I - 1.0) < dim * nb * 2.0**-52
        assert s < 1e-13
        # counts per bin equal the bincount of the bin indices
        _, k, _ = orc.points(e, 0, 0, 0, 3000)
        assert np.allclose(h[0], np.bincount(k[:, 0], minlength=nb), rtol=1e-13)


def test_rambo_phase_space_volume(orc):
    e = orc.uniform_grid(16, 50)
    I, s, _, bad = orc.iterate(e, W.F_RAMBO24, [1000.0, 0.01, 1.0], 2000, seed=0, t=0)
    Wt = math.pi ** 3 * 1000.0 ** 4 / 96
    assert bad == 0
    assert abs(I - Wt) <= 1e-12 * Wt
    assert s <= 1e-12 * Wt


def test_nonfinite_weights_are_counted(orc):
    """A first bin of zero width puts x1 = 0 exactly; with the cut disabled the
    LO toy's x^-1/2 and 1/s_hat blow up there and the weight is 0 * inf."""
    e = np.array([[0.0, 0.0, 0.5, 0.75, 1.0]] * 4)
    I, s, h, bad = orc.iterate(e, W.F_LO_TOY, [13000.0, 91.19, 2.5, -1.0], 4000, 0, 0)
    assert bad > 0
    assert math.isfinite(I) and math.isfinite(s)
    assert np.all(np.isfinite(h))


def test_gauss4d_run_closed_form(orc):
    wl = W.WORKLOADS["gauss4d"]
    I_t, s_t, e, bad = orc.run(wl.dim, wl.nb, wl.fid, wl.params, wl.n_events, wl.seed,
                               wl.n_iter, wl.alpha)
    I, s, chi2 = orc.combine(I_t, s_t)
    assert bad == 0
    assert abs(I - ERF5_4) < 4 * s
    # adaptation: the last iterations are far more precise than the first
    assert s_t[-1] < 0.1 * s_t[0]
    assert np.all(np.diff(e, axis=1) > 0)


def test_sum_listing_toy(orc):
    """The Sec. 3.1 example: sum of x_i over [0,1]^10 integrates to 5."""
    I_t, s_t, _, _ = orc.run(10, 20, W.F_SUM, None, 20_000, seed=0, n_iter=5, alpha=1.5)
    I, s, _ = orc.combine(I_t, s_t)
    assert abs(I - 5.0) < 4 * s


def test_bw_flat_run(orc):
    m, G = 0.37, 0.02
    I_t, s_t, _, _ = orc.run(3, 50, W.F_BW_FLAT, [m, G], 20_000, seed=4, n_iter=6, alpha=1.5)
    I, s, _ = orc.combine(I_t, s_t)
    assert abs(I - W.bw_flat_closed_form(m, G)) < 4 * s


def test_pull_distribution(orc):
    """Pulls (I - I*)/sigma over 120 seeds are standard normal."""
    a, cs = 0.2, [0.45, 0.6]
    ref = W.gauss_closed_form(2, a, cs)
    e = orc.uniform_grid(2, 10)
    pulls = []
    for seed in range(120):
        I, s, _, _ = orc.iterate(e, W.F_GAUSS, [a] + cs, 2000, seed=seed, t=0)
        pulls.append((I - ref) / s)
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 0.35
    assert 0.75 < pulls.std() < 1.3


def test_whole_run_pulls(orc):
    """Whole runs of the 4-D Gaussian workload (5 iterations x 1e5 events,
    refinement after each but the last, inverse-variance combination) over 240
    seeds: the pulls (I - erf(5)^4)/sigma of the combined results have mean 0
    within 3 standard errors and standard deviation in [0.85, 1.15], and the
    chi^2 per degree of freedom averages to 1 within [0.85, 1.15]. This pins
    the multi-iteration run and the combination's sigma through the closed
    form rather than through the oracle's own formulae."""
    wl = W.WORKLOADS["gauss4d"]
    pulls, chi2 = [], []
    for seed in range(240):
        I_t, s_t, _, bad = orc.run(wl.dim, wl.nb, wl.fid, wl.params, wl.n_events, seed,
                                   wl.n_iter, wl.alpha)
        assert bad == 0
        I, s, c = orc.combine(I_t, s_t)
        pulls.append((I - ERF5_4) / s)
        chi2.append(c)
    pulls = np.array(pulls)
    sd = pulls.std(ddof=1)
    assert abs(pulls.mean()) < 3 * sd / math.sqrt(len(pulls)), (pulls.mean(), sd)
    assert 0.85 <= sd <= 1.15, sd
    assert 0.85 <= np.mean(chi2) <= 1.15, np.mean(chi2)


def test_combine_matches_weighted_average(orc):
    I_t = np.array([1.0, 1.2, 0.9, 1.05])
    s_t = np.array([0.1, 0.2, 0.05, 0.1])
    I, s, chi2 = orc.combine(I_t, s_t)
    w = 1 / s_t ** 2
    assert abs(I - np.average(I_t, weights=w)) < 1e-15
    assert abs(s - 1 / math.sqrt(w.sum())) < 1e-15
    assert abs(chi2 - np.sum((I_t - I) ** 2 * w) / 3) < 1e-13
    I, s, chi2 = orc.combine([2.0, 3.0], [0.5, 0.0])
    assert (I, s) == (3.0, 0.0)
    I, s, chi2 = orc.combine([2.0, 2.0, 2.0], [0.1, 0.3, 0.2])
    assert I == pytest.approx(2.0, abs=1e-15) and chi2 == pytest.approx(0.0, abs=1e-25)


def test_rejects_bad_arguments(orc):
    e = orc.uniform_grid(2, 5)
    with pytest.raises(ValueError):
        orc.iterate(e, 17, None, 100, 0, 0)
    with pytest.raises(ValueError):
        orc.iterate(e, W.F_CONST, None, 1, 0, 0)
    with pytest.raises(ValueError):
        orc.iterate(e, W.F_LO_TOY, None, 100, 0, 0)
    with pytest.raises(ValueError):
        orc.refine(e, np.ones((2, 5)), -1.0)
