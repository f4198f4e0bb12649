"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (default launch shape, captured-graph runs), against the FP64 oracle's
own full runs stored in tests/golden/ (written by tests/golden/make_golden.py,
which calls only the oracle):

- the 8-D Gaussian (10 iterations x 1e7 events), the LO 2->2 toy (10 x 1e8)
  and massless 2->4 RAMBO (10 x 5e7), seed 0: FP64 matches every iteration's
  I at 1e-12 and sigma, the final grid and the combination within the bounds
  of tests/tolerances.py; FP32-eval stays within 0.1 sigma of every
  iteration, with sigma within 1 %;
- per-event weights sampled across the LO toy's and RAMBO's whole event
  ranges on the uniform grid, one by one: FP64 at 1e-12, FP32-eval to
  binary32 accuracy.
"""
import numpy as np
import pytest

import tolerances as T
from golden import make_golden as G
from paper_2010_09341_amd import workloads as W

pytestmark = pytest.mark.gpu

NAMES = ["gauss8d", "lo_toy", "rambo24"]


@pytest.fixture(scope="module")
def vg():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2010_09341_amd import vegas
    vegas.lib()
    return vegas


def _handle(vg, wl, prec):
    h = vg.vegas_create(wl.dim, wl.nb)
    vg.vegas_set_params(h, wl.fid, wl.params)
    vg.vegas_set_precision(h, prec)
    return h


def _golden(name):
    rec, I_r, s_r, e_r = G.load(name)
    wl = W.WORKLOADS[name]
    assert (rec["dim"], rec["n_bins"], rec["n_events"], rec["n_iter"], rec["seed"]) == \
        (wl.dim, wl.nb, wl.n_events, wl.n_iter, wl.seed)
    return wl, I_r, s_r, e_r


@pytest.mark.parametrize("name", NAMES)
def test_full_fp64(vg, orc, name):
    wl, I_r, s_r, e_r = _golden(name)
    h = _handle(vg, wl, W.FP64)
    I_t, s_t = vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
    assert vg.vegas_nonfinite(h) == 0
    assert T.rel_close(I_t, I_r), T.max_rel(I_t, I_r)
    assert T.sigma_close(s_t, s_r, I_r, wl.n_events), T.sigma_excess(s_t, s_r, I_r, wl.n_events)
    I, s, _ = vg.vegas_result(h)
    I_o, s_o, _ = orc.combine(I_r, s_r)
    assert T.combine_close(I, s, I_t, s_t, I_o, s_o, wl.n_events), (I, I_o, s, s_o)
    hist = vg.vegas_get_hist(h)
    sums = hist.sum(axis=1)
    assert np.all(np.abs(sums - sums[0]) <= 1e-12 * sums[0])
    # The stored run does not keep the last refinement's inputs: the final
    # edges get the refined-edge bound of the GPU's own grid and histogram
    # before that refinement, which agree with the oracle's to rounding (every
    # iteration's I does, above).
    got = vg.vegas_get_grid(h)
    vg.vegas_reset(h)
    vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter - 1, wl.alpha)
    e_prev, h_last = vg.vegas_get_grid(h), vg.vegas_get_hist(h)
    assert T.edges_close(got, e_r, e_prev, h_last, wl.alpha), \
        T.edges_excess(got, e_r, e_prev, h_last, wl.alpha)


@pytest.mark.parametrize("name", NAMES)
def test_full_fp32_eval(vg, orc, name):
    wl, I_r, s_r, _ = _golden(name)
    h = _handle(vg, wl, W.FP32_EVAL)
    I_t, s_t = vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
    assert vg.vegas_nonfinite(h) == 0
    assert np.all(np.abs(I_t - I_r) < 0.1 * s_r), (I_t - I_r) / s_r
    assert np.all(np.abs(s_t / s_r - 1) < 1e-2), s_t / s_r - 1
    I, s, _ = vg.vegas_result(h)
    I_o, s_o, _ = orc.combine(I_r, s_r)
    assert abs(I - I_o) < 0.1 * s_o, (I - I_o) / s_o
    if name == "gauss8d":
        assert abs(I - W.gauss_closed_form(8, 0.1)) < 4 * s


def _windows(n):
    return [0, n // 3, n // 2 + 12345, n - 2000]


@pytest.mark.parametrize("name", ["lo_toy", "rambo24"])
def test_full_size_sampled_weights(vg, orc, name):
    """Per-event weights on the uniform grid at four windows spanning the
    workload's event range, including its last event: FP64 at 1e-12 relative
    plus the integrand's conditioning (tests/tolerances.py);
    FP32-eval within 2e-4 relative (the binary32 map, integrand and log2
    Jacobian; RAMBO's boost and s_ij products lose a few more bits) plus
    1e-12 of the largest weight (a binary32 coordinate within an ulp of 1
    makes the LO toy's (1 - x)^3 lose all its bits, on weights that small),
    except that a binary32 cut variable within an ulp of its threshold may
    flip the cut (at most 2 events per window)."""
    wl = W.WORKLOADS[name]
    e = orc.uniform_grid(wl.dim, wl.nb)
    for prec in (W.FP64, W.FP32_EVAL):
        h = _handle(vg, wl, prec)
        for first in _windows(wl.n_events):
            w = vg.vegas_dump_weights(h, wl.fid, wl.seed, first, 2000)
            w_r = orc.weights(e, wl.fid, wl.params, wl.seed, 0, first, 2000)
            if prec == W.FP64:
                kap = T.event_kappa(orc, e, wl.fid, wl.params, wl.seed, 0, first, 2000)
                assert T.weights_close(w, w_r, kap), (name, first, T.weights_excess(w, w_r, kap))
            else:
                bad = np.abs(w - w_r) > 2e-4 * np.abs(w_r) + 1e-12 * np.max(np.abs(w_r))
                assert bad.sum() <= 2, (name, first, bad.sum())
