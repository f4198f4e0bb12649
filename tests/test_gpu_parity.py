"""Parity of the HIP path with the FP64 CPU oracle, through the C interface.

FP64 mode must match the oracle within 1e-12 relative: per-event weights, I,
the histogram, and whole runs; sigma, refined edges and the combination within
the bounds that a 1e-12 error of their inputs propagates to (tests/tolerances.py
derives each). FP32-eval mode must stay within 0.1 sigma of the oracle per
iteration, with sigma within 1 %. Inputs are seeded and synthetic
(paper_2010_09341_amd.workloads); nothing here feeds a GPU result into the
oracle.
"""
import math
import zlib

import numpy as np
import pytest

import tolerances as T
from paper_2010_09341_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def vg():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2010_09341_amd import vegas
    vegas.lib()
    return vegas


def _close(a, b, rtol=RTOL, atol=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.all(np.abs(a - b) <= rtol * np.abs(b) + atol)


def _handle(vg, dim, nb, fid=None, params=None, prec=W.FP64, grid=None, t=0):
    h = vg.vegas_create(dim, nb)
    if fid is not None and params is not None:
        vg.vegas_set_params(h, fid, params)
    vg.vegas_set_precision(h, prec)
    if grid is not None:
        vg.vegas_set_grid(h, grid)
    if t:
        vg.vegas_set_iteration(h, t)
    return h


CASES = [
    # (name, dim, nb, fid, params)
    ("const3", 3, 7, W.F_CONST, None),
    ("sum10", 10, 20, W.F_SUM, None),
    ("gauss8", 8, 50, W.F_GAUSS, [0.1]),
    ("gauss5c", 5, 37, W.F_GAUSS, [0.2, 0.3, 0.45, 0.5, 0.6, 0.7]),
    ("lo_toy", 4, 100, W.F_LO_TOY, [13000.0, 91.19, 2.5, 20.0]),
    ("rambo", 16, 50, W.F_RAMBO24, [1000.0, 0.01, 0.0]),
    ("rambo_ps", 16, 50, W.F_RAMBO24, [1000.0, 0.01, 1.0]),
    ("bw5", 5, 30, W.F_BW_FLAT, [0.42, 0.03]),
]


@pytest.mark.parametrize("name,dim,nb,fid,params", CASES, ids=[c[0] for c in CASES])
def test_weights_fp64(vg, orc, name, dim, nb, fid, params):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    grid = W.random_grid(rng, dim, nb)
    seed = (5 << 32) | 17
    t = 3
    first = 2**32 - 1500  # crosses the 32-bit boundary of the event index
    count = 3001
    h = _handle(vg, dim, nb, fid, params, W.FP64, grid, t)
    w_gpu = vg.vegas_dump_weights(h, fid, seed, first, count)
    w_ref = orc.weights(grid, fid, params, seed, t, first, count)
    kap = T.event_kappa(orc, grid, fid, params, seed, t, first, count)
    assert T.weights_close(w_gpu, w_ref, kap), T.weights_excess(w_gpu, w_ref, kap)
    if fid not in (W.F_CONST, W.F_RAMBO24):
        assert np.unique(w_gpu).size > count // 2


@pytest.mark.parametrize("name,dim,nb,fid,params", CASES, ids=[c[0] for c in CASES])
def test_iterate_fp64(vg, orc, name, dim, nb, fid, params):
    rng = np.random.default_rng(1 + zlib.crc32(name.encode()))
    grid = W.random_grid(rng, dim, nb)
    n = 100_003  # several workgroups and a ragged tail
    seed, t = 11, 2
    h = _handle(vg, dim, nb, fid, params, W.FP64, grid, t)
    I, s = vg.vegas_iterate(h, fid, n, seed)
    I_r, s_r, h_r, bad_r = orc.iterate(grid, fid, params, n, seed, t)
    assert vg.vegas_nonfinite(h) == bad_r == 0
    assert _close(I, I_r), (I, I_r)
    assert T.sigma_close(s, s_r, I_r, n), T.sigma_excess(s, s_r, I_r, n)
    hist = vg.vegas_get_hist(h)
    assert T.rel_close(hist, h_r), T.max_rel(hist, h_r)
    assert vg.vegas_get_iteration(h) == t + 1


SHAPES = [(1, 2, 2), (1, 512, 1000), (5, 37, 99_991), (11, 23, 60_001), (12, 20, 30_000),
          (13, 17, 77_777), (32, 64, 50_001), (16, 128, 40_000), (4, 512, 65_536),
          (16, 200, 30_011), (16, 512, 20_000), (32, 256, 12_345)]


@pytest.mark.parametrize("dim,nb,n", SHAPES)
def test_iterate_shapes_fp64(vg, orc, dim, nb, n):
    """Gaussian on random grids across shapes: the minimum (1 dim, 2 bins,
    2 events), the bin maximum, dimensions that leave partial Philox blocks,
    11 and 12 dimensions (kernels built for different workgroup bounds), 32
    dimensions, 2048 cells (four histogram copies in 64 KiB of LDS), 3200
    cells (two copies) and the cell maximum dim * nb = 8192 (one copy)."""
    rng = np.random.default_rng(dim * 1000 + nb)
    grid = W.random_grid(rng, dim, nb)
    params = [0.3] + list(rng.uniform(0.3, 0.7, dim))
    h = _handle(vg, dim, nb, W.F_GAUSS, params, W.FP64, grid)
    I, s = vg.vegas_iterate(h, W.F_GAUSS, n, 123)
    I_r, s_r, h_r, _ = orc.iterate(grid, W.F_GAUSS, params, n, 123, 0)
    assert _close(I, I_r), (I, I_r)
    assert T.sigma_close(s, s_r, I_r, n), T.sigma_excess(s, s_r, I_r, n)
    hist = vg.vegas_get_hist(h)
    assert T.rel_close(hist, h_r), T.max_rel(hist, h_r)


@pytest.mark.parametrize("dim,nb,n", SHAPES)
def test_iterate_shapes_fp32_eval(vg, orc, dim, nb, n):
    """The same shapes in FP32-eval (binary32 map and integrand, binary64
    sums) against the binary64 oracle on the same events. Every event falls in
    the same bin on both sides (the bin index is integer arithmetic on the
    same random word), so each histogram bin, a sum of non-negative w^2 terms,
    and I, a mean of non-negative w, carry at most the per-event relative error
    eps_w of the binary32 weight (twice it for w^2), bounded from the
    arithmetic by tolerances.fp32_gauss_weight_rtol; sigma gets the
    cancellation bound of that error. I also lies within 0.1 sigma wherever
    sigma exceeds the arithmetic's resolution (10 eps_w |I|)."""
    rng = np.random.default_rng(dim * 1000 + nb)
    grid = W.random_grid(rng, dim, nb)
    params = [0.3] + list(rng.uniform(0.3, 0.7, dim))
    eps_w = T.fp32_gauss_weight_rtol(grid, params)
    h = _handle(vg, dim, nb, W.F_GAUSS, params, W.FP32_EVAL, grid)
    I, s = vg.vegas_iterate(h, W.F_GAUSS, n, 123)
    I_r, s_r, h_r, _ = orc.iterate(grid, W.F_GAUSS, params, n, 123, 0)
    assert abs(I - I_r) <= eps_w * abs(I_r), (I, I_r, eps_w)
    if s_r > 10 * eps_w * abs(I_r):
        assert abs(I - I_r) <= 0.1 * s_r, (I, I_r, s_r)
    assert T.sigma_close(s, s_r, I_r, n, eps=2 * eps_w), T.sigma_excess(s, s_r, I_r, n, 2 * eps_w)
    hist = vg.vegas_get_hist(h)
    assert T.rel_close(hist, h_r, eps=2 * eps_w), (T.max_rel(hist, h_r), 2 * eps_w)


@pytest.mark.parametrize("alpha,zeros", [(1.5, 0.0), (1.5, 0.3), (0.0, 0.0), (0.5, 0.1),
                                         (2.0, 0.6)])
@pytest.mark.parametrize("dim,nb", [(1, 2), (3, 50), (8, 100), (2, 512)])
def test_refine_fp64(vg, orc, alpha, zeros, dim, nb):
    rng = np.random.default_rng(int(alpha * 7) + nb + dim)
    grid = W.random_grid(rng, dim, nb)
    hist = W.random_hist(rng, dim, nb, zeros=zeros)
    if dim > 1:
        hist[-1] = 0.0  # an empty dimension keeps its edges
    h = _handle(vg, dim, nb, grid=grid)
    vg.vegas_set_hist(h, hist)
    vg.vegas_refine(h, alpha)
    got = vg.vegas_get_grid(h)
    ref = orc.refine(grid, hist, alpha)
    assert np.all(got[:, 0] == 0.0) and np.all(got[:, -1] == 1.0)
    assert np.all(np.diff(got, axis=1) > 0)
    assert T.edges_close(got, ref, grid, hist, alpha), T.edges_excess(got, ref, grid, hist, alpha)


def test_run_gauss4d_fp64(vg, orc):
    """The 4-D Gaussian workload (5 x 1e5 events, 50 bins, alpha 1.5, seed 0):
    every iteration, the final grid and the combination match the oracle."""
    wl = W.WORKLOADS["gauss4d"]
    h = _handle(vg, wl.dim, wl.nb, wl.fid, wl.params)
    I_t, s_t = vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
    I_r, s_r, e_r, e_prev, h_last = T.oracle_run_steps(orc, wl.dim, wl.nb, wl.fid, wl.params,
                                                       wl.n_events, wl.seed, wl.n_iter, wl.alpha)
    assert _close(I_t, I_r), np.max(np.abs(I_t - I_r) / I_r)
    assert T.sigma_close(s_t, s_r, I_r, wl.n_events), T.sigma_excess(s_t, s_r, I_r, wl.n_events)
    got = vg.vegas_get_grid(h)
    assert T.edges_close(got, e_r, e_prev, h_last, wl.alpha), \
        T.edges_excess(got, e_r, e_prev, h_last, wl.alpha)
    I, s, chi2 = vg.vegas_result(h)
    I_o, s_o, c_o = orc.combine(I_r, s_r)
    assert T.combine_close(I, s, I_r, s_r, I_o, s_o, wl.n_events), (I, I_o, s, s_o)
    assert abs(I - 0.99999999999385016) < 4 * s


def test_iterate_equals_run(vg):
    """vegas_iterate + vegas_refine step by step equals one vegas_run."""
    h1 = _handle(vg, 6, 40, W.F_GAUSS, [0.15])
    h2 = _handle(vg, 6, 40, W.F_GAUSS, [0.15])
    I_run, s_run = vg.vegas_run(h1, W.F_GAUSS, 50_000, 3, 4, 1.5)
    for i in range(4):
        I, s = vg.vegas_iterate(h2, W.F_GAUSS, 50_000, 3)
        assert _close(I, I_run[i], rtol=1e-14)
        if i < 3:
            vg.vegas_refine(h2, 1.5)
    assert np.max(np.abs(vg.vegas_get_grid(h1) - vg.vegas_get_grid(h2))) < 1e-14


@pytest.mark.parametrize("name", ["lo_toy", "rambo24"])
def test_run_physics_fp64(vg, orc, name):
    """The LO toy and RAMBO workloads at reduced event counts, FP64: every
    iteration at 1e-12, sigma and the final grid within their bounds."""
    wl = W.WORKLOADS[name]
    n = 200_000 if name == "lo_toy" else 50_000
    h = _handle(vg, wl.dim, wl.nb, wl.fid, wl.params)
    I_t, s_t = vg.vegas_run(h, wl.fid, n, wl.seed, 4, wl.alpha)
    I_r, s_r, e_r, e_prev, h_last = T.oracle_run_steps(orc, wl.dim, wl.nb, wl.fid, wl.params,
                                                       n, wl.seed, 4, wl.alpha)
    assert _close(I_t, I_r), np.max(np.abs(I_t - I_r) / I_r)
    assert T.sigma_close(s_t, s_r, I_r, n), T.sigma_excess(s_t, s_r, I_r, n)
    got = vg.vegas_get_grid(h)
    assert T.edges_close(got, e_r, e_prev, h_last, wl.alpha), \
        T.edges_excess(got, e_r, e_prev, h_last, wl.alpha)
    I, s, _ = vg.vegas_result(h)
    I_o, s_o, _ = orc.combine(I_r, s_r)
    assert T.combine_close(I, s, I_r, s_r, I_o, s_o, n), (I, I_o, s, s_o)


@pytest.mark.parametrize("name,dim,nb,fid,params", CASES, ids=[c[0] for c in CASES])
def test_iterate_fp32_eval(vg, orc, name, dim, nb, fid, params):
    """FP32-eval: within 0.1 sigma of the FP64 oracle on the same events, and
    sigma within 1%."""
    rng = np.random.default_rng(2 + zlib.crc32(name.encode()))
    grid = W.random_grid(rng, dim, nb, spread=1.5)
    n = 200_000
    h = _handle(vg, dim, nb, fid, params, W.FP32_EVAL, grid, 1)
    I, s = vg.vegas_iterate(h, fid, n, 77)
    I_r, s_r, _, _ = orc.iterate(grid, fid, params, n, 77, 1)
    if s_r > 1e-9 * abs(I_r):
        assert abs(I - I_r) < 0.1 * s_r, (I, I_r, s_r)
        assert abs(s / s_r - 1) < 1e-2
    else:
        assert abs(I - I_r) < 1e-6 * abs(I_r)


def test_fp32_eval_gauss_tails(vg, orc):
    """Narrow 12-D Gaussian (a = 0.05): the outer bins collect w^2 of order
    1e-128, far below the binary32 range; the binary64 weight formed from the
    binary32 log2-sum keeps every bin populated where the oracle's is."""
    dim, nb = 12, 50
    params = [0.05] + [0.5] * dim
    h = _handle(vg, dim, nb, W.F_GAUSS, params, W.FP32_EVAL)
    vg.vegas_iterate(h, W.F_GAUSS, 300_000, 5)
    hist = vg.vegas_get_hist(h)
    _, _, h_r, _ = orc.iterate(orc.uniform_grid(dim, nb), W.F_GAUSS, params, 300_000, 5, 0)
    assert np.all(h_r > 0)
    assert np.all(hist > 0)
    assert _close(hist.sum(axis=1), h_r.sum(axis=1), rtol=1e-3)


def test_nonfinite_counted(vg, orc):
    """LO toy without its cut on a grid whose first bin is 1e-300 wide: the
    weights near x1 = 0 overflow; both sides count the same events."""
    e = np.tile(np.linspace(0, 1, 9), (4, 1))
    e[:, 1] = 1e-300
    params = [13000.0, 91.19, 2.5, -1.0]
    h = _handle(vg, 4, 8, W.F_LO_TOY, params, W.FP64, e)
    I, s = vg.vegas_iterate(h, W.F_LO_TOY, 40_000, 0)
    _, _, _, bad_r = orc.iterate(e, W.F_LO_TOY, params, 40_000, 0, 0)
    assert bad_r > 0
    assert vg.vegas_nonfinite(h) == bad_r
    assert math.isfinite(I) and math.isfinite(s)
    assert np.all(np.isfinite(vg.vegas_get_hist(h)))


def test_full_grid_slot_order(vg, orc):
    """Launches of a whole number of workgroups per CU (the default shape once
    the events fill the GPU) order the event slots per CU; every event is
    still drawn exactly once: an iteration with a ragged last stride matches
    the oracle's estimate and histogram, and a dump on 256 workgroups of 256
    threads (per-CU order on a 256-CU device), the last one partly empty and
    the indices crossing 2^32, matches the oracle event by event."""
    grid = W.random_grid(np.random.default_rng(7), 3, 41)
    n = 1_300_001  # about 2.5 grid strides of 512 x 1024 threads
    h = _handle(vg, 3, 41, W.F_GAUSS, [0.25], W.FP64, grid, 4)
    I, s = vg.vegas_iterate(h, W.F_GAUSS, n, 21)
    I_r, s_r, h_r, bad_r = orc.iterate(grid, W.F_GAUSS, [0.25], n, 21, 4)
    assert bad_r == 0
    assert _close(I, I_r), (I, I_r)
    assert T.sigma_close(s, s_r, I_r, n), T.sigma_excess(s, s_r, I_r, n)
    hist = vg.vegas_get_hist(h)
    assert T.rel_close(hist, h_r), T.max_rel(hist, h_r)

    grid6 = W.random_grid(np.random.default_rng(8), 6, 29)
    seed, t, first, count = (3 << 32) | 5, 2, 2**32 - 30_000, 65_500
    h6 = _handle(vg, 6, 29, W.F_GAUSS, [0.3], W.FP64, grid6, t)
    w = vg.vegas_dump_weights(h6, W.F_GAUSS, seed, first, count)
    w_r = orc.weights(grid6, W.F_GAUSS, [0.3], seed, t, first, count)
    assert T.weights_close(w, w_r), T.max_rel(w, w_r)
    assert np.unique(w).size > count // 2


def test_launch_shape_independence(vg):
    """The estimate does not depend on the launch shape beyond rounding; the
    same shape gives bitwise the same estimate."""
    grid = W.random_grid(np.random.default_rng(3), 7, 33)
    res = []
    for blocks, threads in ((0, 0), (0, 0), (7, 64), (1, 256), (300, 128), (0, 512), (3, 1024),
                            (0, 640), (5, 896), (0, 192)):
        h = _handle(vg, 7, 33, W.F_SUM, None, W.FP64, grid)
        vg.vegas_set_launch(h, blocks, threads)
        res.append(vg.vegas_iterate(h, W.F_SUM, 123_457, 9))
    assert res[0] == res[1]
    for I, s in res[2:]:
        assert _close(I, res[0][0], rtol=1e-14)
    for threads in (-64, 100, 1088):
        with pytest.raises(vg.VegasError) as e:
            vg.vegas_set_launch(h, 0, threads)
        assert e.value.code == vg.VEGAS_EINVAL


def test_workgroup_bound_of_heavy_kernels(vg, orc):
    """Kernels that need more than 128 registers per thread (binary64 above
    12 dimensions and at 11) are built for 256-thread workgroups: asking for 1024
    threads is rejected before any device work, and the handle still runs
    (and matches the oracle) with the default shape."""
    grid = W.random_grid(np.random.default_rng(4), 14, 20)
    h = _handle(vg, 14, 20, W.F_GAUSS, [0.3], W.FP64, grid, 2)
    vg.vegas_set_launch(h, 0, 1024)
    with pytest.raises(vg.VegasError) as e:
        vg.vegas_iterate(h, W.F_GAUSS, 50_000, 1)
    assert e.value.code == vg.VEGAS_EINVAL
    assert vg.vegas_get_iteration(h) == 2
    vg.vegas_set_launch(h, 0, 0)
    I, s = vg.vegas_iterate(h, W.F_GAUSS, 50_000, 1)
    I_r, s_r, _, _ = orc.iterate(grid, W.F_GAUSS, [0.3], 50_000, 1, 2)
    assert _close(I, I_r) and T.sigma_close(s, s_r, I_r, 50_000)


def test_own_memory_matches_torch_memory(vg):
    h1 = vg.vegas_create(5, 20, torch_memory=False)
    h2 = vg.vegas_create(5, 20, torch_memory=True)
    for h in (h1, h2):
        vg.vegas_set_params(h, W.F_GAUSS, [0.2])
    r1 = vg.vegas_run(h1, W.F_GAUSS, 30_000, 1, 3, 1.5)
    r2 = vg.vegas_run(h2, W.F_GAUSS, 30_000, 1, 3, 1.5)
    assert np.allclose(r1[0], r2[0], rtol=1e-14, atol=0)


def test_state_machine(vg):
    h = vg.vegas_create(3, 10)
    with pytest.raises(vg.VegasError) as e:
        vg.vegas_refine(h, 1.5)
    assert e.value.code == vg.VEGAS_ESTATE
    with pytest.raises(vg.VegasError) as e:
        vg.vegas_result(h)
    assert e.value.code == vg.VEGAS_ESTATE
    with pytest.raises(vg.VegasError) as e:
        vg.vegas_iterate(h, W.F_LO_TOY, 100, 0)  # the LO toy needs 4 dimensions
    assert e.value.code == vg.VEGAS_EINVAL
    with pytest.raises(vg.VegasError):
        vg.vegas_iterate(h, W.F_CONST, 1, 0)
    assert vg.vegas_get_iteration(h) == 0
    vg.vegas_iterate(h, W.F_SUM, 1000, 0)
    vg.vegas_refine(h, 1.5)
    with pytest.raises(vg.VegasError):
        vg.vegas_refine(h, 1.5)
    vg.vegas_reset(h)
    assert vg.vegas_get_iteration(h) == 0
    assert np.allclose(vg.vegas_get_grid(h), np.tile(np.arange(11) / 10, (3, 1)), atol=1e-16)
    bad = np.tile(np.linspace(0, 1, 11), (3, 1))
    bad[1, 4] = bad[1, 5]
    with pytest.raises(vg.VegasError):
        vg.vegas_set_grid(h, bad)


def test_graph_replays_match_eager(vg):
    """vegas_run through its captured hipGraph, replayed several times with
    eager work and synchronisations in between, equals eager launches."""
    def make(graph):
        h = vg.vegas_create(8, 50)
        vg.vegas_set_params(h, W.F_GAUSS, [0.1])
        vg.vegas_set_precision(h, W.FP32_EVAL)
        vg.vegas_set_graph(h, graph)
        return h
    hg, he, other = make(True), make(False), make(False)
    for rep in range(4):
        vg.vegas_reset(hg)
        vg.vegas_reset(he)
        I_g, s_g = vg.vegas_run(hg, W.F_GAUSS, 300_000, 5, 6, 1.5)
        vg.vegas_iterate(other, W.F_GAUSS, 100_000, rep)  # unrelated eager work
        I_e, s_e = vg.vegas_run(he, W.F_GAUSS, 300_000, 5, 6, 1.5)
        assert np.all(np.abs(I_g - I_e) <= 1e-13 * np.abs(I_e)), (rep, I_g - I_e)
        assert T.sigma_close(s_g, s_e, I_e, 300_000)
        assert vg.vegas_get_iteration(hg) == 6
    # with kernel timing on, the run launches eagerly and times each iteration
    vg.vegas_timing(hg, True, True)
    vg.vegas_reset(hg)
    I_t, _ = vg.vegas_run(hg, W.F_GAUSS, 300_000, 5, 6, 1.5)
    ms, n = vg.vegas_timing(hg, False)
    assert n == 6 and ms > 0
    assert np.all(np.abs(I_t - I_e) <= 1e-13 * np.abs(I_e))


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_EVAL])
def test_events_limit_batches(vg, orc, prec):
    """An iteration split into launches of at most events_limit events (the
    paper's batching) gives the same run; FP64 still matches the oracle."""
    wl = W.WORKLOADS["gauss4d"]
    ref = None
    for limit in (0, 7_777, 33_333, 100_000):
        h = _handle(vg, wl.dim, wl.nb, wl.fid, wl.params, prec)
        vg.vegas_set_events_limit(h, limit)
        I_t, s_t = vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
        I1, s1 = vg.vegas_iterate(h, wl.fid, 54_321, 3)
        if ref is None:
            ref = (I_t, s_t, I1)
            continue
        assert np.all(np.abs(I_t - ref[0]) <= 1e-13 * np.abs(ref[0])), limit
        assert T.sigma_close(s_t, ref[1], ref[0], wl.n_events)
        assert abs(I1 - ref[2]) <= 1e-13 * abs(ref[2])
    if prec == W.FP64:
        I_r, s_r, _, _ = orc.run(wl.dim, wl.nb, wl.fid, wl.params, wl.n_events, wl.seed,
                                 wl.n_iter, wl.alpha)
        assert np.all(np.abs(I_t - I_r) <= 1e-12 * np.abs(I_r))


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_EVAL])
def test_checkpoint_resume(vg, orc, prec):
    """A run saved after 3 of 6 iterations and resumed in a fresh handle: the
    resumed iterations, the final grid and the combination match the oracle's
    uninterrupted run (FP64 at 1e-12 and the derived bounds; FP32-eval within
    0.1 sigma) and, to rounding, the uninterrupted GPU run; a record for
    another shape, or a truncated one, is rejected without changing the
    handle."""
    wl = W.WORKLOADS["gauss4d"]
    n, seed = 200_000, 9
    I_r, s_r, e_r, e_prev, h_last = T.oracle_run_steps(orc, wl.dim, wl.nb, wl.fid, wl.params,
                                                       n, seed, 6, 1.5)
    full = _handle(vg, wl.dim, wl.nb, wl.fid, wl.params, prec)
    I_full, s_full = vg.vegas_run(full, wl.fid, n, seed, 6, 1.5)
    a = _handle(vg, wl.dim, wl.nb, wl.fid, wl.params, prec)
    I_a, s_a = vg.vegas_run(a, wl.fid, n, seed, 3, 1.5)
    state = vg.vegas_save(a)
    del a
    b = vg.vegas_create(wl.dim, wl.nb)
    vg.vegas_load(b, state)
    assert vg.vegas_get_iteration(b) == 3
    vg.vegas_refine(b, 1.5)
    I_b, s_b = vg.vegas_run(b, wl.fid, n, seed, 3, 1.5)
    I_t, s_t = np.concatenate([I_a, I_b]), np.concatenate([s_a, s_b])
    assert np.allclose(I_t, I_full, rtol=1e-13, atol=0)
    I, s, _ = vg.vegas_result(b)
    I_o, s_o, _ = orc.combine(I_r, s_r)
    if prec == W.FP64:
        assert _close(I_t, I_r), np.max(np.abs(I_t - I_r) / I_r)
        assert T.sigma_close(s_t, s_r, I_r, n), T.sigma_excess(s_t, s_r, I_r, n)
        got = vg.vegas_get_grid(b)
        assert T.edges_close(got, e_r, e_prev, h_last, 1.5), \
            T.edges_excess(got, e_r, e_prev, h_last, 1.5)
        assert T.combine_close(I, s, I_r, s_r, I_o, s_o, n), (I, I_o, s, s_o)
    else:
        assert np.all(np.abs(I_t - I_r) < 0.1 * s_r), (I_t - I_r) / s_r
        assert np.all(np.abs(s_t / s_r - 1) < 1e-2)
        assert abs(I - I_o) < 0.1 * s_o
    other = vg.vegas_create(wl.dim + 1, wl.nb)
    with pytest.raises(vg.VegasError):
        vg.vegas_load(other, state)
    with pytest.raises(vg.VegasError):
        vg.vegas_load(b, state[:-8])
    assert vg.vegas_get_iteration(other) == 0
    assert vg.vegas_get_iteration(b) == 6


def _narrow_grid(rng, dim, nb, narrow_dims, width=1e-12):
    """A random grid whose first bin is `width` wide in each of narrow_dims."""
    e = W.random_grid(rng, dim, nb)
    for d in narrow_dims:
        e[d, 1] = width
    return e


NARROW = [(16, [0, 1, 2, 3, 9, 14]), (32, [0, 1, 2, 3, 12, 13, 14, 15, 20, 31])]


@pytest.mark.parametrize("dim,narrow", NARROW, ids=["16d", "32d"])
def test_narrow_bins_weights(vg, orc, dim, narrow):
    """Grids whose first bin is 1e-12 wide in several dimensions, four of them
    in one Philox block (so that one event can fall into four such bins at
    once: a Jacobian factor of (nb 1e-12)^4 from that block alone). FP64
    weights equal the oracle's at 1e-12 relative event by event. FP32-eval
    weights equal them to binary32 accuracy: the log2 of the Jacobian is a sum
    over pairs of dimensions of P = log2(nb^2 Delta_a Delta_b) (binary32
    widths, each within 2^-24 relative, two binary32 products, a hardware
    log2 within 2^-23 of |P|), so the weight carries a relative error of at
    most 4 * 2^-24 per pair plus ln2 * 2^-24 * (pairs + 4) * (sum |P| +
    |log2 f|) from those roundings and the sums (the pairs' nb^2 Delta Delta,
    down to (4e-12)^2 here, stay in the normal binary32 range); each binary32
    coordinate is off by at most 2^-23, which moves ln f of the Gaussian
    (width a, centres 0.25) by at most 2 * 0.75 / a^2 * 2^-23 per dimension;
    1e-6 covers the final exp2 and scaling."""
    nb = 4
    rng = np.random.default_rng(100 + dim)
    grid = _narrow_grid(rng, dim, nb, narrow)
    params = [0.3] + [0.25] * dim
    seed, t, first, count = 77, 1, 0, 20_000
    x, k, _ = orc.points(grid, seed, t, first, count)
    hits = np.sum(k[:, narrow[:4]] == 0, axis=1)
    assert np.sum(hits == 4) > 10  # events in four narrow bins of one block
    w_ref = orc.weights(grid, W.F_GAUSS, params, seed, t, first, count)
    h = _handle(vg, dim, nb, W.F_GAUSS, params, W.FP64, grid, t)
    w = vg.vegas_dump_weights(h, W.F_GAUSS, seed, first, count)
    assert T.weights_close(w, w_ref), T.max_rel(w, w_ref)
    vg.vegas_set_precision(h, W.FP32_EVAL)
    w32 = vg.vegas_dump_weights(h, W.F_GAUSS, seed, first, count)
    widths = np.diff(grid, axis=1)
    wk = widths[np.arange(dim)[None, :], k]
    P = np.log2(nb * wk[:, 0::2]) + np.log2(nb * wk[:, 1::2])  # dim is even here
    log2f = np.log2(w_ref) - np.sum(P, axis=1)
    pairs = dim // 2
    budget = 4 * 2.0**-24 * pairs + math.log(2) * 2.0**-24 * (pairs + 4) * (
        np.sum(np.abs(P), axis=1) + np.abs(log2f))
    budget += dim * 2.0 * 0.75 / params[0] ** 2 * 2.0**-23 + 1e-6
    rel = np.abs(w32 - w_ref) / w_ref
    assert np.all(rel <= budget), np.max(rel / budget)


@pytest.mark.parametrize("dim,narrow", NARROW, ids=["16d", "32d"])
def test_narrow_bins_iterate(vg, orc, dim, narrow):
    """One iteration on those grids: FP64 matches the oracle (I at 1e-12,
    sigma and histogram within their bounds), FP32-eval within 0.1 sigma."""
    nb = 4
    rng = np.random.default_rng(200 + dim)
    grid = _narrow_grid(rng, dim, nb, narrow)
    params = [0.3] + [0.25] * dim
    n, seed, t = 300_000, 5, 2
    I_r, s_r, h_r, bad = orc.iterate(grid, W.F_GAUSS, params, n, seed, t)
    assert bad == 0
    h = _handle(vg, dim, nb, W.F_GAUSS, params, W.FP64, grid, t)
    I, s = vg.vegas_iterate(h, W.F_GAUSS, n, seed)
    assert _close(I, I_r), (I, I_r)
    assert T.sigma_close(s, s_r, I_r, n), T.sigma_excess(s, s_r, I_r, n)
    hist = vg.vegas_get_hist(h)
    assert T.rel_close(hist, h_r), T.max_rel(hist, h_r)
    h32 = _handle(vg, dim, nb, W.F_GAUSS, params, W.FP32_EVAL, grid, t)
    I32, s32 = vg.vegas_iterate(h32, W.F_GAUSS, n, seed)
    assert abs(I32 - I_r) < 0.1 * s_r, (I32 - I_r) / s_r
    assert abs(s32 / s_r - 1) < 1e-2


def test_rebind_workspace_after_captured_run(vg, orc):
    """A workspace bound after a run was captured in a hipGraph: the next run
    of the same configuration works in the new workspace (the graph of the
    old one is dropped) and matches the oracle, grid included."""
    import torch
    wl = W.WORKLOADS["gauss4d"]
    I_r, s_r, e_r, e_prev, h_last = T.oracle_run_steps(orc, wl.dim, wl.nb, wl.fid, wl.params,
                                                       wl.n_events, wl.seed, wl.n_iter, wl.alpha)
    h = _handle(vg, wl.dim, wl.nb, wl.fid, wl.params)
    vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
    nbytes = vg.vegas_workspace_bytes(wl.dim, wl.nb)
    ws2 = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    vg.vegas_bind_workspace(h, (ws2.data_ptr() + 255) & ~255, nbytes)
    h.workspace = ws2  # the old workspace tensor is released here
    moved = vg.vegas_get_grid(h)  # state moved along
    assert T.edges_close(moved, e_r, e_prev, h_last, wl.alpha)
    vg.vegas_reset(h)
    I_t, s_t = vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
    assert _close(I_t, I_r), np.max(np.abs(I_t - I_r) / I_r)
    assert T.sigma_close(s_t, s_r, I_r, wl.n_events), T.sigma_excess(s_t, s_r, I_r, wl.n_events)
    got = vg.vegas_get_grid(h)
    assert T.edges_close(got, e_r, e_prev, h_last, wl.alpha), \
        T.edges_excess(got, e_r, e_prev, h_last, wl.alpha)


def test_handles_in_threads(vg, orc):
    """Distinct handles are independent: four threads each run a whole FP64
    run (captured graph, own stream) on their own handle at the same time;
    every run matches the oracle's at the bounds the single-threaded run
    tests use."""
    import threading
    runs = [(3, 20, W.F_GAUSS, [0.2], 40_000, 1, 4), (5, 32, W.F_BW_FLAT, [0.4, 0.02], 30_011, 2, 3),
            (8, 50, W.F_GAUSS, [0.1], 100_000, 3, 3), (2, 64, W.F_SUM, None, 20_000, 4, 5)]
    got, errors = {}, []

    def worker(i, dim, nb, fid, params, n, seed, n_iter):
        try:
            h = _handle(vg, dim, nb, fid, params, W.FP64)
            for _ in range(3):  # the later runs replay the captured graph
                vg.vegas_reset(h)
                got[i] = vg.vegas_run(h, fid, n, seed, n_iter, 1.5)
            vg.vegas_destroy(h)
        except Exception as e:  # noqa: BLE001 - reported by the assertion below
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(i,) + r) for i, r in enumerate(runs)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=180.0)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    for i, (dim, nb, fid, params, n, seed, n_iter) in enumerate(runs):
        I_r, s_r, _, _ = orc.run(dim, nb, fid, params, n, seed, n_iter, 1.5)
        I_t, s_t = got[i]
        assert _close(I_t, I_r), (i, I_t, I_r)
        assert T.sigma_close(s_t, s_r, I_r, n), (i, T.sigma_excess(s_t, s_r, I_r, n))
