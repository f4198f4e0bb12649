"""vegas_iterate_noalloc (the entry point that allocates nothing) against
vegas_iterate on a handle holding the same grid and iteration counter: two
calls in a row, the second with a smaller grid and fewer events, in both
precisions, through the C interface. FP64 is also held to the oracle."""
import numpy as np
import pytest

import tolerances as T
from paper_2010_09341_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2010_09341_amd import vegas
    vegas.lib()
    return vegas


CALLS = [
    # (dim, nb, fid, params, n_events, seed, t): the second smaller than the first
    (8, 50, W.F_GAUSS, [0.1], 3_000_001, (7 << 32) | 3, 2),
    (3, 17, W.F_BW_FLAT, [0.42, 0.03], 40_003, 9, 5),
]


def _handle_iteration(vg, dim, nb, fid, params, prec, grid, n, seed, t):
    h = vg.vegas_create(dim, nb)
    vg.vegas_set_params(h, fid, params)
    vg.vegas_set_precision(h, prec)
    vg.vegas_set_grid(h, grid)
    vg.vegas_set_iteration(h, t)
    I, s = vg.vegas_iterate(h, fid, n, seed)
    hist = vg.vegas_get_hist(h)
    vg.vegas_destroy(h)
    return I, s, hist


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_EVAL], ids=["fp64", "fp32_eval"])
def test_noalloc_matches_vegas_iterate(vg, orc, prec):
    import torch
    stream = torch.cuda.Stream()
    for i, (dim, nb, fid, params, n, seed, t) in enumerate(CALLS):
        grid = W.random_grid(np.random.default_rng(40 + i), dim, nb)
        I_h, s_h, hist_h = _handle_iteration(vg, dim, nb, fid, params, prec, grid, n, seed, t)
        edges = torch.tensor(grid, dtype=torch.float64, device="cuda")
        hist = torch.full((dim, nb), -1.0, dtype=torch.float64, device="cuda")
        res = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        vg.vegas_iterate_noalloc(dim, nb, prec, fid, params, edges.data_ptr(), n, seed, t,
                                 hist.data_ptr(), res.data_ptr(), stream.cuda_stream)
        stream.synchronize()
        r = res.cpu().numpy()
        hh = hist.cpu().numpy()
        # same kernels, same launch shape, same grid and counter: I to the
        # bound, sigma to its derived bound, the histogram bin by bin (sums of
        # non-negative terms whose atomic order differs)
        assert abs(r[0] - I_h) <= 1e-12 * abs(I_h), (i, r[0], I_h)
        assert T.sigma_close(r[1], s_h, I_h, n), T.sigma_excess(r[1], s_h, I_h, n)
        assert r[2] == 0.0 and r[3] == t
        assert T.rel_close(hh, hist_h), T.max_rel(hh, hist_h)
        # without a histogram output (kept in the scratch array): the same
        # (I, sigma), bit for bit (fixed-order sums)
        res2 = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
        vg.vegas_iterate_noalloc(dim, nb, prec, fid, params, edges.data_ptr(), n, seed, t,
                                 0, res2.data_ptr(), stream.cuda_stream)
        stream.synchronize()
        assert np.array_equal(res2.cpu().numpy(), r), (res2.cpu().numpy(), r)
        if prec == W.FP64:
            I_o, s_o, h_o, bad = orc.iterate(grid, fid, params, n, seed, t)
            assert abs(r[0] - I_o) <= 1e-12 * abs(I_o), (i, r[0], I_o)
            assert T.sigma_close(r[1], s_o, I_o, n), T.sigma_excess(r[1], s_o, I_o, n)
            assert T.rel_close(hh, h_o), T.max_rel(hh, h_o)


def test_noalloc_rejections(vg):
    import torch
    edges = torch.zeros(4096, dtype=torch.float64, device="cuda")
    res = torch.zeros(4, dtype=torch.float64, device="cuda")
    bad = [
        (33, 10, W.FP64, W.F_CONST, 1000),      # dim above the maximum
        (32, 257, W.FP64, W.F_CONST, 1000),     # more cells than the scratch array holds
        (4, 10, 7, W.F_CONST, 1000),            # unknown precision
        (4, 10, W.FP64, vg.VEGAS_F_USER, 1000),  # run-time integrands are not served
        (4, 10, W.FP64, W.F_CONST, 1),          # too few events
    ]
    for dim, nb, prec, fid, n in bad:
        with pytest.raises(vg.VegasError) as e:
            vg.vegas_iterate_noalloc(dim, nb, prec, fid, None, edges.data_ptr(), n, 0, 0, 0,
                                     res.data_ptr(), 0)
        assert e.value.code == vg.VEGAS_EINVAL, (dim, nb, prec, fid, n)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_EVAL], ids=["fp64", "fp32_eval"])
def test_noalloc_under_graph_capture(vg, prec):
    """The callers it is for: one iteration captured into a hipGraph by torch
    (global capture mode, in which an allocation anywhere in the process makes
    the capture fail), replayed three times with eager work and
    synchronisations between the replays; every replay reproduces the eager
    call's (I, sigma) exactly and its histogram to rounding (atomics add in no
    fixed order)."""
    import torch
    dim, nb, fid, params, n, seed, t = 5, 30, W.F_GAUSS, [0.2], 500_000, 21, 3
    grid = W.random_grid(np.random.default_rng(77), dim, nb)
    edges = torch.tensor(grid, dtype=torch.float64, device="cuda")
    hist = torch.zeros((dim, nb), dtype=torch.float64, device="cuda")
    res = torch.zeros(4, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        vg.vegas_iterate_noalloc(dim, nb, prec, fid, params, edges.data_ptr(), n, seed, t,
                                 hist.data_ptr(), res.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    r_eager, h_eager = res.cpu().numpy().copy(), hist.cpu().numpy().copy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        vg.vegas_iterate_noalloc(dim, nb, prec, fid, params, edges.data_ptr(), n, seed, t,
                                 hist.data_ptr(), res.data_ptr(), stream.cuda_stream)
    for rep in range(3):
        res.fill_(-1.0)
        hist.fill_(-1.0)
        other = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(res.cpu().numpy(), r_eager), (rep, res.cpu().numpy(), r_eager)
        assert T.rel_close(hist.cpu().numpy(), h_eager), (rep, T.max_rel(hist.cpu().numpy(), h_eager))
        assert torch.isfinite(other)
