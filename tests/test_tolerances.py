"""The parity bounds of tests/tolerances.py: an alternative but equally valid
order of the same binary64 arithmetic stays inside them, and a planted error
just above them fails."""
import math

import numpy as np

import tolerances as T
from paper_2010_09341_amd import workloads as W


def _rebin_other_order(edges, hist, alpha):
    """Re-binning with the running sums taken as 64 contiguous segments plus a
    scan of the segment totals, compression as exp(alpha log q), and a
    pairwise total: a different rounding order than the oracle's."""
    out = np.array(edges, dtype=np.float64)
    for d, h in enumerate(hist):
        nb = len(h)
        s = np.empty(nb)
        s[0] = (h[0] + h[1]) / 2
        s[-1] = (h[-2] + h[-1]) / 2
        s[1:-1] = (h[:-2] + h[1:-1] + h[2:]) / 3
        S = math.fsum(s)
        if not S > 0:
            continue
        p = s / S
        r = np.zeros(nb)
        m = (p > 0) & (p < 1)
        r[m] = np.exp(alpha * np.log((1 - p[m]) / -np.log(p[m])))
        r[p >= 1] = 1.0
        seg = -(-nb // 64)
        C = np.zeros(nb + 1)
        off = 0.0
        for lo in range(0, nb, seg):
            c = off
            for i in range(lo, min(lo + seg, nb)):
                c += r[i]
                C[i + 1] = c
            off = c
        delta = C[-1] / nb
        e = edges[d]
        for j in range(1, nb):
            t = j * delta
            k = int(np.searchsorted(C[1:], t, side="left"))
            k = min(k, nb - 1)
            out[d, j] = e[k] + (t - C[k]) / r[k] * (e[k + 1] - e[k])
    return out


def test_refined_edges_bound(orc):
    for seed, (dim, nb, zeros) in enumerate([(3, 50, 0.0), (2, 512, 0.3), (4, 100, 0.6)]):
        rng = np.random.default_rng(seed)
        e = W.random_grid(rng, dim, nb)
        h = W.random_hist(rng, dim, nb, zeros=zeros)
        ref = orc.refine(e, h, 1.5)
        other = _rebin_other_order(e, h, 1.5)
        tol = T.edges_tol(e, h, 1.5, ref)
        assert np.all(np.abs(other - ref) <= tol)
        bad = ref.copy()
        j = nb // 2
        bad[0, j] += 2 * tol[0, j]
        assert not T.edges_close(bad, ref, e, h, 1.5)


def test_sigma_bound():
    # weights that vary little: v small, a large amplification
    assert T.sigma_rtol(1.0, 1e-6, 10**6) > 1e-9
    # v of order one: the bound is close to EPS
    assert T.sigma_rtol(1.0, 1e-3, 10**6) < 3e-12
    assert T.sigma_close([1.0 + 1e-13], [1.0], 1.0, 10**6)
    assert not T.sigma_close([1.0 + 1e-11], [1.0], 1.0, 10**6)


def test_weights_bound():
    assert T.weights_close([1.0, 0.0, 1e-310], [1.0 + 5e-13, 0.0, 1e-310 + 1e-325])
    assert not T.weights_close([1.0 + 2e-12], [1.0])
    assert not T.weights_close([1e-300], [0.0])


def test_kappa_bound(orc):
    """event_kappa is the Gaussian's closed-form condition number
    sum_d |2 x_d (x_d - c) / a^2|, and the LO toy's weights recomputed at
    points moved by up to 4 ulps per coordinate (what two correctly rounded
    maps may differ by) stay inside weights_close with kappa."""
    rng = np.random.default_rng(3)
    grid = W.random_grid(rng, 3, 20)
    x, _, jac = orc.points(grid, 11, 2, 0, 200)
    kap = T.event_kappa(orc, grid, W.F_GAUSS, [0.2], 11, 2, 0, 200)
    exact = np.sum(np.abs(2 * x * (x - 0.5) / 0.04), axis=1)
    assert np.allclose(kap, exact, rtol=1e-6, atol=1e-9)

    params = [13000.0, 91.19, 2.5, 20.0]
    grid = W.random_grid(np.random.default_rng(4), 4, 100)
    n = 3000
    x, _, jac = orc.points(grid, 5, 1, 2**32 - 1500, n)
    w_ref = orc.weights(grid, W.F_LO_TOY, params, 5, 1, 2**32 - 1500, n)
    kap = T.event_kappa(orc, grid, W.F_LO_TOY, params, 5, 1, 2**32 - 1500, n)
    moved = x * (1.0 + rng.uniform(-4, 4, size=x.shape) * T.U)
    w_alt = np.array([orc.integrand(W.F_LO_TOY, moved[i], params) for i in range(n)]) * jac
    assert T.weights_close(w_alt, w_ref, kap), T.weights_excess(w_alt, w_ref, kap)
    assert kap.max() > 1e3  # points within about 1e-3 of x = 1 occur


def _fp32_gauss_weights(orc, grid, params, seed, t, first, count):
    """The Gaussian's weights by one binary32 evaluation of the steps the
    bound fp32_gauss_weight_rtol accounts for, written here with numpy: the
    bin's edge and width rounded to binary32, the point at the centre of its
    2^-23 cell of the bin by one fused multiply-add, the square sum, log2 f by
    one fused multiply-add, log2 of pairwise products nb^2 Delta_a Delta_b,
    their sum, and 2 to that power (a fused multiply-add is the binary64
    result of exact binary32 operands rounded once to binary32)."""
    f32 = np.float32
    e = np.asarray(grid, dtype=np.float64)
    D, nb = e.shape[0], e.shape[1] - 1
    x64, k, _ = orc.points(grid, seed, t, first, count)
    lo = np.take_along_axis(e[:, :-1].T[None, :, :].repeat(count, 0), k[:, None, :], 1)[:, 0, :]
    delta = np.take_along_axis(np.diff(e, axis=1).T[None, :, :].repeat(count, 0),
                               k[:, None, :], 1)[:, 0, :]
    frac = (x64 - lo) / delta
    cell = np.clip(np.floor(frac * 2.0 ** 23), 0, 2 ** 23 - 1)
    y = (1.0 + cell * 2.0 ** -23).astype(f32)
    w32 = delta.astype(f32)
    e32 = (lo - w32.astype(np.float64) * (1.0 - 2.0 ** -24)).astype(f32)
    x32 = (y.astype(np.float64) * w32 + e32.astype(np.float64)).astype(f32)
    a = float(params[0])
    c32 = np.asarray(params[1:1 + D], dtype=np.float64).astype(f32)
    acc = np.zeros(count, dtype=f32)
    for d in range(D):
        z = (x32[:, d] - c32[d]).astype(f32)
        acc = (z.astype(np.float64) * z + acc).astype(f32)
    k32 = f32(np.log2(np.e) / (a * a))
    c0 = f32(-D * np.log2(a * np.sqrt(np.pi)))
    log2f = (-np.float64(k32) * acc + np.float64(c0)).astype(f32)
    l2j = np.zeros(count, dtype=f32)
    for d in range(0, D, 2):
        if d + 1 < D:
            pw = (w32[:, d] * f32(nb * nb)).astype(f32) * w32[:, d + 1]
        else:
            pw = (w32[:, d] * f32(nb)).astype(f32)
        l2j = (l2j + np.log2(pw.astype(np.float64)).astype(f32)).astype(f32)
    l2 = (l2j + log2f).astype(f32)
    fl = np.floor(l2)
    m = np.exp2((l2 - fl).astype(np.float64)).astype(f32)
    return m.astype(np.float64) * np.exp2(fl.astype(np.float64))


def test_fp32_gauss_weight_bound(orc):
    """A binary32 evaluation of the Gaussian's weights stays within
    fp32_gauss_weight_rtol of the oracle's binary64 weights at 1, 8 and 32
    dimensions (random grids, events crossing 2^32), and the bound is not
    vacuous: the same weights moved by twice it fail."""
    for dim, nb in ((1, 2), (8, 50), (32, 256)):
        rng = np.random.default_rng(dim * 1000 + nb)
        grid = W.random_grid(rng, dim, nb)
        params = [0.3] + list(rng.uniform(0.3, 0.7, dim))
        bound = T.fp32_gauss_weight_rtol(grid, params)
        n, first = 4000, 2**32 - 2000
        w64 = orc.weights(grid, W.F_GAUSS, params, 9, 1, first, n)
        w32 = _fp32_gauss_weights(orc, grid, params, 9, 1, first, n)
        rel = np.abs(w32 / w64 - 1.0)
        assert rel.max() <= bound, (dim, nb, rel.max(), bound)
        assert rel.max() > 1e-8  # the evaluation is a binary32 one
        assert not T.rel_close(w32 * (1.0 + 2.0 * bound), w64, bound)
