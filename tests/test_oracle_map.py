"""Pins for the oracle's grid map (steps O1, O3).

The bin index is an exact integer function of the random word, checked with
Python integers; on the uniform grid the map is the identity of the point
y = (r + 1/(2 nb)) / 2^32 and the Jacobian is 1; on any grid the Jacobian is
the derivative of the map (finite differences inside a bin), the map is
monotone in r and stays inside its bin.
"""
import numpy as np

from paper_2010_09341_amd import workloads as W


def test_uniform_grid_edges(orc):
    e = orc.uniform_grid(3, 7)
    assert e.shape == (3, 8)
    assert np.array_equal(e[:, 0], np.zeros(3)) and np.array_equal(e[:, -1], np.ones(3))
    assert np.allclose(e, np.tile(np.arange(8) / 7.0, (3, 1)), rtol=0, atol=1e-16)


def test_bin_index_exact(orc):
    rng = np.random.default_rng(5)
    for nb in (2, 3, 50, 100, 512, 4096):
        e = orc.uniform_grid(1, nb)[0]
        rs = [0, 1, 2**31, 2**32 - 1] + [int(v) for v in rng.integers(0, 2**32, 300)]
        for r in rs:
            x, k, _ = orc.map_dim(nb, e, r)
            assert k == (r * nb) >> 32
            # the fraction is the centre of the remaining 2^-32 cell
            frac = (((r * nb) & 0xFFFFFFFF) + 0.5) / 2**32
            assert 0.0 < frac < 1.0
            assert e[k] <= x <= e[k + 1]


def test_uniform_grid_is_identity(orc):
    rng = np.random.default_rng(6)
    for nb in (2, 50, 100):
        e = orc.uniform_grid(1, nb)[0]
        for r in [0, 2**32 - 1] + [int(v) for v in rng.integers(0, 2**32, 500)]:
            x, k, jf = orc.map_dim(nb, e, r)
            y = (r + 0.5 / nb) / 2**32
            assert abs(x - y) <= 4e-16
            assert abs(jf - 1.0) <= nb * 2.0**-52


def test_jacobian_is_derivative_of_map(orc):
    rng = np.random.default_rng(7)
    nb = 20
    e = W.random_grid(rng, 1, nb)[0]
    step = 2**20
    for r in rng.integers(0, 2**32 - step, 200):
        r = int(r)
        x0, k0, jf = orc.map_dim(nb, e, r)
        x1, k1, _ = orc.map_dim(nb, e, r + step)
        if k0 != k1:
            continue
        dxdy = (x1 - x0) / (step / 2**32)
        assert abs(dxdy - jf) <= 1e-9 * jf
        assert abs(jf - nb * (e[k0 + 1] - e[k0])) <= 1e-15 * jf


def test_map_monotone_and_in_bin(orc):
    rng = np.random.default_rng(8)
    nb = 37
    e = W.random_grid(rng, 1, nb)[0]
    rs = np.sort(rng.integers(0, 2**32, 2000))
    xs = []
    for r in rs:
        x, k, _ = orc.map_dim(nb, e, int(r))
        assert e[k] <= x <= e[k + 1]
        xs.append(x)
    assert np.all(np.diff(xs) >= 0)


def test_points_words_per_dimension(orc):
    """Dimension d of event n uses word d%4 of Philox block d//4, counter
    (n_lo, n_hi, t, d//4), key (seed_lo, seed_hi)."""
    nb = 64
    dim = 6
    e = orc.uniform_grid(dim, nb)
    seed = (3 << 32) | 11
    for n in (0, 5, (1 << 32) + 7):
        for t in (0, 4):
            x, k, jac = orc.points(e, seed, t, n, 1)
            for d in range(dim):
                words = orc.philox4x32_10([n & 0xFFFFFFFF, n >> 32, t, d // 4], [11, 3])
                assert k[0, d] == (int(words[d % 4]) * nb) >> 32
            assert abs(jac[0] - 1.0) < 1e-13
