"""Pins for the oracle's integrands (step O4).

Each integrand is pinned by an independent route: deterministic quadrature of
the oracle's own function against a closed form (Gaussian, Breit-Wigner,
sum), structural properties (LO toy: angular factor, cut, symmetry, resonance
half-width), and the known properties of flat massless phase space (RAMBO:
momentum conservation, masslessness, isotropy, the single-particle energy
spectrum 6x(1-x) for n = 4).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2010_09341_amd import workloads as W


def test_const_and_sum(orc):
    assert orc.integrand(W.F_CONST, [0.3, 0.9]) == 1.0
    assert orc.integrand(W.F_SUM, [0.25, 0.5, 0.125]) == 0.875


@pytest.mark.parametrize("a,c", [(0.1, 0.5), (0.05, 0.3), (0.3, 0.8)])
def test_gauss_1d_quadrature(orc, a, c):
    val, err = integrate.quad(lambda x: orc.integrand(W.F_GAUSS, [x], [a, c]), 0, 1,
                              points=[c], epsabs=1e-14, epsrel=1e-12, limit=200)
    assert abs(val - W.gauss_closed_form(1, a, [c])) < 1e-10


def test_gauss_is_product_over_dimensions(orc):
    a = 0.2
    cs = [0.3, 0.6, 0.45]
    x = [0.1, 0.7, 0.5]
    f = orc.integrand(W.F_GAUSS, x, [a] + cs)
    prod = 1.0
    for xi, ci in zip(x, cs):
        prod *= orc.integrand(W.F_GAUSS, [xi], [a, ci])
    assert abs(f - prod) <= 1e-14 * prod
    # default centres are 0.5 and the default width 0.1
    assert orc.integrand(W.F_GAUSS, [0.5, 0.5]) == orc.integrand(W.F_GAUSS, [0.5, 0.5], [0.1])
    assert abs(orc.integrand(W.F_GAUSS, [0.5], [0.1]) - 1 / (0.1 * math.sqrt(math.pi))) < 1e-13


def test_gauss_2d_quadrature(orc):
    a, cs = 0.15, [0.4, 0.55]
    val, _ = integrate.dblquad(lambda y, x: orc.integrand(W.F_GAUSS, [x, y], [a] + cs),
                               0, 1, 0, 1, epsabs=1e-12, epsrel=1e-10)
    assert abs(val - W.gauss_closed_form(2, a, cs)) < 1e-9


def test_bw_flat_quadrature(orc):
    m, G = 0.42, 0.03
    val, _ = integrate.quad(lambda x: orc.integrand(W.F_BW_FLAT, [x, 0.3], [m, G]), 0, 1,
                            points=[m], epsabs=1e-13, epsrel=1e-12, limit=400)
    assert abs(val - W.bw_flat_closed_form(m, G)) < 1e-10
    # flat in the other dimensions
    assert orc.integrand(W.F_BW_FLAT, [0.4, 0.1], [m, G]) == orc.integrand(
        W.F_BW_FLAT, [0.4, 0.9], [m, G])


def test_sum_2d_quadrature(orc):
    val, _ = integrate.dblquad(lambda y, x: orc.integrand(W.F_SUM, [x, y]), 0, 1, 0, 1)
    assert abs(val - 1.0) < 1e-12


LO = [13000.0, 91.19, 2.5, 20.0]


def _lo(orc, x1, x2, u3, u4):
    return orc.integrand(W.F_LO_TOY, [x1, x2, u3, u4], LO)


def test_lo_angular_factor(orc):
    """Integrating over cos(theta) and phi multiplies the c = 0 slice by 4/3
    (int (1+c^2) dc = 8/3 over [-1,1], dc = 2 du, dphi = 2 pi du)."""
    x1, x2 = 0.02, 0.003
    mid = _lo(orc, x1, x2, 0.5, 0.0)
    val, _ = integrate.dblquad(lambda u4, u3: _lo(orc, x1, x2, u3, u4), 0, 1, 0, 1,
                               epsabs=0, epsrel=1e-12)
    assert abs(val / mid - 4.0 / 3.0) < 1e-10
    assert _lo(orc, x1, x2, 0.3, 0.1) == _lo(orc, x1, x2, 0.3, 0.8)
    # c -> -c symmetry (2u - 1 rounds differently for u and 1 - u)
    assert _lo(orc, x1, x2, 0.2, 0.5) == pytest.approx(_lo(orc, x1, x2, 0.8, 0.5), rel=1e-15)


def test_lo_cut_symmetry_and_resonance(orc):
    s = 13000.0 ** 2
    x2 = 0.5
    # cut at sqrt(s_hat) = 20
    x1_cut = 400.0 / (x2 * s)
    assert _lo(orc, x1_cut * (1 - 1e-9), x2, 0.5, 0.0) == 0.0
    assert _lo(orc, x1_cut * (1 + 1e-9), x2, 0.5, 0.0) > 0.0
    assert _lo(orc, 0.3, 0.01, 0.5, 0.0) == _lo(orc, 0.01, 0.3, 0.5, 0.0)
    # Breit-Wigner half maximum at s_hat = m^2 +- m G. g(x) = x^-1/2 (1-x)^3 is the
    # configured parton density; divide it and 1/s_hat out.
    m, G = 91.19, 2.5

    def core(shat):
        x1 = shat / (x2 * s)
        g = x1 ** -0.5 * (1 - x1) ** 3
        return _lo(orc, x1, x2, 0.5, 0.0) * shat / g

    peak = core(m * m)
    assert abs(core(m * m + m * G) / peak - 0.5) < 1e-12
    assert abs(core(m * m - m * G) / peak - 0.5) < 1e-12
    # the peak value itself: g(x2) (m G/pi)/(m G)^2 * 4 pi
    g2 = x2 ** -0.5 * (1 - x2) ** 3
    assert abs(peak - g2 * (1 / (math.pi * m * G)) * 4 * math.pi) < 1e-12 * peak


def test_lo_total_by_quadrature(orc):
    """The 4-D oracle Vegas run of the LO toy against 2-D quadrature of the
    configured formula with the two angles integrated analytically."""
    s = 13000.0 ** 2
    m, G = 91.19, 2.5

    def f2(x2, x1):
        shat = x1 * x2 * s
        if shat <= 400.0:
            return 0.0
        g = lambda x: x ** -0.5 * (1 - x) ** 3
        bw = (m * G / math.pi) / ((shat - m * m) ** 2 + (m * G) ** 2)
        return g(x1) * g(x2) * bw / shat

    # integrate in (log tau, log x1) where tau = x1 x2 with breakpoints at the peak
    tau0 = m * m / s

    def in_tau(lt, lx1):
        tau = math.exp(lt)
        x1 = math.exp(lx1)
        x2 = tau / x1
        if x2 >= 1.0:
            return 0.0
        return f2(x2, x1) * tau  # dx1 dx2 = dtau dx1 / x1 = tau x1 dlt dlx1 / x1

    lo_t = math.log(400.0 / s)
    pts = [math.log(tau0 * (1 + k * G / m)) for k in (-8, -2, -1, 0, 1, 2, 8)]
    edges = [lo_t] + pts + [0.0]
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        v, _ = integrate.dblquad(lambda lx1, lt: in_tau(lt, lx1), a, b,
                                 lambda lt: lt, lambda lt: 0.0, epsabs=0, epsrel=1e-9)
        total += v
    expect = total * (8.0 / 3.0) * 2 * math.pi
    I_t, s_t, _, bad = orc.run(4, 100, W.F_LO_TOY, LO, 200_000, seed=3, n_iter=6, alpha=1.5)
    I, sig, _ = orc.combine(I_t[1:], s_t[1:])
    assert bad == 0
    assert abs(I - expect) < 4 * sig, (I, sig, expect)
    assert sig < 0.05 * expect


RSQRT = 1000.0


def _rambo_events(orc, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        p, Wt = orc.rambo4(RSQRT, rng.uniform(size=16))
        out.append(p)
    return np.array(out), Wt


def test_rambo_conservation_and_mass(orc):
    P, Wt = _rambo_events(orc, 2000, 1)
    tot = P.sum(axis=1)
    assert np.allclose(tot[:, 0], RSQRT, rtol=0, atol=1e-9)
    assert np.allclose(tot[:, 1:], 0.0, rtol=0, atol=1e-9)
    m2 = P[..., 0] ** 2 - (P[..., 1:] ** 2).sum(-1)
    assert np.max(np.abs(m2)) < 1e-12 * RSQRT ** 2 * 10
    assert np.all(P[..., 0] > 0)
    assert abs(Wt - math.pi ** 3 * RSQRT ** 4 / 96) < 1e-3


def test_rambo_flat_phase_space(orc):
    """n = 4 massless flat phase space: x = 2E/sqrt(s) has density 6x(1-x);
    directions are isotropic."""
    P, _ = _rambo_events(orc, 40000, 2)
    x = 2 * P[:, 0, 0] / RSQRT
    ks = stats.kstest(x, lambda v: 3 * v ** 2 - 2 * v ** 3)
    assert ks.pvalue > 1e-4
    cos = P[:, :, 3] / P[:, :, 0]
    ks2 = stats.kstest(cos.ravel(), "uniform", args=(-1, 2))
    assert ks2.pvalue > 1e-4


def test_rambo_integrand_modes(orc):
    rng = np.random.default_rng(4)
    s = RSQRT ** 2
    n_zero = 0
    for _ in range(3000):
        u = rng.uniform(size=16)
        p, Wt = orc.rambo4(RSQRT, u)
        f0 = orc.integrand(W.F_RAMBO24, u, [RSQRT, 0.01, 0.0])
        f1 = orc.integrand(W.F_RAMBO24, u, [RSQRT, 0.01, 1.0])
        assert f1 == Wt
        sij = [2 * (p[i, 0] * p[j, 0] - p[i, 1:] @ p[j, 1:]) for i, j in
               ((0, 1), (1, 2), (2, 3), (3, 0))]
        if min(sij) <= 0.01 * s:
            assert f0 == 0.0
            n_zero += 1
        else:
            assert abs(f0 - Wt / np.prod(sij)) <= 1e-12 * f0
    assert 0 < n_zero < 3000


# ---------------------------------------------------------------------------
# The RAMBO cut integrand against a second, independently written flat
# phase-space generator: sequential two-body decays. Flat massless 4-body phase
# space (no (2 pi) factors, the convention of the RAMBO weight) factorises as
#   R_4(s) = int dM3^2 dM2^2 R_2(s; M3, 0) R_2(M3^2; M2, 0) R_2(M2^2; 0, 0),
# with R_2(s; m, 0) = (pi/2)(s - m^2)/s and isotropic decays in each rest frame:
# P -> p4 + Q3, Q3 -> p3 + Q2, Q2 -> p1 + p2. Sampling M3^2 = s u0 and
# M2^2 = M3^2 u1 gives the event weight (pi/2)^3 s^2 u0 (1 - u0)(1 - u1), whose
# mean is the volume pi^3 s^2 / 96. Nothing here calls the oracle's RAMBO.
# ---------------------------------------------------------------------------
def _iso(u1, u2, k):
    ct = 2.0 * u1 - 1.0
    st = np.sqrt(1.0 - ct * ct)
    ph = 2.0 * math.pi * u2
    return np.stack([k, k * st * np.cos(ph), k * st * np.sin(ph), k * ct], -1)


def _to_lab(p, Q, M):
    """p given in the rest frame of Q (lab four-momentum Q, mass M)."""
    qp = (Q[:, 1:] * p[:, 1:]).sum(-1)
    out = np.empty_like(p)
    out[:, 0] = (Q[:, 0] * p[:, 0] + qp) / M
    out[:, 1:] = p[:, 1:] + Q[:, 1:] * (qp / (M * (Q[:, 0] + M)) + p[:, 0] / M)[:, None]
    return out


def _sequential_decays(rng, n, sqrt_s):
    s = sqrt_s ** 2
    u = rng.uniform(size=(n, 8))
    M3sq = s * u[:, 0]
    M2sq = M3sq * u[:, 1]
    M3, M2 = np.sqrt(M3sq), np.sqrt(M2sq)
    weight = (math.pi / 2) ** 3 * s * s * u[:, 0] * (1.0 - u[:, 0]) * (1.0 - u[:, 1])
    k4 = (s - M3sq) / (2.0 * sqrt_s)
    p4 = _iso(u[:, 2], u[:, 3], k4)
    Q3 = np.stack([sqrt_s - k4, -p4[:, 1], -p4[:, 2], -p4[:, 3]], -1)
    k3 = (M3sq - M2sq) / (2.0 * M3)
    p3r = _iso(u[:, 4], u[:, 5], k3)
    Q2r = np.stack([M3 - k3, -p3r[:, 1], -p3r[:, 2], -p3r[:, 3]], -1)
    p3, Q2 = _to_lab(p3r, Q3, M3), _to_lab(Q2r, Q3, M3)
    k1 = M2 / 2.0
    p1r = _iso(u[:, 6], u[:, 7], k1)
    p2r = np.stack([k1, -p1r[:, 1], -p1r[:, 2], -p1r[:, 3]], -1)
    return np.stack([_to_lab(p1r, Q2, M2), _to_lab(p2r, Q2, M2), p3, p4], 1), weight


def test_sequential_decay_generator():
    """The test's own generator: momentum conservation, masslessness, and the
    phase-space volume pi^3 s^2 / 96."""
    P, weight = _sequential_decays(np.random.default_rng(5), 400_000, RSQRT)
    tot = P.sum(axis=1)
    assert np.allclose(tot[:, 0], RSQRT, rtol=0, atol=1e-9)
    assert np.allclose(tot[:, 1:], 0.0, rtol=0, atol=1e-9)
    m2 = P[..., 0] ** 2 - (P[..., 1:] ** 2).sum(-1)
    assert np.max(np.abs(m2)) < 1e-12 * RSQRT ** 2 * 10
    vol = math.pi ** 3 * RSQRT ** 4 / 96
    se = weight.std() / math.sqrt(len(weight))
    assert abs(weight.mean() - vol) < 4 * se


def test_rambo_cut_integrand_against_sequential_decays(orc):
    """The RAMBO24 integrand of the configured workload (mode 0: the phase-space
    weight times the product of 1/s_ij over the cyclic neighbours, zero unless
    every one of those s_ij exceeds 0.01 s), integrated by the oracle with
    plain Monte Carlo on the uniform grid (one iteration, 1e6 events), equals
    the same physics integral from the sequential-decay generator within 4
    combined standard deviations (each about 0.3-0.4 % of the value). The flat
    measure is symmetric in the four momenta, so any labelling of the decay
    products gives the same integral."""
    n = 1_000_000
    s = RSQRT ** 2
    P, weight = _sequential_decays(np.random.default_rng(11), n, RSQRT)
    prod = np.ones(n)
    keep = np.ones(n, dtype=bool)
    for i, j in ((0, 1), (1, 2), (2, 3), (3, 0)):
        sij = 2.0 * (P[:, i, 0] * P[:, j, 0] - (P[:, i, 1:] * P[:, j, 1:]).sum(-1))
        keep &= sij > 0.01 * s
        prod *= sij
    f = np.where(keep, weight / prod, 0.0)
    I_seq, e_seq = f.mean(), f.std() / math.sqrt(n)
    e = orc.uniform_grid(16, 50)
    I_o, s_o, _, bad = orc.iterate(e, W.F_RAMBO24, [RSQRT, 0.01, 0.0], n, seed=3, t=0)
    assert bad == 0
    assert e_seq < 0.01 * I_seq and s_o < 0.01 * I_o
    assert abs(I_o - I_seq) < 4 * math.hypot(e_seq, s_o), (I_o, I_seq, e_seq, s_o)
