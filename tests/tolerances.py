"""Comparison bounds of the FP64 parity tests, each derived from the arithmetic.

The FP64 path must match the oracle within EPS = 1e-12 relative. That bound is
applied directly to the quantities that are sums or products of per-event
values (per-event weights, I = S1/N, histogram bins: sums of non-negative
terms). Quantities that are ill-conditioned functions of such sums get the bound
that an EPS-relative error of their inputs propagates to:

- sigma (sigma^2 = (S2/N - I^2)/(N-1)): with I and S2/N each within EPS,
  |d sigma|/sigma <= EPS (3 + v)/(2 v), v = (S2/N - I^2)/I^2 = (N-1) sigma^2/I^2
  (the cancellation of S2/N against I^2, worst when the weights vary little);
- a refined edge (new edge j in old bin k: e_k + (j delta - C_k)/r_k Delta_k,
  delta = C_nb/nb): with every compressed weight r_i and running sum C_i
  within EPS, |d e_j| <= EPS (|e_j| + 2 (j delta + C_k) Delta_k / r_k) (the
  subtraction j delta - C_k and the division by a small r_k amplify);
- a per-event weight w = f(x) J: the GPU's point and the oracle's point each
  lie within two roundings of the exact point (the oracle forms e_k + frac
  Delta_k, the GPU one fma of the remainder with Delta_k 2^-32 onto
  e_k + 2^-33 Delta_k), so they differ by at most 4 u |x_d| per coordinate
  (u = 2^-53), and J is the same product of the same factors in the same
  order; the weights then differ by at most EPS (the integrand's own
  evaluation) plus 4 u kappa(x), kappa = sum_d |x_d d ln f / d x_d| the
  integrand's relative condition number at the point (large where f falls
  steeply to zero, such as the LO toy's (1 - x)^3 factor at x near 1);
- the inverse-variance combination I = sum(I_t/sigma_t^2)/sum(1/sigma_t^2):
  |dI| <= max_t |dI_t| + max_t(2 |d sigma_t|/sigma_t) max_t |I_t - I|, and
  |d sigma|/sigma <= max_t |d sigma_t|/sigma_t.

The numpy re-statement of smoothing and compression below serves only to size
the refined-edge bound; the reference edges themselves come from the oracle.
"""
from __future__ import annotations

import numpy as np

EPS = 1e-12
# Smallest normal binary64 number: below it a result carries an absolute
# rounding error of 2^-1075, so the bound there is EPS times this value.
TINY = 2.2250738585072014e-308


def sigma_rtol(I: float, sigma: float, n: int, eps: float = EPS) -> float:
    """Relative bound on sigma for an iteration of n events with estimate I."""
    if sigma == 0.0 or I == 0.0:
        return eps
    v = (n - 1) * sigma * sigma / (I * I)
    return eps * max(1.0, (3.0 + v) / (2.0 * v))


def sigma_close(s, s_ref, I_ref, n, eps: float = EPS) -> bool:
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    s_ref = np.atleast_1d(np.asarray(s_ref, dtype=np.float64))
    I_ref = np.broadcast_to(np.asarray(I_ref, dtype=np.float64), s_ref.shape)
    tol = np.array([sigma_rtol(i, v, n, eps) for i, v in zip(I_ref, s_ref)])
    return bool(np.all(np.abs(s - s_ref) <= tol * np.abs(s_ref)))


def sigma_excess(s, s_ref, I_ref, n, eps: float = EPS) -> float:
    """Largest |s - s_ref| / bound (<= 1 passes), for messages."""
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    s_ref = np.atleast_1d(np.asarray(s_ref, dtype=np.float64))
    I_ref = np.broadcast_to(np.asarray(I_ref, dtype=np.float64), s_ref.shape)
    tol = np.array([sigma_rtol(i, v, n, eps) for i, v in zip(I_ref, s_ref)])
    return float(np.max(np.abs(s - s_ref) / (tol * np.abs(s_ref) + 1e-300)))


def rel_close(a, b, eps: float = EPS) -> bool:
    """|a - b| <= eps |b| elementwise (b the reference); zeros must match."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return bool(np.all(np.abs(a - b) <= eps * np.abs(b)))


def max_rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.abs(a - b)
    return float(np.max(np.where(d == 0, 0.0, d / np.maximum(np.abs(b), TINY))))


U = 2.0 ** -53  # unit roundoff of binary64


def weights_rtol(kappa=None, eps: float = EPS):
    """Relative bound on a per-event weight whose integrand has relative
    condition number kappa at the event's point (see the module docstring)."""
    if kappa is None:
        return eps
    return eps + 4.0 * U * np.asarray(kappa, dtype=np.float64)


def weights_close(w, w_ref, kappa=None, eps: float = EPS) -> bool:
    """Per-event weights: EPS (plus 4 u kappa where the integrand's condition
    number kappa is given) relative for every weight in the normal binary64
    range, that times TINY absolute below it (zeros must be zeros)."""
    w = np.asarray(w, dtype=np.float64)
    w_ref = np.asarray(w_ref, dtype=np.float64)
    tol = weights_rtol(kappa, eps) * np.maximum(np.abs(w_ref), TINY)
    return bool(np.all(np.abs(w - w_ref) <= tol))


def weights_excess(w, w_ref, kappa=None, eps: float = EPS) -> float:
    """Largest |w - w_ref| / bound (<= 1 passes), for messages."""
    w = np.asarray(w, dtype=np.float64)
    w_ref = np.asarray(w_ref, dtype=np.float64)
    tol = weights_rtol(kappa, eps) * np.maximum(np.abs(w_ref), TINY)
    return float(np.max(np.abs(w - w_ref) / tol))


U32 = 2.0 ** -24  # unit roundoff of binary32


def fp32_gauss_weight_rtol(edges, params) -> float:
    """Relative bound on the FP32-eval Gaussian's per-event weight against the
    binary64 weight of the same event, over every point of the grid `edges`
    (params = [a, c_1 .. c_D]). The FP32-eval path forms log2 w = log2 f +
    log2 J in binary32 and exponentiates it in binary64, so the weight's
    relative error is ln 2 times the absolute error of that sum:
    - the binary32 point x_d and centre c_d are each within 3 units of
      binary32 roundoff u of the exact ones (the bin's lower edge and width
      rounded, the fraction kept to 23 bits), so |dz_d| <= 6u, z_d = x_d - c_d;
    - acc = sum z_d^2: |d acc| <= sum 2 |z_d| 6u + (D + 1) u acc;
    - log2 f = -k acc + c0 (k = log2 e / a^2, c0 = -D log2(a sqrt pi), both
      rounded): |d log2 f| <= k |d acc| + 2u k acc + 2u |c0| + u |log2 f|;
    - log2 J = sum over pairs of dimensions of log2((nb Delta_a)(nb Delta_b)):
      each product within 5u relative (the widths and nb Delta rounded, the
      product rounded), so its log2 within 5u/ln 2 + 2^-21 (the hardware
      log2), then D/2 additions each within u |log2 J|;
    - the sum log2 f + log2 J rounded once more (u |log2 f| + u |log2 J|), and
      2 to the power of its fraction taken by the hardware exp2 (2^-22
      relative).
    Maxima over the unit cube bound |z_d|, acc and |log2 f|; the grid's
    narrowest and widest bins bound |log2 J|."""
    e = np.asarray(edges, dtype=np.float64)
    D, nb = e.shape[0], e.shape[1] - 1
    a = float(params[0])
    c = np.asarray(params[1:1 + D], dtype=np.float64)
    if c.size < D:
        c = np.full(D, 0.5)
    zmax = np.maximum(np.abs(c), np.abs(1.0 - c))
    acc = float(np.sum(zmax * zmax))
    k = np.log2(np.e) / (a * a)
    c0 = abs(D * np.log2(a * np.sqrt(np.pi)))
    u = U32
    d_acc = 12.0 * u * float(np.sum(zmax)) + (D + 1) * u * acc
    log2f = k * acc + c0
    d_log2f = k * d_acc + 2 * u * k * acc + 2 * u * c0 + 2 * u * log2f
    log2_nbd = np.abs(np.log2(nb * np.diff(e, axis=1)))
    log2J = float(np.sum(np.max(log2_nbd, axis=1)))
    pairs = (D + 1) // 2
    d_log2J = pairs * (5 * u / np.log(2.0) + 2.0 ** -21) + (pairs + 1) * u * log2J
    return float(np.log(2.0) * (d_log2f + d_log2J) + 2.0 ** -22)


def event_kappa(orc, edges, fid, params, seed, t, first, count, h: float = 1e-7):
    """kappa(x) = sum_d |x_d d ln f / d x_d| of the oracle's integrand at the
    points of events first .. first+count-1, by central differences of
    relative step h (0 where f = 0). A point within h of a cut reads a large
    kappa, which only loosens the bound for that event."""
    x, _, _ = orc.points(edges, seed, t, first, count)
    kap = np.zeros(count)
    for i in range(count):
        f0 = orc.integrand(fid, x[i], params)
        if f0 == 0.0 or not np.isfinite(f0):
            continue
        s = 0.0
        for d in range(x.shape[1]):
            xp = x[i].copy()
            xm = x[i].copy()
            xp[d] *= 1.0 + h
            xm[d] *= 1.0 - h
            s += abs((orc.integrand(fid, xp, params) - orc.integrand(fid, xm, params))
                     / (2.0 * h * f0))
        kap[i] = s
    return kap


def _refine_terms(edges, hist, alpha):
    """Per dimension: (r, C) of the re-binning, or None for a dimension whose
    smoothed histogram sums to zero (its edges are kept)."""
    out = []
    for h in np.asarray(hist, dtype=np.float64):
        nb = len(h)
        s = np.empty(nb)
        s[0] = (h[0] + h[1]) / 2
        s[-1] = (h[-2] + h[-1]) / 2
        s[1:-1] = (h[:-2] + h[1:-1] + h[2:]) / 3
        S = s.sum()
        if not S > 0:
            out.append(None)
            continue
        p = s / S
        r = np.zeros(nb)
        mid = (p > 0) & (p < 1)
        r[mid] = ((1 - p[mid]) / (-np.log(p[mid]))) ** alpha
        r[p >= 1] = 1.0
        C = np.concatenate([[0.0], np.cumsum(r)])
        out.append((r, C))
    return out


def edges_tol(edges, hist, alpha, e_ref, eps: float = EPS):
    """Per-edge absolute bound on refined edges (see the module docstring)."""
    edges = np.asarray(edges, dtype=np.float64)
    e_ref = np.asarray(e_ref, dtype=np.float64)
    tol = eps * np.abs(e_ref)
    for d, terms in enumerate(_refine_terms(edges, hist, alpha)):
        if terms is None:
            continue
        r, C = terms
        nb = len(r)
        delta = C[-1] / nb
        width = np.diff(edges[d])
        for j in range(1, nb):
            target = j * delta
            k = int(np.searchsorted(C[1:], target, side="left"))
            k = min(k, nb - 1)
            # either neighbour may be the oracle's bin at a near-tie
            amp = 0.0
            for kk in (k - 1, k, k + 1):
                if 0 <= kk < nb and r[kk] > 0:
                    amp = max(amp, 2.0 * (target + C[kk]) * width[kk] / r[kk])
            tol[d, j] += eps * amp
    return tol


def edges_close(got, e_ref, edges, hist, alpha, eps: float = EPS) -> bool:
    got = np.asarray(got, dtype=np.float64)
    return bool(np.all(np.abs(got - e_ref) <= edges_tol(edges, hist, alpha, e_ref, eps)))


def edges_excess(got, e_ref, edges, hist, alpha, eps: float = EPS) -> float:
    got = np.asarray(got, dtype=np.float64)
    tol = edges_tol(edges, hist, alpha, e_ref, eps)
    return float(np.max(np.abs(got - e_ref) / (tol + 1e-300)))


def combine_close(I, s, I_t, s_t, I_ref, s_ref, n, eps: float = EPS) -> bool:
    """The combination of iterations matched to EPS (I_t) and their sigma
    bounds (s_t), compared with the oracle's combination (I_ref, s_ref)."""
    I_t = np.asarray(I_t, dtype=np.float64)
    s_t = np.asarray(s_t, dtype=np.float64)
    srel = max(sigma_rtol(i, v, n, eps) for i, v in zip(I_t, s_t))
    dI = eps * np.max(np.abs(I_t)) + 2 * srel * np.max(np.abs(I_t - I_ref))
    return abs(I - I_ref) <= dI and abs(s - s_ref) <= srel * abs(s_ref)


def oracle_run_steps(orc, dim, nb, fid, params, n, seed, n_iter, alpha, grid=None, t0=0):
    """The oracle's run taken step by step (iterate, refine), returning the
    per-iteration results, the final grid, and the grid and histogram the last
    refinement started from (what the refined-edge bound needs)."""
    e = orc.uniform_grid(dim, nb) if grid is None else np.asarray(grid, dtype=np.float64)
    I_t, s_t = [], []
    e_prev, h_last = e, None
    for i in range(n_iter):
        I, s, h, bad = orc.iterate(e, fid, params, n, seed, t0 + i)
        I_t.append(I)
        s_t.append(s)
        if i + 1 < n_iter:
            e_prev, h_last = e, h
            e = orc.refine(e, h, alpha)
    return np.array(I_t), np.array(s_t), e, e_prev, h_last
