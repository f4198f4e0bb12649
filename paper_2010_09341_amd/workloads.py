"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload descriptions and random input generators only; it
contains none of the method's arithmetic (no Philox, no grid map, no
integrand, no refinement). Both the HIP path and the CPU oracle consume what
it produces.

Workloads. The paper measures a single-top leading-order integration with
PDF sets (Fig. 2) and an unnamed integral on a cluster (Table 1); neither is
available, so the synthetic integrands below stand in for them: normalised
Gaussians (closed-form integral), an LO-style 2->2 toy with a Breit-Wigner
resonance and a parton-density-like factor, and massless 2->4 RAMBO phase
space with pair-invariant cuts. The serving trace is a Poisson stream of mixed
integrals.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Integrand identifiers: the same values as the VEGAS_F_* constants of the
# C interface.
F_CONST, F_SUM, F_GAUSS, F_LO_TOY, F_RAMBO24, F_BW_FLAT = range(6)
FP64, FP32_EVAL = 0, 1


@dataclass
class Workload:
    name: str
    dim: int
    nb: int
    fid: int
    params: list
    n_events: int
    n_iter: int
    alpha: float = 1.5
    seed: int = 0
    precs: tuple = (FP64,)
    note: str = ""


#: The small 4-D Gaussian parity case, the 8-D Gaussian throughput case, the
#: LO toy and RAMBO 2->4 (the first four entries of the benchmark's config
#: list, in order).
WORKLOADS = {
    "gauss4d": Workload("gauss4d", 4, 50, F_GAUSS, [0.1], 100_000, 5, precs=(FP64,),
                        note="4-D normalised Gaussian, a=0.1, 50 bins, 5 x 1e5 events"),
    "gauss8d": Workload("gauss8d", 8, 50, F_GAUSS, [0.1], 10_000_000, 10,
                        precs=(FP64, FP32_EVAL),
                        note="8-D normalised Gaussian, a=0.1, 50 bins, 10 x 1e7 events"),
    "lo_toy": Workload("lo_toy", 4, 100, F_LO_TOY, [13000.0, 91.19, 2.5, 20.0],
                       100_000_000, 10, precs=(FP32_EVAL,),
                       note="LO 2->2 toy, sqrt(s)=13 TeV, BW(91.19, 2.5), 100 bins, 10 x 1e8"),
    "rambo24": Workload("rambo24", 16, 50, F_RAMBO24, [1000.0, 0.01, 0.0], 50_000_000, 10,
                        precs=(FP32_EVAL,),
                        note="massless 2->4 RAMBO at sqrt(s)=1000, cyclic 1/s_ij, "
                             "s_ij > 0.01 s, 50 bins, 10 x 5e7"),
}


def gauss_closed_form(dim, a, centres=None):
    """Integral over [0,1]^D of the normalised Gaussian product."""
    c = [0.5] * dim if centres is None else list(centres)
    out = 1.0
    for ci in c:
        out *= 0.5 * (math.erf((1.0 - ci) / a) + math.erf(ci / a))
    return out


def bw_flat_closed_form(m, G):
    """Integral over [0,1] of the unit-normalised Cauchy density of width G."""
    h = G / 2.0
    return (math.atan((1.0 - m) / h) + math.atan(m / h)) / math.pi


def random_grid(rng: np.random.Generator, dim: int, nb: int, spread: float = 3.0):
    """Random strictly increasing edges with e_0 = 0 and e_nb = 1 ([dim][nb+1])."""
    w = rng.uniform(1.0, spread, size=(dim, nb))
    c = np.cumsum(w, axis=1)
    e = np.zeros((dim, nb + 1))
    e[:, 1:] = c / c[:, -1:]
    e[:, -1] = 1.0
    return e


def random_hist(rng: np.random.Generator, dim: int, nb: int, zeros: float = 0.0):
    """Random non-negative histogram [dim][nb]; a fraction `zeros` of bins is empty."""
    h = rng.lognormal(mean=0.0, sigma=2.0, size=(dim, nb))
    if zeros > 0:
        h[rng.uniform(size=h.shape) < zeros] = 0.0
    return h


def random_philox_inputs(rng: np.random.Generator, n: int):
    """Random (counter[4], key[2]) pairs plus the all-zero and all-one corners."""
    c = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    k = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    c[0], k[0] = 0, 0
    c[1], k[1] = 0xFFFFFFFF, 0xFFFFFFFF
    return c, k


@dataclass
class Request:
    """One integral of the serving stream."""
    index: int
    arrival_s: float
    dim: int
    nb: int
    fid: int
    params: list
    n_events: int
    n_iter: int
    alpha: float = 1.5
    seed: int = 0
    prec: int = FP32_EVAL
    extra: dict = field(default_factory=dict)


def serving_trace(n_requests=1000, rate_per_s=200.0, seed=0, prec=FP32_EVAL,
                  max_events=10_000_000):
    """The serving stream: Poisson arrivals; dims uniform in 2..12; a Gaussian
    (width uniform in 0.05..0.3, centres uniform in 0.2..0.8) or a 1-D
    Breit-Wigner (mass uniform in 0.3..0.7, width uniform in 0.01..0.05) times
    flat, chosen with equal probability; bins uniform in 20..100; events per
    iteration log-uniform in 1e4..1e7; 5..10 iterations; request seed =
    request index."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        dim = int(rng.integers(2, 13))
        nb = int(rng.integers(20, 101))
        if rng.uniform() < 0.5:
            a = float(rng.uniform(0.05, 0.3))
            centres = [float(v) for v in rng.uniform(0.2, 0.8, size=dim)]
            fid, params = F_GAUSS, [a] + centres
        else:
            fid = F_BW_FLAT
            params = [float(rng.uniform(0.3, 0.7)), float(rng.uniform(0.01, 0.05))]
        n_events = int(round(10 ** rng.uniform(4.0, 7.0)))
        n_events = max(2, min(n_events, max_events))
        n_iter = int(rng.integers(5, 11))
        out.append(Request(i, t, dim, nb, fid, params, n_events, n_iter, 1.5, i, prec))
    return out


def request_closed_form(r: Request):
    if r.fid == F_GAUSS:
        return gauss_closed_form(r.dim, r.params[0], r.params[1:])
    if r.fid == F_BW_FLAT:
        return bw_flat_closed_form(r.params[0], r.params[1])
    raise ValueError("no closed form for this integrand")
