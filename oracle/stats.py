"""ORACLE (test infrastructure): statistics of a growth vector, written from
their definitions. Only ``tests/`` may import this module.

The growth gamma(0..D) is read as a distribution of the distance d over the
reached states, p(d) = gamma(d) / sum(gamma) (paper, section "Table of
results: hundreds of new conjectures on Cayley graphs": mean, mode,
variance, skewness, kurtosis, and a Gaussian or Gumbel shape for the growth).

* moments are computed exactly with ``fractions.Fraction`` and converted to
  float at the end (population moments; kurtosis is the excess kurtosis);
* the fitted shapes match the first two moments (Gaussian: mean and
  standard deviation; Gumbel of the maximum when the skewness is >= 0, of
  the minimum otherwise, scale sd * sqrt(6) / pi, location mean -/+ Euler's
  gamma times the scale);
* a fit's distance is the total variation between p and the model's mass
  on the unit cells [d - 1/2, d + 1/2), counting the model's mass outside
  the cells of 0..D as mismatch.

Pinned in tests/test_stats_cpu.py by the closed forms of the Mahonian
(adjacent transpositions) and Stirling (all transpositions) growths, by
scipy's skew/kurtosis on the expanded sample and by scipy's distribution
functions.
"""

from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, Sequence

EULER_GAMMA = 0.5772156649015329


def _trim(sizes: Sequence[int]):
    s = [int(x) for x in sizes]
    while s and s[-1] == 0:
        s.pop()
    if not s:
        raise ValueError("growth has no reached state")
    return s


def moments(sizes: Sequence[int]) -> Dict[str, float]:
    s = _trim(sizes)
    total = sum(s)
    mean = Fraction(sum(d * g for d, g in enumerate(s)), total)
    m = [sum(Fraction(g, total) * (d - mean) ** k for d, g in enumerate(s)) for k in (2, 3, 4)]
    m2, m3, m4 = m
    var = float(m2)
    skew = float(m3) / var ** 1.5 if m2 else 0.0
    kurt = float(m4 / (m2 * m2)) - 3.0 if m2 else 0.0
    mode = max(range(len(s)), key=lambda d: (s[d], -d))
    return {"total": total, "diameter": len(s) - 1, "mode": mode, "max_layer": s[mode], "antipodes": s[-1],
            "mean": float(mean), "variance": var, "skewness": skew, "kurtosis": kurt}


def normal_cdf(x: float, mu: float, sigma: float) -> float:
    return 0.5 * (1.0 + math.erf((x - mu) / (sigma * math.sqrt(2.0))))


def gumbel_cdf(x: float, mu: float, beta: float, minimum: bool) -> float:
    z = (x - mu) / beta
    return 1.0 - math.exp(-math.exp(z)) if minimum else math.exp(-math.exp(-z))


def total_variation(sizes: Sequence[int], cdf) -> float:
    s = _trim(sizes)
    total = sum(s)
    tv = cdf(-0.5) + (1.0 - cdf(len(s) - 0.5))
    for d, g in enumerate(s):
        tv += abs(g / total - (cdf(d + 0.5) - cdf(d - 0.5)))
    return tv / 2.0


def growth_stats(sizes: Sequence[int]) -> Dict[str, float]:
    out = moments(sizes)
    sd = math.sqrt(out["variance"])
    minimum = out["skewness"] < 0
    beta = sd * math.sqrt(6.0) / math.pi
    mu_g = out["mean"] + EULER_GAMMA * beta if minimum else out["mean"] - EULER_GAMMA * beta
    out.update(gauss_mu=out["mean"], gauss_sigma=sd, gumbel_mu=mu_g, gumbel_beta=beta, gumbel_min=minimum)
    if sd > 0:
        out["gauss_tv"] = total_variation(sizes, lambda x: normal_cdf(x, out["mean"], sd))
        out["gumbel_tv"] = total_variation(sizes, lambda x: gumbel_cdf(x, mu_g, beta, minimum))
    else:
        out["gauss_tv"] = out["gumbel_tv"] = 1.0
    out["best_fit"] = "gumbel" if out["gumbel_tv"] < out["gauss_tv"] else "gaussian"
    return out
