"""Normalized band-gap objective.

Paper: Methods, "Topology optimization formulation", Eq. (10):
f = 2 (min_k lambda_{t+1} - max_k lambda_t) / (min_k lambda_{t+1} + max_k lambda_t).
Every gap the paper reports is a frequency ratio (band edges in kHz), so
the default variable here is omega; ``on="lambda"`` evaluates Eq. (10) as
printed (reading Q9).  Bands are numbered from 1 in ascending order.
The KS form replaces max/min by the Kreisselmeier-Steinhauser aggregate
KS_beta(x) = x_max + ln(sum exp(beta (x - x_max))) / beta.
"""
from __future__ import annotations

import numpy as np


def gap(omega: np.ndarray, t: int, on: str = "omega") -> float:
    x = omega ** 2 if on == "lambda" else omega
    hi = x[:, t].min()        # band t+1
    lo = x[:, t - 1].max()    # band t
    return 2.0 * (hi - lo) / (hi + lo)


def gap_weights(omega: np.ndarray, t: int):
    """d f / d omega (nk, nb) for the omega-form of Eq. (10) (arg-min/arg-max unique)."""
    hi_k = int(np.argmin(omega[:, t]))
    lo_k = int(np.argmax(omega[:, t - 1]))
    a, b = omega[hi_k, t], omega[lo_k, t - 1]
    w = np.zeros_like(omega)
    w[hi_k, t] += 4.0 * b / (a + b) ** 2
    w[lo_k, t - 1] += -4.0 * a / (a + b) ** 2
    return w


def ks_max(x: np.ndarray, beta: float) -> float:
    m = np.max(x)
    return float(m + np.log(np.sum(np.exp(beta * (x - m)))) / beta)


def ks_weights(x: np.ndarray, beta: float) -> np.ndarray:
    m = np.max(x)
    e = np.exp(beta * (x - m))
    return e / e.sum()


def ks_gap(omega: np.ndarray, t: int, beta: float, scale: float) -> float:
    """Eq. (10) with max/min replaced by KS aggregates on omega / scale."""
    hi = -ks_max(-omega[:, t] / scale, beta) * scale
    lo = ks_max(omega[:, t - 1] / scale, beta) * scale
    return 2.0 * (hi - lo) / (hi + lo)


def ks_gap_weights(omega: np.ndarray, t: int, beta: float, scale: float) -> np.ndarray:
    hi = -ks_max(-omega[:, t] / scale, beta) * scale
    lo = ks_max(omega[:, t - 1] / scale, beta) * scale
    dfa = 4.0 * lo / (hi + lo) ** 2
    dfb = -4.0 * hi / (hi + lo) ** 2
    w = np.zeros_like(omega)
    w[:, t] = dfa * ks_weights(-omega[:, t] / scale, beta)
    w[:, t - 1] = dfb * ks_weights(omega[:, t - 1] / scale, beta)
    return w
