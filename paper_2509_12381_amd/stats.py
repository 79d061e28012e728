"""Ensemble statistics over the observable planes (host side, numpy): the
probability of complex formation and the distributions of scattering angle
and complex lifetime (Sec. 4.2: percentage of trajectories forming a complex;
Sec. 4.1: observables)."""
from __future__ import annotations

import math

import numpy as np

from . import workload as W

O = W.OBS


def complexes(obs: np.ndarray) -> np.ndarray:
    """Mask of trajectories that formed a complex (two or more bounces)."""
    return obs[O["bounces"]] >= 2


def complex_probability(obs: np.ndarray) -> float:
    n = obs.shape[1]
    return float(complexes(obs).sum()) / n if n else 0.0


def angle_histogram(obs: np.ndarray, bins: int = 64):
    """Histogram of the scattering angle over log10-spaced bins on [1e-10, pi]
    (angles below 1e-10 go to the first bin)."""
    edges = np.logspace(-10.0, math.log10(math.pi), bins + 1)
    ang = np.clip(obs[O["angle"]], edges[0], edges[-1])
    return np.histogram(ang, edges)[0], edges


def lifetime_histogram(obs: np.ndarray, tmax: float, bins: int = 64):
    """Histogram of complex lifetimes (complexes only), linear bins on [0, tmax]."""
    edges = np.linspace(0.0, tmax, bins + 1)
    return np.histogram(obs[O["lifetime"]][complexes(obs)], edges)[0], edges


def two_proportion_sigma(k1: int, n1: int, k2: int, n2: int) -> float:
    """|p1 - p2| in units of the pooled binomial standard deviation."""
    p = (k1 + k2) / (n1 + n2)
    sd = math.sqrt(max(p * (1 - p), 1e-300) * (1.0 / n1 + 1.0 / n2))
    return abs(k1 / n1 - k2 / n2) / sd if sd > 0 else 0.0


def block_relative_difference(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per trajectory, the largest of |da|/|b| over the blocks x_ion, v_ion,
    x_atom, v_atom of (12, n) final states."""
    out = np.zeros(a.shape[1])
    for blk in (slice(0, 3), slice(3, 6), slice(6, 9), slice(9, 12)):
        num = np.linalg.norm(a[blk] - b[blk], axis=0)
        den = np.linalg.norm(b[blk], axis=0)
        out = np.maximum(out, num / np.where(den > 0, den, 1.0))
    return out
