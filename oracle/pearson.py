"""Pearson's correlation coefficient and the non-linearity index, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's engine reports both beside the four MINE statistics (Sec. 2,
Fig. 1; the supplement's Performance experiment 2A times the six together and
its Microbiome tables list them) without defining them.  They are taken here
as the textbook definitions: rho = sum (x - mean x)(y - mean y) / sqrt(sum
(x - mean x)^2 sum (y - mean y)^2), two passes in FP64 (means first), and the
MINE non-linearity index MIC - rho^2.
"""
from __future__ import annotations

import math

import numpy as np


def pearson(x, y) -> float:
    """rho of two samples of equal length n >= 2; NaN when either is constant."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape != y.shape or x.ndim != 1 or len(x) < 2:
        raise ValueError("pearson: two 1-D samples of equal length >= 2")
    dx = x - x.sum() / len(x)
    dy = y - y.sum() / len(y)
    sxx, syy = float((dx * dx).sum()), float((dy * dy).sum())
    if sxx == 0.0 or syy == 0.0:
        return float("nan")
    r = float((dx * dy).sum()) / math.sqrt(sxx * syy)
    return min(1.0, max(-1.0, r))


def nonlinearity(mic: float, rho: float) -> float:
    """The non-linearity index MIC - rho^2 (NaN when rho is NaN)."""
    return float(mic) - float(rho) * float(rho)
