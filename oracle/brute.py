"""Exhaustive search over column partitions, for tiny inputs.

TEST INFRASTRUCTURE ONLY (pins the oracle's OptimizeXAxis).  For a fixed row
assignment Q, OptimizeXAxis (Appendix A item 10 of the paper; the dynamic
program of Reshef et al.'s OptimizeXAxis) claims the largest mutual
information I(P;Q) over all column partitions P with at most l columns.  This
module computes that maximum by enumerating every set of cuts -- a different
computation from the dynamic program -- so a dropped term, a wrong index or a
wrong recurrence in the oracle shows up as a mismatch.

Cuts are allowed only between consecutive points (in first-coordinate order)
whose first coordinates differ, or, when ``allowed`` is given, only at those
positions.  Mutual information is computed from the grid's joint counts as
sum_ij p_ij ln(p_ij / (p_i p_j)).
"""
from __future__ import annotations

import itertools

import numpy as np


def grid_mi(cols: np.ndarray, rows: np.ndarray) -> float:
    """I(P;Q) in nats from per-point column and row labels."""
    n = len(cols)
    _, ci = np.unique(cols, return_inverse=True)
    _, ri = np.unique(rows, return_inverse=True)
    joint = np.zeros((ci.max() + 1, ri.max() + 1))
    np.add.at(joint, (ci, ri), 1.0)
    p = joint / n
    pc = p.sum(axis=1, keepdims=True)
    pr = p.sum(axis=0, keepdims=True)
    nz = p > 0
    return float((p[nz] * np.log(p[nz] / (pc @ pr)[nz])).sum())


def best_partitions(a_sorted, q, lmax: int, allowed=None):
    """best[l] = max I(P;Q) over partitions with at most l columns, l = 1..lmax.

    a_sorted: first coordinates in ascending order; q: row of each point in
    the same order; allowed: optional set of cut positions i (a cut between
    points i-1 and i)."""
    a = np.asarray(a_sorted, dtype=np.float64)
    q = np.asarray(q)
    n = len(a)
    cand = [i for i in range(1, n) if a[i] != a[i - 1]]
    if allowed is not None:
        cand = [i for i in cand if i in allowed]
    best = {l: -np.inf for l in range(1, lmax + 1)}
    for r in range(0, min(len(cand), lmax - 1) + 1):
        for cuts in itertools.combinations(cand, r):
            cols = np.zeros(n, dtype=np.int64)
            for c in cuts:
                cols[c:] += 1
            v = grid_mi(cols, q)
            for l in range(r + 1, lmax + 1):
                if v > best[l]:
                    best[l] = v
    return best
