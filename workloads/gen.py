"""Seeded synthetic workloads.

Every generator uses ``numpy.random.default_rng(seed)``.  The shapes, value
distributions and dependence structure follow the paper's workloads: a
transcriptomics-sized matrix (n = 1340 samples, as in its Table 1 microarray
set, Sec. "Transcriptomic datasets"), RNA-seq-like integer counts with many
zeros, a mix of functional relationships, and its C++ usage example.  The
paper's datasets themselves are not available; these inputs stand in for them.
"""
from __future__ import annotations

import numpy as np

# Relationship types applied to a base column (the mixed-relations matrix and the uneven stream).
RELATIONS = ("linear", "parabola", "cubic", "exponential", "sine1", "sine8", "circle", "step")


def _relation(kind: str, u: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """A noiseless function of u in [0, 1], scaled to roughly [0, 1]."""
    if kind == "linear":
        f = u
    elif kind == "parabola":
        f = 4.0 * (u - 0.5) ** 2
    elif kind == "cubic":
        f = 4.0 * (u - 0.5) ** 3 + 0.5 * (u - 0.5) + 0.5
        f = (f - f.min()) / max(f.max() - f.min(), 1e-12)
    elif kind == "exponential":
        f = (np.exp(10.0 * u) - 1.0) / (np.exp(10.0) - 1.0)
    elif kind == "sine1":
        f = 0.5 + 0.5 * np.sin(2.0 * np.pi * u)
    elif kind == "sine8":
        f = 0.5 + 0.5 * np.sin(16.0 * np.pi * u)
    elif kind == "circle":
        sign = rng.choice(np.array([-1.0, 1.0]), size=u.shape)
        f = 0.5 + 0.5 * sign * np.sqrt(np.clip(1.0 - (2.0 * u - 1.0) ** 2, 0.0, 1.0))
    elif kind == "step":
        f = np.floor(4.0 * np.clip(u, 0.0, 1.0 - 1e-12)) / 3.0
    else:
        raise ValueError(kind)
    return f


def sine_pair(seed: int = 1, n: int = 200):
    """Single pair, float64: x ~ U[0,1], y = sin(4 pi x) + N(0, 0.1^2)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, n)
    y = np.sin(4.0 * np.pi * x) + rng.normal(0.0, 0.1, n)
    return x.astype(np.float64), y.astype(np.float64)


def relations_matrix(seed: int = 2, m: int = 64, n: int = 400) -> np.ndarray:
    """m x n float32: 16 uniform base columns, 32 noisy functions of them
    (8 relation types x 4 noise levels sigma in {0, 1/3, 2/3, 1}), 16 N(0,1)
    columns.  Row-major, one variable per row."""
    rng = np.random.default_rng(seed)
    X = np.empty((m, n), dtype=np.float64)
    nb = 16
    X[:nb] = rng.uniform(0.0, 1.0, (nb, n))
    sigmas = (0.0, 1.0 / 3.0, 2.0 / 3.0, 1.0)
    col = nb
    for t, kind in enumerate(RELATIONS):
        for k, s in enumerate(sigmas):
            if col >= m:
                break
            base = X[(col - nb) % nb]
            X[col] = _relation(kind, base, rng) + (rng.normal(0.0, s, n) if s > 0 else 0.0)
            col += 1
    while col < m:
        X[col] = rng.normal(0.0, 1.0, n)
        col += 1
    return X.astype(np.float32)


def microarray_matrix(seed: int = 3, m: int = 1000, n: int = 1340, planted: int = 50):
    """Microarray-shaped m x n float64: exp(N(6, 1.5^2)) rounded to 2 decimals
    (ties), with `planted` disjoint dependent pairs (i, j): column j is a noisy
    function of standardised log column i.  Returns (X, planted_list) where
    planted_list rows are (i, j, relation index, sigma)."""
    rng = np.random.default_rng(seed)
    X = np.round(np.exp(rng.normal(6.0, 1.5, (m, n))), 2)
    idx = rng.permutation(m)[: 2 * planted].reshape(planted, 2)
    plist = []
    for p, (i, j) in enumerate(idx):
        z = np.log(X[i])
        z = (z - z.mean()) / max(z.std(), 1e-12)
        kind = p % len(RELATIONS)
        u = (z - z.min()) / max(z.max() - z.min(), 1e-12)
        g = _relation(RELATIONS[kind], u, rng)
        g = (g - g.mean()) / max(g.std(), 1e-12)
        s = rng.uniform(0.0, 0.5)
        X[j] = np.round(np.exp(6.0 + 1.5 * g + rng.normal(0.0, s, n) if s > 0 else 6.0 + 1.5 * g), 2)
        plist.append((int(i), int(j), kind, float(s)))
    return X.astype(np.float64), np.array(plist, dtype=np.float64)


def counts_matrix(seed: int = 4, m: int = 2000, n: int = 1340) -> np.ndarray:
    """RNA-seq-shaped m x n int32 counts: per feature a mean mu log-uniform in
    [0.5, 5000], negative binomial with dispersion 0.2 (size 5), then
    structural zeros with probability pi ~ U[0.3, 0.6] per feature."""
    rng = np.random.default_rng(seed)
    mu = np.exp(rng.uniform(np.log(0.5), np.log(5000.0), m))
    size = 1.0 / 0.2
    p = size / (size + mu)
    C = rng.negative_binomial(size, p[:, None], (m, n))
    pi = rng.uniform(0.3, 0.6, m)
    zero = rng.uniform(0.0, 1.0, (m, n)) < pi[:, None]
    C[zero] = 0
    return C.astype(np.int32)


def uneven_stream(seed: int = 5, npairs: int = 8192, nmin: int = 50, nmax: int = 8000):
    """Uneven stream of independent pairs.  Returns (data float32 packed,
    offsets_x, offsets_y, ns, alphas, cs).  n is log-uniform in [nmin, nmax];
    the relation is one of the 8 types or independent, with noise sigma ~ U[0,1];
    alpha in {0.55, 0.6, 0.75} and c in {5, 15} drawn per pair."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), npairs))).astype(np.int64)
    alphas = rng.choice(np.array([0.55, 0.6, 0.75]), npairs)
    cs = rng.choice(np.array([5.0, 15.0]), npairs)
    total = int(2 * ns.sum())
    data = np.empty(total, dtype=np.float32)
    offx = np.empty(npairs, dtype=np.int64)
    offy = np.empty(npairs, dtype=np.int64)
    pos = 0
    for p in range(npairs):
        n = int(ns[p])
        x = rng.uniform(0.0, 1.0, n)
        kind = int(rng.integers(0, len(RELATIONS) + 1))
        s = rng.uniform(0.0, 1.0)
        if kind == len(RELATIONS):
            y = rng.uniform(0.0, 1.0, n)
        else:
            y = _relation(RELATIONS[kind], x, rng) + rng.normal(0.0, s, n)
        offx[p] = pos
        data[pos:pos + n] = x
        pos += n
        offy[p] = pos
        data[pos:pos + n] = y
        pos += n
    return data, offx, offy, ns, alphas, cs


def cpp_example():
    """The paper's C++ usage example input: n = 1001, x_i = i/1000,
    y_i = sin(10 * PI * x_i) + x_i with PI = 3.14159265 as the example sets it."""
    n = 1001
    PI = 3.14159265
    x = np.array([i / (n - 1) for i in range(n)], dtype=np.float64)
    y = np.sin(10.0 * PI * x) + x
    return x, y


def fig2_points():
    """The 14 points of the paper's Fig. 2 (GetClumpsPartition example)."""
    pts = [(1, 1), (1, 2), (1, 3), (1, 4), (2, 3), (2, 4), (3, 5), (4, 6), (5, 6), (6, 6),
           (7, 5), (8, 3), (9, 2), (9, 1)]
    a = np.array([p[0] for p in pts], dtype=np.float64)
    b = np.array([p[1] for p in pts], dtype=np.float64)
    return a, b


def boundary_cases(seed: int = 7):
    """Edge inputs: sample sizes where floor(n^alpha) sits on a power
    (n = 11, 243, 1024, 3125, 7776 at alpha 0.6; 81, 256, 4096 at 0.75), a
    constant column, an all-ties column and a two-valued column.  Returns a
    list of (name, x, y, alpha)."""
    rng = np.random.default_rng(seed)
    cases = []
    for n in (11, 243, 1024, 3125, 7776):
        x = rng.uniform(0, 1, n)
        cases.append(("n%d_a0.6" % n, x, np.sin(3 * x) + rng.normal(0, 0.2, n), 0.6))
    for n in (81, 256, 4096):
        x = rng.uniform(0, 1, n)
        cases.append(("n%d_a0.75" % n, x, x ** 2 + rng.normal(0, 0.2, n), 0.75))
    n = 300
    x = rng.uniform(0, 1, n)
    cases.append(("const_y", x, np.full(n, 3.0), 0.6))
    cases.append(("ties_both", np.floor(rng.uniform(0, 5, n)), np.floor(rng.uniform(0, 3, n)), 0.6))
    cases.append(("two_valued", x, (x > 0.5).astype(np.float64), 0.6))
    return cases
