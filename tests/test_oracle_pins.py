"""Pins of the FP64 oracle to facts that do not come from the oracle itself.

- Fig. 2 of the paper: EquipartitionYAxis(D, 3) and GetClumpsPartition(D, Q)
  on 14 printed points (integer, exact).
- The paper's C++ example: printed MIC, MAS, MEV, MCN (6 decimals, +-5e-7),
  plus the closed forms MIC = MEV = H_2(500/1001)/ln 2 and MCN = log2(24).
- Exhaustive enumeration of column partitions (oracle/brute.py) for tiny n:
  OptimizeXAxis must reach the exact optimum.
- Closed forms on noiseless monotone data, invariance under strictly
  increasing transforms, exact transposition under swapping the variables,
  and the bounds 0 <= M <= 1, MEV <= MIC, MAS <= MIC, 2 <= MCN <= log2 B.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- Fig. 2 --
def test_fig2_equipartition_rows():
    rows = np.array(_read_golden("fig2_getclumps.txt"), dtype=np.float64)
    a, b, Q = rows[:, 0], rows[:, 1], rows[:, 2].astype(int)
    order = np.argsort(b, kind="stable")
    q_sorted, yhat = oracle.equipartition(b[order], 3)
    q = np.empty(len(b), dtype=int)
    q[order] = q_sorted
    assert yhat == 3
    assert (q + 1 == Q).all()


def test_fig2_clumps():
    rows = np.array(_read_golden("fig2_getclumps.txt"), dtype=np.float64)
    a, Q, P = rows[:, 0], rows[:, 2].astype(int), rows[:, 3].astype(int)
    assert (np.diff(a) >= 0).all()          # the table is printed in a-order
    p, k = oracle.clumps(a, Q - 1)
    assert k == 5
    assert (p + 1 == P).all()


def test_fig2_points_match_generator():
    rows = np.array(_read_golden("fig2_getclumps.txt"), dtype=np.float64)
    a, b = workloads.fig2_points()
    assert (rows[:, 0] == a).all() and (rows[:, 1] == b).all()


# ----------------------------------------------------------- C++ example --
def test_cpp_example_printed_values():
    x, y = workloads.cpp_example()
    st = oracle.score(x, y, 0.6, 15)["stats"]
    want = {r[0]: float(r[1]) for r in _read_golden("cpp_example.txt")}
    for i, name in enumerate(("MIC", "MAS", "MEV", "MCN")):
        assert abs(st[i] - want[name]) <= 5e-7 + 1e-12, (name, st[i], want[name])


def test_cpp_example_closed_forms():
    # The best 2-row grid is pure: I = H(Q) with rows of 500 and 501 points,
    # so MIC = MEV = H_2(500/1001) / ln 2; it needs 12 columns (the curve
    # crosses the row boundary 11 times), so MCN = log2(12 * 2).
    x, y = workloads.cpp_example()
    st = oracle.score(x, y, 0.6, 15)["stats"]
    p = 500.0 / 1001.0
    h2 = -(p * math.log(p) + (1 - p) * math.log(1 - p))
    assert abs(st[0] - h2 / math.log(2)) < 1e-12
    assert abs(st[2] - h2 / math.log(2)) < 1e-12
    assert abs(st[3] - math.log2(24)) < 1e-12


def test_cpp_example_rejects_index_combination():
    # Combining the orientations at equal (equipartitioned, optimised) index
    # instead of equal grid shape does not reproduce the printed MAS.
    x, y = workloads.cpp_example()
    st = oracle.score(x, y, 0.6, 15, flags=oracle.COMBINE_INDEX)["stats"]
    assert abs(st[1] - 0.728144) > 1e-3


# ------------------------------------------------------------ brute force --
def _tiny_dataset(rng, n, ties):
    if ties:
        x = rng.integers(0, max(2, n // 2), n).astype(np.float64)
        y = rng.integers(0, max(2, n // 2), n).astype(np.float64)
    else:
        x = rng.uniform(0, 1, n)
        y = np.sin(4 * x) + rng.normal(0, 0.3, n)
    return x, y


@pytest.mark.parametrize("seed", range(12))
def test_optimize_x_axis_reaches_exhaustive_optimum(seed):
    """For fixed rows Q, the DP's I_l equals the exhaustive maximum over all
    column partitions with at most l columns (cuts between distinct first
    coordinates).  With superclumping the enumeration is restricted to the
    superclump boundaries."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(8, 13))
    x, y = _tiny_dataset(rng, n, ties=(seed % 2 == 1))
    c = [15.0, 0.6, 1.0][seed % 3]
    alpha = 1.0
    B = oracle.grid_bound(n, alpha)
    for orient in (0, 1):
        u, v = (x, y) if orient == 0 else (y, x)
        ou, ov = np.argsort(u, kind="stable"), np.argsort(v, kind="stable")
        for ry in range(2, B // 2 + 1):
            cx = B // ry
            qv, yhat = oracle.equipartition(v[ov], ry)
            rowpt = np.empty(n, dtype=np.int32)
            rowpt[ov] = qv
            qu = rowpt[ou]
            khat = int(math.floor(c * cx))
            col, K, k = oracle.superclumps(u[ou], qu, khat)
            I, _ = oracle.optimize_x_axis(col, qu, K, yhat, cx)
            if k > khat:
                allowed = {i for i in range(1, n) if col[i] != col[i - 1]}
            else:
                allowed = None
            best = brute.best_partitions(u[ou], qu, cx, allowed)
            for l in range(2, cx + 1):
                assert abs(I[l - 2] - best[l]) < 1e-12, (orient, ry, l, I[l - 2], best[l])


@pytest.mark.parametrize("seed", range(6))
def test_score_entries_match_exhaustive_search(seed):
    """The whole-pair path: A_xy[ry][l] * ln min(l, yhat) equals the exhaustive
    optimum over column partitions of x for y's equipartition (no
    superclumping with c = 15 at these sizes)."""
    rng = np.random.default_rng(2000 + seed)
    n = 12
    x, y = _tiny_dataset(rng, n, ties=(seed % 2 == 0))
    r = oracle.score(x, y, 1.0, 15.0)
    B = r["B"]
    ov, ou = np.argsort(y, kind="stable"), np.argsort(x, kind="stable")
    for ry in range(2, B // 2 + 1):
        qv, yhat = oracle.equipartition(y[ov], ry)
        rowpt = np.empty(n, dtype=np.int32)
        rowpt[ov] = qv
        best = brute.best_partitions(x[ou], rowpt[ou], B // ry)
        for l in range(2, B // ry + 1):
            norm = min(l, yhat)
            want = best[l] / math.log(norm) if norm >= 2 else 0.0
            assert abs(r["Axy"][ry - 2, l - 2] - want) < 1e-12


# ---------------------------------------------------------- closed forms --
def test_noiseless_monotone_closed_form():
    # Strictly increasing relation, no ties, n divisible by every row count
    # used: the equipartition rows can be matched exactly by columns, so
    # M_{r,r} = 1 for every r with r^2 <= B, and MIC = 1.
    n = 240
    x = np.linspace(0.0, 1.0, n)
    y = x ** 3 + x
    r = oracle.score(x, y, 0.6, 15)
    B = r["B"]
    for k in range(2, int(math.isqrt(B)) + 1):
        assert abs(r["M"][k - 2, k - 2] - 1.0) < 1e-12
    assert abs(r["stats"][0] - 1.0) < 1e-12


def test_noiseless_odd_n_two_by_two():
    # Odd n: the best 2x2 grid splits floor(n/2) : ceil(n/2), so
    # M_{2,2} = H_2(floor(n/2)/n) / ln 2.
    n = 201
    x = np.linspace(0.0, 1.0, n)
    r = oracle.score(x, np.exp(x), 0.6, 15)
    p = (n // 2) / n
    h2 = -(p * math.log(p) + (1 - p) * math.log(1 - p))
    assert abs(r["M"][0, 0] - h2 / math.log(2)) < 1e-12


# ------------------------------------------------------------ invariances --
def _rank_transform(v):
    # strictly increasing map of the values onto 0, 1, 2, ... (ties kept)
    u, inv = np.unique(v, return_inverse=True)
    return inv.astype(np.float64)


@pytest.mark.parametrize("seed", range(3))
def test_invariance_under_increasing_transforms(seed):
    rng = np.random.default_rng(3000 + seed)
    n = 300
    x = rng.uniform(0, 1, n)
    y = np.round(np.cos(5 * x) + rng.normal(0, 0.3, n), 1)     # ties in y
    r0 = oracle.score(x, y, 0.6, 15)
    xr = _rank_transform(x)
    r1 = oracle.score(np.exp(xr / 40.0), y, 0.6, 15)
    r2 = oracle.score(x, _rank_transform(y) * 3.0 + 7.0, 0.6, 15)
    for r in (r1, r2):
        assert np.array_equal(np.nan_to_num(r0["M"], nan=-1), np.nan_to_num(r["M"], nan=-1))
        assert np.array_equal(r0["stats"], r["stats"])


@pytest.mark.parametrize("seed", range(3))
def test_swap_transposes_matrix(seed):
    rng = np.random.default_rng(4000 + seed)
    n = 250
    x = rng.uniform(0, 1, n)
    y = (x - 0.5) ** 2 + rng.normal(0, 0.05, n)
    a = oracle.score(x, y, 0.6, 15)
    b = oracle.score(y, x, 0.6, 15)
    assert np.array_equal(np.nan_to_num(a["M"], nan=-1), np.nan_to_num(b["M"].T, nan=-1))
    assert np.array_equal(a["stats"], b["stats"])


# ----------------------------------------------------------------- bounds --
@pytest.mark.parametrize("seed", range(4))
def test_bounds(seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(40, 400))
    x = rng.uniform(0, 1, n)
    y = rng.uniform(0, 1, n) if seed % 2 else np.sin(6 * x) + rng.normal(0, 0.5, n)
    r = oracle.score(x, y, 0.6, 15)
    M = r["M"][~np.isnan(r["M"])]
    mic, mas, mev, mcn = r["stats"]
    assert (M >= -1e-15).all() and (M <= 1 + 1e-12).all()
    assert mev <= mic + 1e-15 and mas <= mic + 1e-15
    assert 2.0 - 1e-12 <= mcn <= math.log2(r["B"]) + 1e-12


def test_constant_variable_scores_zero():
    x = np.linspace(0, 1, 120)
    st = oracle.score(x, np.full(120, 2.5), 0.6, 15)["stats"]
    assert st[0] == 0.0 and st[1] == 0.0 and st[2] == 0.0 and st[3] == 2.0


# ------------------------------------------- GetSuperclumpsPartition (Alg. 2) --
def superclump_goldens():
    """Hand-worked cases of Algorithm 2 (tests/golden/superclumps_alg2.txt):
    (name, khat, clump sizes, superclump ends)."""
    out = []
    for r in _read_golden("superclumps_alg2.txt"):
        out.append((r[0], int(r[1]), [int(v) for v in r[2].split(",")],
                    [int(v) for v in r[3].split(",")]))
    return out


def clump_input(sizes):
    """Points in column order (distinct first coordinates) whose row labels
    alternate 0, 1, 0, ... from one clump to the next, so that
    GetClumpsPartition returns exactly clumps of the given sizes."""
    a = np.arange(sum(sizes), dtype=np.float64)
    q = np.repeat(np.arange(len(sizes)) % 2, sizes).astype(np.int32)
    return a, q


def superclump_ends(p):
    n = len(p)
    return [i + 1 for i in range(n) if i == n - 1 or p[i + 1] != p[i]]


@pytest.mark.parametrize("case", superclump_goldens(), ids=lambda c: c[0])
def test_superclumps_hand_worked(case):
    # Algorithm 2 with Appendix A items 3 and 7: the merge is EquipartitionYAxis
    # over the points with each clump a tie group, closing rows on equality
    name, khat, sizes, ends = case
    a, q = clump_input(sizes)
    p, K, k = oracle.superclumps(a, q, khat)
    assert k == len(sizes)
    assert K == len(ends) <= khat
    assert superclump_ends(p) == ends


def test_superclump_bound_below_one_column():
    # c < 1/2 with two columns gives floor(c x) = 0: the bound is taken as one
    # superclump, so the single column carries no information and every
    # entry of such a row count is exactly 0
    x, y = workloads.sine_pair()
    c = 0.3
    B = oracle.grid_bound(len(x), 0.6)
    r = oracle.score(x, y, 0.6, c)
    seen = 0
    for orient, A in ((0, r["Axy"]), (1, r["Ayx"])):
        for ry in range(2, B // 2 + 1):
            cx = B // ry
            it = oracle.item(x, y, 0.6, c, orient, ry)
            kh = max(1, math.floor(c * cx))
            assert it["K"] <= kh
            if kh == 1:
                seen += 1
                assert it["K"] == 1 and list(it["ends"]) == [len(x)]
                assert (A[ry - 2, : cx - 1] == 0.0).all()
    assert seen > 0


def test_superclumps_respect_khat():
    x, y = workloads.sine_pair()
    B = oracle.grid_bound(len(x), 0.6)
    for orient in (0, 1):
        for ry in range(2, B // 2 + 1):
            it = oracle.item(x, y, 0.6, 15, orient, ry)
            khat = 15 * (B // ry)
            assert it["K"] <= max(it["k"] if it["k"] <= khat else khat, 1)
            assert (np.diff(it["ends"]) > 0).all() and it["ends"][-1] == len(x)
            assert it["yhat"] <= ry


def test_independent_data_mic_falls_with_n():
    # Sanity only (no exact value exists): MIC of independent uniforms falls
    # as n grows.
    rng = np.random.default_rng(6000)
    small = np.mean([oracle.score(rng.uniform(0, 1, 60), rng.uniform(0, 1, 60))["stats"][0]
                     for _ in range(20)])
    large = np.mean([oracle.score(rng.uniform(0, 1, 1500), rng.uniform(0, 1, 1500))["stats"][0]
                     for _ in range(4)])
    assert large < small


# ------------------------------------------------ Pearson's rho, MIC - rho^2
def test_pearson_worked_examples():
    # hand-computed: centred sums 4 / sqrt(5 * 5) and 1 / sqrt(2 * 2)
    assert abs(oracle.pearson([1, 2, 3, 4], [1, 3, 2, 4]) - 0.8) <= 1e-15
    assert abs(oracle.pearson([0, 1, 2], [0, 2, 1]) - 0.5) <= 1e-15


def test_pearson_closed_forms():
    rng = np.random.default_rng(41)
    x = rng.normal(size=300)
    y = rng.normal(size=300)
    assert abs(oracle.pearson(x, 3.0 * x - 7.0) - 1.0) <= 1e-14
    assert abs(oracle.pearson(x, -0.5 * x + 2.0) + 1.0) <= 1e-14
    r = oracle.pearson(x, y)
    assert oracle.pearson(y, x) == r
    assert abs(oracle.pearson(2.0 * x + 1.0, -3.0 * y + 5.0) + r) <= 1e-14
    assert np.isnan(oracle.pearson(x, np.full(300, 4.25)))


def test_nonlinearity_index():
    # noiseless linear data: MIC = 1 (even n) and rho = 1, so the index is 0;
    # a monotone non-linear relation keeps MIC = 1 with rho < 1
    x = np.arange(400, dtype=np.float64) / 400.0
    mic_lin = oracle.score(x, 2.0 * x + 1.0)["stats"][0]
    assert abs(oracle.nonlinearity(mic_lin, oracle.pearson(x, 2.0 * x + 1.0))) <= 1e-12
    y = np.exp(8.0 * x)
    mic = oracle.score(x, y)["stats"][0]
    rho = oracle.pearson(x, y)
    assert abs(mic - 1.0) <= 1e-12 and rho < 0.9
    assert abs(oracle.nonlinearity(mic, rho) - (1.0 - rho * rho)) <= 1e-15


# ------------------------------------------- count table and tie-group starts
def test_fig2_count_table():
    # App. A item 10a on Fig. 2's data: with the printed rows Q and clumps P
    # (no superclumping: khat = 15 * floor(14/3) > 5 clumps), N[t][r] counts
    # the points of clumps 1..t in row r+1
    rows = np.array(_read_golden("fig2_getclumps.txt"), dtype=np.float64)
    a, b = rows[:, 0], rows[:, 1]
    Q, P = rows[:, 2].astype(int), rows[:, 3].astype(int)
    K = P.max()
    want = np.zeros((K + 1, 3), dtype=np.int32)
    for t in range(1, K + 1):
        for r in range(3):
            want[t, r] = int(((P <= t) & (Q == r + 1)).sum())
    got = oracle.counts(a, b, 1.0, 15.0, 0, 3)
    assert np.array_equal(got, want)


def test_count_table_invariants_on_tied_data():
    # the last row holds the row sizes; each step adds exactly the points of
    # one superclump (its size from the item's ends); counts never decrease
    rng = np.random.default_rng(31)
    n = 300
    x = np.floor(rng.uniform(0, 30, n))
    y = np.floor(rng.uniform(0, 12, n))
    for orient in (0, 1):
        for ry, c in ((2, 15.0), (4, 15.0), (5, 1.0), (9, 2.0)):
            it = oracle.item(x, y, 0.6, c, orient, ry)
            N = oracle.counts(x, y, 0.6, c, orient, ry)
            assert N.shape == (it["K"] + 1, it["yhat"])
            sizes = np.diff(np.concatenate([it["row_starts"][:it["yhat"]], [n]]))
            assert np.array_equal(N[-1], sizes)
            steps = np.diff(N, axis=0)
            assert (steps >= 0).all()
            assert np.array_equal(steps.sum(axis=1), np.diff(np.concatenate([[0], it["ends"]])))


def test_group_starts_brute_force():
    rng = np.random.default_rng(32)
    for n in (1, 2, 17, 200):
        v = np.floor(rng.uniform(0, 6, n)) * 0.5
        want = np.array([int((v < v[j]).sum()) for j in range(n)], dtype=np.int32)
        assert np.array_equal(oracle.group_starts(v), want)
