"""GPU path vs the FP64 oracle, through the C ABI.

Integer stages (rows, clumps, superclumps) must match bit for bit; matrix
entries and MIC/MAS/MEV must agree within 1e-6 absolute (the FP64 form is in
fact within ~1e-12); MCN must select the same cell.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _log(msg):
    print(msg, flush=True)


def _cmp_scores(got, want, tol=TOL):
    gm, wm = got["M"], want["M"]
    assert gm.shape == wm.shape
    assert np.array_equal(np.isnan(gm), np.isnan(wm))
    ok = ~np.isnan(wm)
    for key in ("M", "Axy", "Ayx"):
        d = np.abs(got[key][ok] - want[key][ok]).max()
        assert d <= tol, (key, d)
    gs, ws = got["stats"], want["stats"]
    assert np.abs(gs[:3] - ws[:3]).max() <= tol, (gs, ws)
    assert abs(gs[3] - ws[3]) < 1e-9, (gs, ws)


def test_cpp_example(micx):
    _log("case cpp_example")
    x, y = workloads.cpp_example()
    got = micx.compute_score(x, y, 0.6, 15)
    want = oracle.score(x, y, 0.6, 15)
    _cmp_scores(got, want)
    printed = (0.999999, 0.728144, 0.999999, 4.584963)
    for v, p in zip(got["stats"], printed):
        assert abs(v - p) <= 5e-7 + 1e-12


def test_sine_pair_full_matrix(micx):
    _log("case sine_pair")
    x, y = workloads.sine_pair()
    _cmp_scores(micx.compute_score(x, y, 0.6, 15), oracle.score(x, y, 0.6, 15), tol=1e-10)


@pytest.mark.parametrize("name", [c[0] for c in workloads.boundary_cases()])
def test_boundary_cases(micx, name):
    case = [c for c in workloads.boundary_cases() if c[0] == name][0]
    _, x, y, alpha = case
    _log("case boundary %s n=%d" % (name, len(x)))
    _cmp_scores(micx.compute_score(x, y, alpha, 15), oracle.score(x, y, alpha, 15), tol=1e-10)


def _integer_stage_cases():
    rng = np.random.default_rng(11)
    cases = [("sine_pair",) + workloads.sine_pair() + (0.6, 15.0)]
    a, b = workloads.fig2_points()
    cases.append(("fig2", a, b, 1.0, 15.0))
    n = 500
    x = np.floor(rng.uniform(0, 40, n))
    y = np.floor(rng.uniform(0, 25, n))
    cases.append(("ties", x, y, 0.6, 15.0))
    cases.append(("ties_c2", x, y, 0.6, 2.0))
    x = rng.uniform(0, 1, 777)
    cases.append(("sine_c5", x, np.sin(9 * x) + rng.normal(0, 0.2, 777), 0.7, 5.0))
    # 43 row counts (several items per partition wave) with c = 40: the items'
    # end counts take every remainder mod 4 for clump ends and for superclump
    # ends, the partition kernel's tails of four-at-a-time stores
    r2 = np.random.default_rng(23)
    x = r2.uniform(0, 1, 600)
    cases.append(("flat_c40", x, np.sin(6 * x) + r2.normal(0, 0.3, 600), 0.7, 40.0))
    return cases


@pytest.mark.parametrize("case", _integer_stage_cases(), ids=lambda c: c[0])
def test_integer_stages_bit_exact(micx, case):
    name, x, y, alpha, c = case
    _log("case integer stages %s" % name)
    B = oracle.grid_bound(len(x), alpha)
    tails = {0: set(), 1: set()}   # K mod 4 of items ending in clumps (0) / superclumps (1)
    for orient in (0, 1):
        for ry in range(2, B // 2 + 1):
            g = micx.debug_item(x, y, alpha, c, orient, ry)
            w = oracle.item(x, y, alpha, c, orient, ry)
            assert g["yhat"] == w["yhat"], (orient, ry)
            assert np.array_equal(g["row_starts"], w["row_starts"]), (orient, ry)
            assert g["k"] == w["k"] and g["K"] == w["K"], (orient, ry, g["k"], w["k"], g["K"], w["K"])
            assert np.array_equal(g["ends"], w["ends"]), (orient, ry)
            tails[0 if w["k"] <= int(np.floor(c * (B // ry))) else 1].add(w["K"] % 4)
    if name == "flat_c40":
        assert tails[0] == tails[1] == {0, 1, 2, 3}, tails


def test_relations_allpairs(micx):
    import torch
    _log("case relations allpairs")
    X = workloads.relations_matrix()
    got = micx.allpairs(torch.from_numpy(X).cuda(), 0.6, 15).cpu().numpy()
    want = oracle.allpairs(X.astype(np.float64), 0.6, 15)
    assert got.shape == want.shape
    assert np.abs(got[:, :3] - want[:, :3]).max() <= TOL
    assert (np.abs(got[:, 3] - want[:, 3]) < 1e-9).all()


def test_microarray_subset_allpairs(micx):
    import torch
    _log("case microarray subset")
    X, planted = workloads.microarray_matrix()
    rows = sorted(set([0, 1, 2, 3, 4, 5] + [int(planted[k, 0]) for k in range(6)] +
                      [int(planted[k, 1]) for k in range(6)]))
    Xs = X[rows]
    got = micx.allpairs(torch.from_numpy(Xs).cuda(), 0.6, 15).cpu().numpy()
    want = oracle.allpairs(Xs, 0.6, 15)
    assert np.abs(got[:, :3] - want[:, :3]).max() <= TOL
    assert (np.abs(got[:, 3] - want[:, 3]) < 1e-9).all()


@pytest.mark.parametrize("form", ["fp64", "dp32"])
def test_partition_waves_of_several_items(micx, form):
    """22 to 64 row counts: a partition wave serves up to four items (26 row
    counts at n = 800, alpha 0.6), the last wave ragged; ties, monotone and
    noisy relations among the pairs."""
    import torch
    _log("case several items per partition wave (%s)" % form)
    rng = np.random.default_rng(23)
    n, m = 800, 9
    base = rng.uniform(0.0, 1.0, n)
    X = np.stack([base,
                  np.sin(6.0 * base) + rng.normal(0.0, 0.1, n),
                  np.round(rng.uniform(0.0, 1.0, n) * 30.0) / 30.0,
                  base ** 2,
                  np.floor(rng.uniform(0.0, 6.0, n)),
                  rng.normal(0.0, 1.0, n),
                  np.abs(base - 0.5) + rng.normal(0.0, 0.05, n),
                  rng.uniform(0.0, 1.0, n),
                  np.round(base * 10.0)]).astype(np.float64)
    B = oracle.grid_bound(n, 0.6)
    assert 22 <= B // 2 - 1 <= 31, B
    assert (m * (m - 1) * (B // 2 - 1)) % 64 != 0   # the last wave is ragged
    mode = micx.MODE_DP32 if form == "dp32" else micx.MODE_FP64
    got = micx.allpairs(torch.from_numpy(X).cuda(), 0.6, 15, mode=mode).cpu().numpy()
    want = oracle.allpairs(X, 0.6, 15)
    tol = TOL
    if form == "dp32":
        bound, nfx, _ = _bound(micx)
        assert nfx > 0
        tol = min(TOL, bound + 1e-12)
    d = np.abs(got[:, :3] - want[:, :3]).max()
    assert d <= tol, (d, tol)
    assert (np.abs(got[:, 3] - want[:, 3]) < 1e-9).all()


def test_counts_int32_pairs(micx):
    import torch
    _log("case counts int32 subset")
    C = workloads.counts_matrix(m=40)
    got = micx.allpairs(torch.from_numpy(C).cuda(), 0.6, 15).cpu().numpy()
    want = oracle.allpairs(C.astype(np.float64), 0.6, 15)
    assert np.abs(got[:, :3] - want[:, :3]).max() <= TOL
    assert (np.abs(got[:, 3] - want[:, 3]) < 1e-9).all()


def test_pair_list_matches_allpairs(micx):
    import torch
    _log("case pair list")
    X = workloads.relations_matrix()[:12]
    Xd = torch.from_numpy(X).cuda()
    allp = micx.allpairs(Xd, 0.6, 15).cpu().numpy()
    m = X.shape[0]
    lst = [(i, j) for i in range(m) for j in range(i + 1, m)][::-1]
    got = micx.pairs(Xd, lst, 0.6, 15).cpu().numpy()
    idx = {p: k for k, p in enumerate([(i, j) for i in range(m) for j in range(i + 1, m)])}
    for k, p in enumerate(lst):
        assert np.array_equal(got[k], allp[idx[p]])
    # swapped order: MIC, MEV, MCN unchanged, MAS unchanged (|M - M^T| is symmetric)
    got_sw = micx.pairs(Xd, [(j, i) for (i, j) in lst], 0.6, 15).cpu().numpy()
    assert np.abs(got_sw - got).max() <= 1e-12


def test_error_paths(micx):
    _log("case error paths")
    import torch
    x = np.linspace(0, 1, 100)
    with pytest.raises(micx.MicxError) as e:
        micx.compute_score(x, x, 0.0, 15)
    assert e.value.code == micx.MICX_EINVAL
    with pytest.raises(micx.MicxError) as e:
        micx.compute_score(x[:8], x[:8], 0.6, 15)
    assert e.value.code == micx.MICX_ESMALLN
    bad = x.copy()
    bad[17] = np.nan
    with pytest.raises(micx.MicxError) as e:
        micx.compute_score(bad, x, 0.6, 15)
    assert e.value.code == micx.MICX_ENONFINITE
    big = np.zeros(micx.MAX_N + 1)
    with pytest.raises(micx.MicxError) as e:
        micx.compute_score(big, big, 0.6, 15)
    assert e.value.code == micx.MICX_ETOOBIG
    Xd = torch.zeros((3, 100), dtype=torch.float64, device="cuda")
    Xd[1, 5] = float("inf")
    out = torch.full((3, 4), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(micx.MicxError) as e:
        micx.allpairs(Xd, 0.6, 15, out=out)
    assert e.value.code == micx.MICX_ENONFINITE
    assert (out == -7.0).all(), "outputs must stay untouched on error"


# ------------------------------------------------------------------ DP32 form
def _bound(micx):
    p = micx.get_profile()
    return p["dp32_bound"], p["dp32_classes"], p["fp64_classes"]


def test_dp32_cpp_example(micx):
    _log("case dp32 cpp_example")
    x, y = workloads.cpp_example()
    got = micx.compute_score(x, y, 0.6, 15, mode=micx.MODE_DP32)
    bound, nfx, _ = _bound(micx)
    assert nfx > 0 and bound <= 5e-7
    want = oracle.score(x, y, 0.6, 15)
    _cmp_scores(got, want, tol=bound + 1e-12)
    for v, p in zip(got["stats"], (0.999999, 0.728144, 0.999999, 4.584963)):
        assert abs(v - p) <= 5e-7 + bound


def test_dp32_sine_pair_matrix_within_bound(micx):
    _log("case dp32 sine_pair")
    x, y = workloads.sine_pair()
    got = micx.compute_score(x, y, 0.6, 15, mode=micx.MODE_DP32)
    bound, nfx, _ = _bound(micx)
    assert nfx > 0
    _cmp_scores(got, oracle.score(x, y, 0.6, 15), tol=bound + 1e-12)


def test_dp32_relations_allpairs(micx):
    import torch
    _log("case dp32 relations allpairs")
    X = workloads.relations_matrix()
    got = micx.allpairs(torch.from_numpy(X).cuda(), 0.6, 15, mode=micx.MODE_DP32).cpu().numpy()
    bound, nfx, nf64 = _bound(micx)
    assert nfx > 0
    want = oracle.allpairs(X.astype(np.float64), 0.6, 15)
    d = np.abs(got[:, :3] - want[:, :3]).max()
    assert d <= min(TOL, bound + 1e-12), (d, bound)
    mism = int((np.abs(got[:, 3] - want[:, 3]) > 1e-9).sum())
    _log("dp32 relations: max|d|=%.3g bound=%.3g mcn mismatches=%d of %d" % (d, bound, mism, len(got)))
    assert mism == 0


def test_dp32_tolerance_falls_back_to_fp64(micx):
    # With a tolerance below every class bound the whole DP runs in FP64 and
    # matches the FP64 form bit for bit.
    import torch
    _log("case dp32 tolerance fallback")
    X = torch.from_numpy(workloads.relations_matrix()[:10]).cuda()
    micx.set_dp32_tolerance(1e-30)
    try:
        a = micx.allpairs(X, 0.6, 15, mode=micx.MODE_DP32).cpu().numpy()
        _, nfx, nf64 = _bound(micx)
    finally:
        micx.set_dp32_tolerance(5e-7)
    b = micx.allpairs(X, 0.6, 15, mode=micx.MODE_FP64).cpu().numpy()
    assert nfx == 0 and nf64 > 0
    assert np.array_equal(a, b)


def test_alternating_forms_full_matrices(micx):
    # Calls that alternate the two forms and the sample count reuse every
    # device buffer; each call must depend on its own inputs only.  Row
    # counts 3 and 5 with norm ln 3, ln 5 are the entries to watch.
    _log("case alternating forms")
    rng = np.random.default_rng(7)
    for n in (1000, 1023, 1024):
        x = rng.uniform(0, 1, n)
        y = np.sin(3 * x) + rng.normal(0, 0.2, n)
        want = oracle.score(x, y, 0.6, 15)
        for mode in (micx.MODE_DP32, micx.MODE_FP64, micx.MODE_DP32):
            got = micx.compute_score(x, y, 0.6, 15, mode=mode)
            tol = 1e-10 if mode == micx.MODE_FP64 else _bound(micx)[0] + 1e-12
            _cmp_scores(got, want, tol=tol)


# ------------------------------------------------------------ batch stream
def _stream_case(seed, npairs, nmin, nmax):
    data, offx, offy, ns, alphas, cs = workloads.uneven_stream(seed=seed, npairs=npairs, nmin=nmin,
                                                             nmax=nmax)
    return data, offx, offy, ns, alphas, cs


def _stream_oracle(data, offx, offy, ns, alphas, cs, rows):
    want = []
    for k in rows:
        n = int(ns[k])
        x = data[offx[k]:offx[k] + n].astype(np.float64)
        y = data[offy[k]:offy[k] + n].astype(np.float64)
        want.append(oracle.score(x, y, float(alphas[k]), float(cs[k]))["stats"])
    return np.array(want)


@pytest.mark.parametrize("seed,npairs,nmin,nmax", [(51, 96, 50, 60), (52, 40, 50, 1500)],
                         ids=["shared_n", "wide_n"])
def test_batch_stream_matches_oracle(micx, seed, npairs, nmin, nmax):
    import torch
    _log("case batch stream seed=%d npairs=%d n in [%d, %d]" % (seed, npairs, nmin, nmax))
    data, offx, offy, ns, alphas, cs = _stream_case(seed, npairs, nmin, nmax)
    got = micx.batch(torch.from_numpy(data).cuda(), offx, offy, ns, alphas, cs).cpu().numpy()
    want = _stream_oracle(data, offx, offy, ns, alphas, cs, range(npairs))
    assert np.abs(got[:, :3] - want[:, :3]).max() <= TOL
    assert (np.abs(got[:, 3] - want[:, 3]) < 1e-9).all()
    # the DP32 form stays within its stated bound
    got32 = micx.batch(torch.from_numpy(data).cuda(), offx, offy, ns, alphas, cs,
                       mode=micx.MODE_DP32).cpu().numpy()
    bound = micx.get_profile()["dp32_bound"]
    assert np.abs(got32[:, :3] - want[:, :3]).max() <= max(bound, 1e-12) + 1e-12
    assert (np.abs(got32[:, 3] - want[:, 3]) < 1e-9).all()


def test_batch_equals_single_pair_calls(micx):
    import torch
    _log("case batch vs compute_score")
    data, offx, offy, ns, alphas, cs = _stream_case(53, 12, 60, 900)
    got = micx.batch(torch.from_numpy(data).cuda(), offx, offy, ns, alphas, cs).cpu().numpy()
    for k in range(len(ns)):
        n = int(ns[k])
        x = data[offx[k]:offx[k] + n].astype(np.float64)
        y = data[offy[k]:offy[k] + n].astype(np.float64)
        one = micx.compute_score(x, y, float(alphas[k]), float(cs[k]))["stats"]
        assert np.abs(got[k] - one).max() <= 1e-12, (k, got[k], one)


def test_batch_largest_pair(micx):
    # the heaviest kind of pair in the stream: n near the maximum at alpha 0.75
    import torch
    _log("case batch largest pair n=7966 alpha=0.75")
    rng = np.random.default_rng(54)
    n = 7966
    x = rng.uniform(0, 1, n)
    y = np.sin(6 * x) + rng.normal(0, 0.3, n)
    data = np.concatenate([x, y]).astype(np.float32)
    dd = torch.from_numpy(data).cuda()
    got = micx.batch(dd, [0], [n], [n], [0.75], [15.0]).cpu().numpy()
    want = oracle.score(data[:n].astype(np.float64), data[n:].astype(np.float64), 0.75, 15)["stats"]
    assert np.abs(got[0, :3] - want[:3]).max() <= TOL, (got, want)
    assert abs(got[0, 3] - want[3]) < 1e-9
    # the DP32 form on the same pair: two-byte labels, passes of at most 24
    # layers with three targets per lane in the fixed-point descriptor kernels
    _log("case batch largest pair, dp32")
    got32 = micx.batch(dd, [0], [n], [n], [0.75], [15.0], mode=micx.MODE_DP32).cpu().numpy()
    p = micx.get_profile()
    _log("largest pair dp32: bound %.3g, %d fixed-point row counts, %d fp64, max|d| %.3g" %
         (p["dp32_bound"], p["dp32_classes"], p["fp64_classes"], np.abs(got32[0, :3] - want[:3]).max()))
    assert p["dp32_classes"] > 0
    assert np.abs(got32[0, :3] - want[:3]).max() <= 2 * p["dp32_bound"] + 1e-12, (got32, want)
    assert abs(got32[0, 3] - want[3]) < 1e-9
    # the single-pair call on the same pair in the 32-bit form: its near-tie
    # recheck reads every row's counts from LDS, so the row counts whose
    # records would not fit there beside the FP64 table run in FP64
    _log("case single-pair largest pair, dp32")
    x64, y64 = data[:n].astype(np.float64), data[n:].astype(np.float64)
    s32 = micx.compute_score(x64, y64, 0.75, 15.0, mode=micx.MODE_DP32)
    p = micx.get_profile()
    assert p["dp32_classes"] > 0 and p["fp64_classes"] > 0
    assert np.abs(s32["stats"][:3] - want[:3]).max() <= 2 * p["dp32_bound"] + 1e-12
    assert abs(s32["stats"][3] - want[3]) < 1e-9


def test_batch_errors_leave_output(micx):
    import torch
    _log("case batch errors")
    data, offx, offy, ns, alphas, cs = _stream_case(55, 6, 50, 200)
    dd = torch.from_numpy(data).cuda()
    out = torch.full((6, 4), -7.0, dtype=torch.float64, device="cuda")
    bad_n = ns.copy()
    bad_n[3] = 6                       # floor(6^alpha) < 4 for alpha <= 0.75: no grid cell
    with pytest.raises(micx.MicxError) as e:
        micx.batch(dd, offx, offy, bad_n, alphas, cs, out=out)
    assert e.value.code == micx.MICX_ESMALLN
    bad_a = alphas.copy()
    bad_a[2] = 1.5
    with pytest.raises(micx.MicxError) as e:
        micx.batch(dd, offx, offy, ns, bad_a, cs, out=out)
    assert e.value.code == micx.MICX_EINVAL
    nan_data = data.copy()
    nan_data[offy[4] + 3] = np.nan
    with pytest.raises(micx.MicxError) as e:
        micx.batch(torch.from_numpy(nan_data).cuda(), offx, offy, ns, alphas, cs, out=out)
    assert e.value.code == micx.MICX_ENONFINITE
    assert (out == -7.0).all(), "outputs must stay untouched on error"


def test_too_large_grid_is_rejected(micx):
    # alpha = 1 at n = 8192 gives B = 8192: the y = 2 item would need about
    # 8,192 superclumps of count records beside the table, more than one
    # compute unit's LDS.  The call must refuse before any work.
    import torch
    _log("case too large")
    x = np.linspace(0, 1, 8192)
    with pytest.raises(micx.MicxError) as e:
        micx.compute_score(x, x[::-1].copy(), 1.0, 15)
    assert e.value.code == micx.MICX_ETOOBIG
    out = torch.full((1, 4), -7.0, dtype=torch.float64, device="cuda")
    data = torch.from_numpy(np.concatenate([x, x]).astype(np.float32)).cuda()
    with pytest.raises(micx.MicxError) as e:
        micx.batch(data, [0], [8192], [8192], [1.0], [15.0], out=out)
    assert e.value.code == micx.MICX_ETOOBIG
    assert (out == -7.0).all()


def test_master_variable_mode(micx):
    # one variable against all others equals the matching rows of all pairs
    import torch
    _log("case master variable")
    X = workloads.relations_matrix()[:14]
    Xd = torch.from_numpy(X).cuda()
    allp = micx.allpairs(Xd, 0.6, 15).cpu().numpy()
    m = X.shape[0]
    idx = {p: k for k, p in enumerate([(a, b) for a in range(m) for b in range(a + 1, m)])}
    for i in (0, 5, m - 1):
        got = micx.master(Xd, i, 0.6, 15).cpu().numpy()
        assert got.shape == (m - 1, 4)
        for r, j in enumerate([j for j in range(m) if j != i]):
            assert np.abs(got[r] - allp[idx[(min(i, j), max(i, j))]]).max() <= 1e-12


# ----------------------------------------------------- compatibility variants
_COMPAT_CASES = [1, 2, 4, 8, 16, 32, 1 | 2 | 32, 4 | 8 | 16]


def _compat_inputs():
    rng = np.random.default_rng(61)
    n = 500
    tied = (np.floor(rng.uniform(0, 40, n)), np.floor(rng.uniform(0, 25, n)))
    # three row values: yhat stays below the requested row count (normalisation variant)
    three = (rng.uniform(0, 1, 400), np.floor(rng.uniform(0, 3, 400)))
    return [("tied", tied), ("three", three), ("cpp", workloads.cpp_example()),
            ("sine_pair", workloads.sine_pair())]


@pytest.mark.parametrize("flags", _COMPAT_CASES)
def test_compat_variants_match_oracle(micx, flags):
    _log("case compat flags=%d" % flags)
    micx.set_compat(flags)
    try:
        for name, (x, y) in _compat_inputs():
            got = micx.compute_score(x, y, 0.6, 15)
            want = oracle.score(x, y, 0.6, 15, flags=flags)
            _cmp_scores(got, want, tol=1e-10)
            if flags & (1 | 2 | 32) and name == "tied":
                B = oracle.grid_bound(len(x), 0.6) - (1 if flags & 16 else 0)
                for orient in (0, 1):
                    for ry in range(2, B // 2 + 1):
                        g = micx.debug_item(x, y, 0.6, 15, orient, ry)
                        w = oracle.item(x, y, 0.6, 15, orient, ry, flags=flags)
                        assert g["yhat"] == w["yhat"] and g["K"] == w["K"], (orient, ry)
                        assert np.array_equal(g["ends"], w["ends"]), (orient, ry)
    finally:
        micx.set_compat(0)


def test_compat_in_batch(micx):
    import torch
    _log("case compat batch")
    data, offx, offy, ns, alphas, cs = workloads.uneven_stream(seed=62, npairs=12, nmin=60, nmax=900)
    flags = 1 | 8 | 16 | 32
    micx.set_compat(flags)
    try:
        got = micx.batch(torch.from_numpy(data).cuda(), offx, offy, ns, alphas, cs).cpu().numpy()
    finally:
        micx.set_compat(0)
    for k in range(len(ns)):
        n = int(ns[k])
        w = oracle.score(data[offx[k]:offx[k] + n].astype(np.float64),
                         data[offy[k]:offy[k] + n].astype(np.float64), float(alphas[k]), float(cs[k]),
                         flags=flags)["stats"]
        assert np.abs(got[k, :3] - w[:3]).max() <= TOL and abs(got[k, 3] - w[3]) < 1e-9


def test_compat_rejects_unknown_bits(micx):
    with pytest.raises(micx.MicxError) as e:
        micx.set_compat(64)
    assert e.value.code == micx.MICX_EINVAL


# ------------------------------------------------ Pearson's rho, MIC - rho^2
def test_pearson_allpairs_matches_oracle(micx):
    import torch
    _log("case pearson allpairs relations")
    X = workloads.relations_matrix()            # float32, 64 x 400
    Xd = torch.from_numpy(X).cuda()
    stats = micx.allpairs(Xd, 0.6, 15.0)
    got = micx.pearson(Xd, stats=stats).cpu().numpy()
    st = stats.cpu().numpy()
    X64 = X.astype(np.float64)
    m = X.shape[0]
    k = 0
    for i in range(m):
        for j in range(i + 1, m):
            r = oracle.pearson(X64[i], X64[j])
            assert abs(got[k, 0] - r) <= 1e-12, (i, j, got[k, 0], r)
            assert abs(got[k, 1] - (st[k, 0] - got[k, 0] ** 2)) <= 1e-15
            k += 1
    want = oracle.allpairs(X64, 0.6, 15.0)
    idx = np.array([oracle.nonlinearity(want[q, 0], got[q, 0]) for q in range(len(want))])
    assert np.abs(got[:, 1] - idx).max() <= 1e-6


def test_pearson_pairs_constant_and_int32(micx):
    import torch
    _log("case pearson pairs, constant variable, int32")
    rng = np.random.default_rng(71)
    X = rng.integers(0, 50, (5, 333)).astype(np.int32)
    X[3] = 7                                # a constant variable
    Xd = torch.from_numpy(X).cuda()
    pl = [(0, 1), (3, 0), (2, 2), (4, 1)]
    got = micx.pearson(Xd, pl).cpu().numpy()
    for k, (i, j) in enumerate(pl):
        r = oracle.pearson(X[i].astype(np.float64), X[j].astype(np.float64))
        if np.isnan(r):
            assert np.isnan(got[k, 0])
        else:
            assert abs(got[k, 0] - r) <= 1e-12
        assert np.isnan(got[k, 1])          # no MINE records given
    assert abs(got[2, 0] - 1.0) <= 1e-15


def test_pearson_errors(micx):
    import ctypes
    import torch
    X = torch.zeros((4, 20), dtype=torch.float64, device="cuda")
    out = torch.empty((6, 2), dtype=torch.float64, device="cuda")
    lib = micx.load_library()
    ctx = micx.context(0)
    # npairs must be m(m-1)/2 without a pair list
    rc = lib.micx_pearson(ctx, ctypes.c_void_p(X.data_ptr()), 1, 4, 20, None, 5, None,
                          ctypes.c_void_p(out.data_ptr()), None)
    assert rc == micx.MICX_EINVAL
    with pytest.raises(micx.MicxError):
        micx.pearson(X, [(0, 4)])


def test_cli_end_to_end(micx, tmp_path):
    # the mine-style front end: all pairs and master mode against the oracle
    # (printed with 6 decimals)
    from paper_1208_4271_amd import cli
    _log("case cli end to end")
    rng = np.random.default_rng(72)
    x = rng.uniform(0, 1, 300)
    V = np.stack([x, np.sin(6 * x) + rng.normal(0, 0.2, 300), rng.normal(size=300), x ** 2])
    src = tmp_path / "v.csv"
    src.write_text("".join("v%d,%s\n" % (i, ",".join(repr(float(t)) for t in row)) for i, row in enumerate(V)))
    for extra, ij in (([], [(i, j) for i in range(4) for j in range(i + 1, 4)]),
                      (["-m", "2"], [(1, 0), (1, 2), (1, 3)])):
        out = tmp_path / "o.tsv"
        assert cli.main([str(src), "-a", "0.6", "-c", "15", "--fp64", "-o", str(out)] + extra) == 0
        lines = out.read_text().splitlines()
        assert lines[0] == cli.HEADER and len(lines) == 1 + len(ij)
        for line, (i, j) in zip(lines[1:], ij):
            f = line.split("\t")
            assert f[:2] == ["v%d" % i, "v%d" % j]
            w = oracle.score(V[i], V[j], 0.6, 15.0)["stats"]
            r = oracle.pearson(V[i], V[j])
            vals = np.array([float(t) for t in f[2:]])
            want = np.array([w[0], w[1], w[2], w[3], r, oracle.nonlinearity(w[0], r)])
            assert np.abs(vals - want).max() <= 1.5e-6, (i, j, vals, want)


def test_microarray_full_size_sampled(micx):
    # the benchmark workload at full size (1000 x 1340, all 499,500 pairs) in
    # both forms; pairs sampled for the oracle: the planted ones + 128 seeded
    import torch
    _log("case microarray full size, sampled pairs")
    X, planted = workloads.microarray_matrix()
    m = X.shape[0]
    rng = np.random.default_rng(91)
    pl = {(int(min(a, b)), int(max(a, b))) for a, b in planted[:, :2]}
    while len(pl) < len(planted) + 128:
        a, b = rng.integers(0, m, 2)
        if a != b:
            pl.add((int(min(a, b)), int(max(a, b))))
    pl = sorted(pl)
    idx = np.array([i * m - i * (i + 1) // 2 + (j - i - 1) for i, j in pl])
    want = oracle.allpairs(X, 0.6, 15.0, pairs=np.array(pl))
    Xd = torch.from_numpy(X).cuda()
    got64 = micx.allpairs(Xd, 0.6, 15.0, micx.MODE_FP64).cpu().numpy()[idx]
    assert np.abs(got64[:, :3] - want[:, :3]).max() <= TOL
    assert (np.abs(got64[:, 3] - want[:, 3]) < 1e-9).all()
    got32 = micx.allpairs(Xd, 0.6, 15.0, micx.MODE_DP32).cpu().numpy()[idx]
    bound = micx.get_profile()["dp32_bound"]
    assert np.abs(got32[:, :3] - want[:, :3]).max() <= max(bound, 1e-12) + 1e-12
    assert (np.abs(got32[:, 3] - want[:, 3]) < 1e-9).all()
