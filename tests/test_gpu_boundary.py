"""The C ABI's boundary behaviour on the GPU: the debug readback of ranks and
the DP's own count table (bit-exact against the oracle), asynchronous calls
with their device-side status, replay of captured launch graphs, and MCN
with eps > 0 against its definition (App. A item 2)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _table_cases():
    rng = np.random.default_rng(41)
    cases = [("sine_pair",) + workloads.sine_pair() + (0.6, 15.0, (2, 3, 7, 12))]
    a, b = workloads.fig2_points()
    cases.append(("fig2", a, b, 1.0, 15.0, (2, 3, 7)))
    n = 500
    x = np.floor(rng.uniform(0, 40, n))
    y = np.floor(rng.uniform(0, 25, n))
    cases.append(("ties", x, y, 0.6, 15.0, (2, 5, 9, 20)))
    cases.append(("ties_c2", x, y, 0.6, 2.0, (2, 3, 10)))
    C = workloads.counts_matrix(m=6)
    cases.append(("counts", C[0].astype(np.float64), C[1].astype(np.float64), 0.6, 15.0, (2, 4, 30, 37)))
    u = rng.uniform(0, 1, 4300)
    cases.append(("labels16", u, np.sin(5 * u) + rng.normal(0, 0.3, 4300), 0.75, 5.0, (2, 100, 257, 265)))
    return cases


@pytest.mark.parametrize("case", _table_cases(), ids=lambda c: c[0])
def test_debug_tables_bit_exact(micx, case):
    # tie-group starts of both variables and the count table the DP kernel
    # builds in LDS (item 10a), against the oracle's plain definitions
    name, x, y, alpha, c, rys = case
    _log("case debug tables %s" % name)
    gx, gy = oracle.group_starts(x), oracle.group_starts(y)
    for orient in (0, 1):
        for ry in rys:
            got = micx.debug_tables(x, y, alpha, c, orient, ry)
            assert np.array_equal(got["group_start_x"], gx)
            assert np.array_equal(got["group_start_y"], gy)
            want = oracle.counts(x, y, alpha, c, orient, ry)
            assert got["counts"].shape == want.shape, (orient, ry)
            assert np.array_equal(got["counts"], want), (orient, ry)


def test_async_allpairs_and_status(micx):
    import torch
    _log("case async allpairs")
    X = workloads.relations_matrix()[:20]
    Xd = torch.from_numpy(X).cuda()
    out = micx.allpairs(Xd, 0.6, 15.0, wait=False)
    assert micx.status() == micx.MICX_OK
    want = oracle.allpairs(X.astype(np.float64), 0.6, 15.0)
    got = out.cpu().numpy()
    assert np.abs(got[:, :3] - want[:, :3]).max() <= 1e-10
    assert np.abs(got[:, 3] - want[:, 3]).max() < 1e-9
    # a NaN: the call itself returns normally; the status says so and the
    # output stays untouched
    bad = X.copy()
    bad[3, 7] = np.nan
    out2 = torch.full((190, 4), -7.0, dtype=torch.float64, device="cuda")
    micx.allpairs(torch.from_numpy(bad).cuda(), 0.6, 15.0, out=out2, wait=False)
    assert micx.status() == micx.MICX_ENONFINITE
    assert (out2 == -7.0).all()
    # batch stream: the same contract
    data, offx, offy, ns, alphas, cs = workloads.uneven_stream(seed=43, npairs=5, nmin=60, nmax=300)
    data[offy[2] + 1] = np.inf
    out3 = torch.full((5, 4), -7.0, dtype=torch.float64, device="cuda")
    micx.batch(torch.from_numpy(data).cuda(), offx, offy, ns, alphas, cs, out=out3, wait=False)
    assert micx.status() == micx.MICX_ENONFINITE
    assert (out3 == -7.0).all()
    # the profile reports the batch call's own host time (it returned before
    # the device finished); pair calls report none
    h = micx.get_profile()["host_ms"]
    assert 0.0 < h < 60e3
    micx.allpairs(Xd, 0.6, 15.0)
    assert micx.get_profile()["host_ms"] == 0.0
    # a replayed graph reports the profile of its captured call, not of the
    # calls in between
    o4 = torch.empty((190, 4), dtype=torch.float64, device="cuda")
    micx.allpairs(Xd, 0.6, 15.0, out=o4)   # first call with these arguments (eager)
    micx.allpairs(Xd, 0.6, 15.0, out=o4)   # captured
    p_cap = micx.get_profile()
    micx.batch(torch.from_numpy(data).cuda(), [offx[0]], [offy[0]], [ns[0]], [0.6], [15.0])
    assert micx.get_profile()["host_ms"] > 0.0
    micx.allpairs(Xd, 0.6, 15.0, out=o4)   # replayed
    assert micx.get_profile() == p_cap


@pytest.mark.parametrize("mode_name", ["fp64", "dp32"])
def test_graph_replay_matches_eager(micx, mode_name):
    # first call eager, second captured, later ones replayed: every result
    # equal to the eager one, and a replay reads the input's current values
    import torch
    mode = micx.MODE_FP64 if mode_name == "fp64" else micx.MODE_DP32
    _log("case graph replay %s" % mode_name)
    X = workloads.relations_matrix()[:24]
    Y = workloads.relations_matrix()[24:48].copy()
    Xd = torch.from_numpy(X.copy()).cuda()
    out = torch.empty((276, 4), dtype=torch.float64, device="cuda")
    micx.set_graphs(False)
    ref = micx.allpairs(Xd, 0.6, 15.0, mode, out=out).cpu().numpy()
    Xd.copy_(torch.from_numpy(Y))
    refY = micx.allpairs(Xd, 0.6, 15.0, mode, out=out).cpu().numpy()
    micx.set_graphs(True)
    try:
        Xd.copy_(torch.from_numpy(X))
        for k in range(4):
            out.fill_(-1.0)
            got = micx.allpairs(Xd, 0.6, 15.0, mode, out=out).cpu().numpy()
            assert np.array_equal(got, ref), k
        # same pointer, new contents: the replayed graph reads them
        Xd.copy_(torch.from_numpy(Y))
        for k in range(2):
            got = micx.allpairs(Xd, 0.6, 15.0, mode, out=out).cpu().numpy()
            assert np.array_equal(got, refY), k
    finally:
        micx.set_graphs(True)
    want = oracle.allpairs(Y.astype(np.float64), 0.6, 15.0)
    assert np.abs(refY[:, :3] - want[:, :3]).max() <= 1e-6
    assert np.abs(refY[:, 3] - want[:, 3]).max() < 1e-9


def test_mcn_with_eps_follows_its_definition(micx):
    # App. A item 2: MCN(eps) = min log2(xy) over cells with M >= (1 - eps) MIC,
    # computed here from the oracle's matrix and compared with micx_mcn on the
    # returned score
    _log("case mcn eps")
    rng = np.random.default_rng(44)
    for x, y in (workloads.sine_pair(), workloads.cpp_example(),
                 (rng.uniform(0, 1, 600), rng.uniform(0, 1, 600))):
        eps = (0.0, 0.01, 0.05, 0.2, 0.5)
        got = micx.compute_score(x, y, 0.6, 15.0, mcn_eps=eps)
        want = oracle.score(x, y, 0.6, 15.0)
        M = want["M"]
        W = M.shape[0]
        mic = np.nanmax(M)
        for e in eps:
            best = np.inf
            for yy in range(2, W + 2):
                for xx in range(2, W + 2):
                    if xx * yy <= want["B"] and M[yy - 2, xx - 2] >= (1.0 - e) * mic - 1e-12:
                        best = min(best, np.log2(xx * yy))
            assert abs(got["mcn"][e] - best) < 1e-9, (e, got["mcn"][e], best)
        assert got["mcn"][0.0] == got["stats"][3]


def test_autotune_keeps_results_bit_identical(micx, tmp_path):
    # every launch shape the tuner may pick gives the same bits (it checks
    # this itself per row count); the tuned table must leave the results of
    # both forms unchanged, also after a save/load round trip
    import torch
    _log("case autotune")
    X = workloads.relations_matrix()
    Xd = torch.from_numpy(X).cuda()
    micx.tune_clear()
    try:
        ref64 = micx.allpairs(Xd, 0.6, 15.0, micx.MODE_FP64).cpu().numpy()
        ref32 = micx.allpairs(Xd, 0.6, 15.0, micx.MODE_DP32).cpu().numpy()
        path = str(tmp_path / "tune.txt")
        micx.autotune(Xd, 0.6, 15.0, micx.MODE_DP32)
        micx.autotune(Xd, 0.6, 15.0, micx.MODE_FP64, cache_path=path)
        lines = open(path).read().splitlines()
        assert lines[0] == "micx-tune 1 gfx950" and len(lines) > 10
        assert np.array_equal(micx.allpairs(Xd, 0.6, 15.0, micx.MODE_FP64).cpu().numpy(), ref64)
        assert np.array_equal(micx.allpairs(Xd, 0.6, 15.0, micx.MODE_DP32).cpu().numpy(), ref32)
        micx.tune_clear()
        micx.tune_load(path)
        assert np.array_equal(micx.allpairs(Xd, 0.6, 15.0, micx.MODE_DP32).cpu().numpy(), ref32)
    finally:
        micx.tune_clear()
