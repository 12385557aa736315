"""GPU path vs the FP64 oracle on configurations with their own code paths.

- 16-bit row labels: floor(B/2) > 256 row counts (n = 4300 at alpha 0.75
  gives B = 531) store two bytes per label in the partition kernel and read
  them back in the DP's count table;
- the RNA-seq-shaped counts matrix at full size (2000 x 1340 int32, 30-60%
  zeros per feature): heavy ties shrink the clumps, superclumps and yhat;
- the DP32 form on the heaviest kind of stream item (n near 8000 at alpha
  0.75) is covered beside the FP64 form in test_gpu_parity.py.

Integer stages are compared bit for bit, scores within 1e-6 (FP64 form:
1e-10), and MCN must select the same cell in both forms.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _log(msg):
    print(msg, flush=True)


def _cmp_full(got, want, tol):
    ok = ~np.isnan(want["M"])
    assert np.array_equal(np.isnan(got["M"]), np.isnan(want["M"]))
    for key in ("M", "Axy", "Ayx"):
        d = np.abs(got[key][ok] - want[key][ok]).max()
        assert d <= tol, (key, d)
    assert np.abs(got["stats"][:3] - want["stats"][:3]).max() <= tol, (got["stats"], want["stats"])
    assert got["stats"][3] == want["stats"][3] or abs(got["stats"][3] - want["stats"][3]) < 1e-9, \
        (got["stats"], want["stats"])


def _sixteen_bit_pair():
    rng = np.random.default_rng(81)
    n = 4300
    x = rng.uniform(0, 1, n)
    y = np.sin(5 * x) + rng.normal(0, 0.3, n)
    return x, y


def test_sixteen_bit_labels_single_pair(micx):
    # n = 4300 at alpha 0.75: B = 531, row counts y = 2..265, so labels take
    # two bytes (k_part<true>, the DP's 16-bit label scans)
    x, y = _sixteen_bit_pair()
    B = oracle.grid_bound(len(x), 0.75)
    assert B // 2 > 256
    _log("case 16-bit labels n=%d alpha=0.75 B=%d" % (len(x), B))
    want = oracle.score(x, y, 0.75, 15.0)
    _cmp_full(micx.compute_score(x, y, 0.75, 15.0, mode=micx.MODE_FP64), want, 1e-10)
    # the row counts with thousands of superclumps ran cooperatively (one item
    # per workgroup) in both forms
    assert micx.get_profile()["coop_classes"] > 0
    got32 = micx.compute_score(x, y, 0.75, 15.0, mode=micx.MODE_DP32)
    p = micx.get_profile()
    assert p["coop_classes"] > 0
    _log("16-bit labels dp32: bound %.3g, %d fixed-point row counts, %d fp64" %
         (p["dp32_bound"], p["dp32_classes"], p["fp64_classes"]))
    assert p["dp32_classes"] > 0
    _cmp_full(got32, want, p["dp32_bound"] + 1e-12)


def test_sixteen_bit_labels_integer_stages(micx):
    x, y = _sixteen_bit_pair()
    _log("case 16-bit labels integer stages")
    for orient in (0, 1):
        for ry in (2, 3, 200, 255, 256, 257, 265):
            g = micx.debug_item(x, y, 0.75, 15.0, orient, ry)
            w = oracle.item(x, y, 0.75, 15.0, orient, ry)
            assert g["yhat"] == w["yhat"], (orient, ry)
            assert np.array_equal(g["row_starts"], w["row_starts"]), (orient, ry)
            assert g["k"] == w["k"] and g["K"] == w["K"], (orient, ry)
            assert np.array_equal(g["ends"], w["ends"]), (orient, ry)


def test_sixteen_bit_labels_allpairs(micx):
    # the all-pairs launch path with two-byte labels, both forms (c = 5 keeps
    # the oracle's share of the test short)
    import torch
    rng = np.random.default_rng(82)
    n = 4300
    u = rng.uniform(0, 1, n)
    X = np.stack([u, u ** 2 + rng.normal(0, 0.1, n), rng.normal(0, 1, n),
                  np.floor(8 * u) + rng.normal(0, 0.05, n)])
    _log("case 16-bit labels allpairs m=4 n=%d" % n)
    want = oracle.allpairs(X, 0.75, 5.0)
    Xd = torch.from_numpy(X).cuda()
    got = micx.allpairs(Xd, 0.75, 5.0, micx.MODE_FP64).cpu().numpy()
    assert np.abs(got[:, :3] - want[:, :3]).max() <= 1e-10
    assert np.array_equal(got[:, 3], want[:, 3]) or np.abs(got[:, 3] - want[:, 3]).max() < 1e-9
    got32 = micx.allpairs(Xd, 0.75, 5.0, micx.MODE_DP32).cpu().numpy()
    bound = micx.get_profile()["dp32_bound"]
    assert np.abs(got32[:, :3] - want[:, :3]).max() <= 2 * bound + 1e-12
    assert np.abs(got32[:, 3] - want[:, 3]).max() < 1e-9


def _zero_heavy_pairs(C, k):
    zf = (C == 0).mean(axis=1)
    order = np.argsort(-zf, kind="stable")
    return [(int(min(order[2 * i], order[2 * i + 1])), int(max(order[2 * i], order[2 * i + 1])))
            for i in range(k)], zf


def test_counts_full_size_sampled(micx):
    # the RNA-seq-shaped workload at full size: 2000 x 1340 int32, 1,999,000
    # pairs, both forms; 256 seeded pairs plus the most zero-heavy pairs
    # against the oracle, MCN identical
    import torch
    C = workloads.counts_matrix()
    m = C.shape[0]
    heavy, zf = _zero_heavy_pairs(C, 8)
    _log("case counts full size m=%d n=%d, zero fraction %.2f..%.2f" % (m, C.shape[1], zf.min(), zf.max()))
    assert zf.min() >= 0.2 and zf.max() >= 0.5
    rng = np.random.default_rng(92)
    pl = set(heavy)
    while len(pl) < 256 + len(heavy):
        a, b = rng.integers(0, m, 2)
        if a != b:
            pl.add((int(min(a, b)), int(max(a, b))))
    pl = sorted(pl)
    idx = np.array([i * m - i * (i + 1) // 2 + (j - i - 1) for i, j in pl])
    want = oracle.allpairs(C.astype(np.float64), 0.6, 15.0, pairs=np.array(pl))
    Cd = torch.from_numpy(C).cuda()
    got64 = micx.allpairs(Cd, 0.6, 15.0, micx.MODE_FP64).cpu().numpy()[idx]
    d64 = np.abs(got64[:, :3] - want[:, :3]).max()
    assert d64 <= 1e-10, d64
    assert np.abs(got64[:, 3] - want[:, 3]).max() < 1e-9
    micx.set_profiling(True)
    try:
        got32 = micx.allpairs(Cd, 0.6, 15.0, micx.MODE_DP32).cpu().numpy()[idx]
        prof = micx.get_profile()
    finally:
        micx.set_profiling(False)
    bound = prof["dp32_bound"]
    # heavy ties leave near-tied cells: the statistics kernel flags pairs and
    # queues their items for the FP64 recheck
    assert prof["recheck_pairs"] > 0 and prof["recheck_items"] > 0, prof
    d32 = np.abs(got32[:, :3] - want[:, :3]).max()
    _log("counts full size: fp64 max|d| %.3g, dp32 max|d| %.3g (bound %.3g)" % (d64, d32, bound))
    assert d32 <= 2 * bound + 1e-12
    mism = np.flatnonzero(np.abs(got32[:, 3] - want[:, 3]) >= 1e-9)
    assert len(mism) == 0, [(pl[k], got32[k], want[k]) for k in mism[:5]]


def test_counts_integer_stages_heavy_zeros(micx):
    # bit-exact integer stages on four of the most zero-heavy pairs, every row
    # count, both orientations
    C = workloads.counts_matrix()
    heavy, _ = _zero_heavy_pairs(C, 4)
    for i, j in heavy:
        x, y = C[i].astype(np.float64), C[j].astype(np.float64)
        _log("case counts integer stages pair (%d, %d)" % (i, j))
        B = oracle.grid_bound(len(x), 0.6)
        for orient in (0, 1):
            for ry in range(2, B // 2 + 1):
                g = micx.debug_item(x, y, 0.6, 15.0, orient, ry)
                w = oracle.item(x, y, 0.6, 15.0, orient, ry)
                assert g["yhat"] == w["yhat"], (i, j, orient, ry)
                assert np.array_equal(g["row_starts"], w["row_starts"]), (i, j, orient, ry)
                assert g["k"] == w["k"] and g["K"] == w["K"], (i, j, orient, ry)
                assert np.array_equal(g["ends"], w["ends"]), (i, j, orient, ry)
