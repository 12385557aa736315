"""micx_score_noalloc, the entry point that allocates nothing, against
micx_compute_score (same computation, host in/out, library-owned buffers),
through the C ABI: two calls in a row, the second on a smaller input, in both
numeric forms; error handling; no device memory taken by the calls."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _pair(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, n)
    return x, np.sin(7 * x) + rng.normal(0, 0.25, n)


def _noalloc(micx, x, y, alpha, c, mode):
    import torch
    B = micx.grid_bound(len(x), alpha)
    W = B // 2 - 1
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float64)).cuda()
    stats = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
    mats = torch.full((3 * W * W,), -7.0, dtype=torch.float64, device="cuda")
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    micx.score_noalloc(xd, yd, alpha, c, mode, stats, mats, status)
    torch.cuda.synchronize()
    m = mats.cpu().numpy().reshape(3, W, W)
    return {"stats": stats.cpu().numpy(), "M": m[0], "Axy": m[1], "Ayx": m[2],
            "status": int(status.cpu().numpy()[0])}


@pytest.mark.parametrize("mode_name", ["fp64", "dp32"])
def test_noalloc_matches_compute_score(micx, mode_name):
    mode = micx.MODE_FP64 if mode_name == "fp64" else micx.MODE_DP32
    # the second call on a smaller input: buffers of the first stay in the
    # array and must not leak into the second
    for seed, n, alpha in ((1, 3000, 0.6), (2, 700, 0.65)):
        x, y = _pair(seed, n)
        _log("case noalloc %s n=%d alpha=%.2f" % (mode_name, n, alpha))
        got = _noalloc(micx, x, y, alpha, 15.0, mode)
        want = micx.compute_score(x, y, alpha, 15.0, mode=mode)
        assert got["status"] == micx.MICX_OK
        ok = ~np.isnan(want["M"])
        assert np.array_equal(np.isnan(got["M"]), ~ok)
        for key in ("M", "Axy", "Ayx"):
            assert np.abs(got[key][ok] - want[key][ok]).max() <= 1e-12, key
        assert np.abs(got["stats"] - want["stats"]).max() <= 1e-12, (got["stats"], want["stats"])


def test_noalloc_paper_example_and_errors(micx):
    import torch
    x, y = workloads.cpp_example()
    got = _noalloc(micx, x, y, 0.6, 15.0, micx.MODE_FP64)
    for v, p in zip(got["stats"], (0.999999, 0.728144, 0.999999, 4.584963)):
        assert abs(v - p) <= 5e-7 + 1e-12
    # a NaN: the device-side status says so, the outputs stay untouched
    bad = x.copy()
    bad[10] = np.nan
    got = _noalloc(micx, bad, y, 0.6, 15.0, micx.MODE_DP32)
    assert got["status"] == micx.MICX_ENONFINITE
    assert (got["stats"] == -7.0).all() and (got["M"] == -7.0).all()
    # beyond the array: refused before any work
    n = 8000
    xd = torch.zeros(n, dtype=torch.float64, device="cuda")
    stats = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(micx.MicxError) as e:
        micx.score_noalloc(xd, xd, 0.75, 15.0, micx.MODE_FP64, stats)
    assert e.value.code == micx.MICX_ETOOBIG
    with pytest.raises(micx.MicxError) as e:
        micx.score_noalloc(xd[:5], xd[:5], 0.6, 15.0, micx.MODE_FP64, stats)
    assert e.value.code == micx.MICX_ESMALLN
    torch.cuda.synchronize()
    assert (stats.cpu().numpy() == -7.0).all()


def test_noalloc_takes_no_device_memory(micx):
    import torch
    x, y = _pair(5, 2500)
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y).cuda()
    stats = torch.empty(4, dtype=torch.float64, device="cuda")
    micx.score_noalloc(xd, yd, 0.6, 15.0, micx.MODE_DP32, stats)   # warm-up (code objects)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        micx.score_noalloc(xd, yd, 0.6, 15.0, micx.MODE_DP32, stats)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
