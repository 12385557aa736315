"""The C-ABI library builds, loads and exports every symbol include/micx.h
declares.  Host-only entry points (no kernel launch) are exercised here;
compute calls need a GPU and live in test_gpu_*.py."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_1208_4271_amd as micx
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "micx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(micx_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = micx.load_library()
    declared = _declared_functions()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(micx.EXPORTS) == declared


def test_library_is_built_for_gfx950():
    data = open(micx.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_check_param_messages():
    assert micx.check_param(0.6, 15) is None
    assert micx.check_param(0.0, 15) is not None
    assert micx.check_param(1.2, 15) is not None
    assert micx.check_param(0.6, 0.0) is not None
    assert micx.check_param(0.6, -1.0) is not None
    assert micx.check_param(1.0, 1e-3) is None


def test_grid_bound_matches_oracle_on_boundary_sizes():
    for n in (11, 243, 1024, 3125, 7776, 1340, 400, 200):
        assert micx.grid_bound(n, 0.6) == oracle.grid_bound(n, 0.6)
    for n in (81, 256, 4096, 8000):
        assert micx.grid_bound(n, 0.75) == oracle.grid_bound(n, 0.75)


def test_strerror_covers_codes():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert micx.strerror(code)
    assert micx.strerror(-99) == "unknown error"


def test_workloads_shapes():
    X = workloads.relations_matrix()
    assert X.shape == (64, 400) and X.dtype == np.float32
    x, y = workloads.sine_pair()
    assert len(x) == 200 and x.dtype == np.float64


def test_build_reads_dp_resource_usage():
    # The build rejects DP kernels that spill; it reads the compiler's
    # kernel-resource-usage remarks.  The parser must key each DP instance by
    # (fixed-point, NL, YR, T) and pick up its scratch and spill figures.
    from paper_1208_4271_amd import _build
    text = "\n".join([
        "x.h:1:1: remark: Function Name: _ZN4micx4k_dpIjLi36ELi2ELi2ELb0EEEvNS_6DpArgsE [-Rpass-analysis]",
        "x.h:1:1: remark:     VGPRs: 180 [-Rpass-analysis]",
        "x.h:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis]",
        "x.h:1:1: remark:     VGPRs Spill: 0 [-Rpass-analysis]",
        "x.h:1:1: remark: Function Name: _ZN4micx4k_dpIdLi10ELi5ELi1ELb1EEEvNS_6DpArgsE [-Rpass-analysis]",
        "x.h:1:1: remark:     VGPRs: 128 [-Rpass-analysis]",
        "x.h:1:1: remark:     ScratchSize [bytes/lane]: 152 [-Rpass-analysis]",
        "x.h:1:1: remark:     VGPRs Spill: 37 [-Rpass-analysis]",
        "x.h:1:1: remark: Function Name: _ZN4micx6k_partILb0EEEvNS_8PartArgsE [-Rpass-analysis]",
        "x.h:1:1: remark:     ScratchSize [bytes/lane]: 64 [-Rpass-analysis]",
    ])
    u = _build.dp_resource_usage(text)
    assert set(u) == {(1, 36, 2, 2), (0, 10, 5, 1)}
    assert u[(1, 36, 2, 2)]["ScratchSize"] == 0 and u[(1, 36, 2, 2)]["VGPRs"] == 180
    assert u[(0, 10, 5, 1)]["ScratchSize"] == 152 and u[(0, 10, 5, 1)]["VGPRs Spill"] == 37
    assert _build.spilling(u) == [(0, 10, 5, 1)]


def test_build_flags_agpr_spills():
    # VGPRs parked in accumulation registers count as a spill too
    from paper_1208_4271_amd import _build
    text = "\n".join([
        "x.h:1:1: remark: Function Name: _ZN4micx4k_dpIdLi36ELi2ELi2ELb1EEEvNS_6DpArgsE [-Rpass-analysis]",
        "x.h:1:1: remark:     VGPRs: 256 [-Rpass-analysis]",
        "x.h:1:1: remark:     AGPRs: 4 [-Rpass-analysis]",
        "x.h:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis]",
        "x.h:1:1: remark:     VGPRs Spill: 0 [-Rpass-analysis]",
        "x.h:1:1: remark: Function Name: _ZN4micx4k_dpIjLi36ELi2ELi3ELb0EEEvNS_6DpArgsE [-Rpass-analysis]",
        "x.h:1:1: remark:     VGPRs: 226 [-Rpass-analysis]",
        "x.h:1:1: remark:     AGPRs: 0 [-Rpass-analysis]",
        "x.h:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis]",
    ])
    u = _build.dp_resource_usage(text)
    assert u[(0, 36, 2, 2)]["AGPRs"] == 4
    assert _build.spilling(u) == [(0, 36, 2, 2)]


def test_cli_reads_csv_and_modes(tmp_path):
    # the mine-style front end: CSV parsing and pair selection (no GPU needed)
    from paper_1208_4271_amd import cli
    p = tmp_path / "d.csv"
    p.write_text("gA,1,2,3,4\n5,6,7,8\ngC,0.5,0.25,0.125,1e-3\n")
    names, X = cli.read_csv(str(p))
    assert names == ["gA", "2", "gC"] and X.shape == (3, 4) and X[2, 3] == 1e-3
    assert cli.pair_list(3) is None
    assert cli.pair_list(3, master=2) == [(1, 0), (1, 2)]
    assert cli.pair_list(3, pair=(3, 1)) == [(2, 0)]
    with pytest.raises(ValueError):
        cli.pair_list(3, master=4)
    with pytest.raises(ValueError):
        cli.pair_list(3, pair=(2, 2))
    bad = tmp_path / "bad.csv"
    bad.write_text("a,1,2,3\nb,1,2\n")
    with pytest.raises(ValueError):
        cli.read_csv(str(bad))
    args = cli.parse(["x.csv", "-a", "0.55", "-c", "10", "-m", "3", "-o", "o.tsv"])
    assert args.alpha == 0.55 and args.clumps == 10 and args.master == 3 and args.output == "o.tsv"


def test_bench_refuses_more_than_one_gpu():
    # the path runs on one GPU; bench.py says so and exits before any GPU work
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_tune_table_round_trip(tmp_path):
    # the autotuner's table: load a file, save it back (host only, no device)
    src = tmp_path / "in.txt"
    src.write_text("micx-tune 1 gfx950\n1 11 2 37 10 3 36 2\n0 11 5 15 8 1 14 4\n")
    micx.tune_clear()
    try:
        micx.tune_load(str(src))
        out = tmp_path / "out.txt"
        micx.tune_save(str(out))
        lines = out.read_text().splitlines()
        assert lines[0] == "micx-tune 1 gfx950"
        assert sorted(lines[1:]) == sorted(["1 11 2 37 10 3 36 2", "0 11 5 15 8 1 14 4"])
        bad = tmp_path / "bad.txt"
        bad.write_text("micx-tune 1 gfx942\n")
        with pytest.raises(micx.MicxError):
            micx.tune_load(str(bad))
    finally:
        micx.tune_clear()


def test_dp32_bound_is_the_largest_entry_bound():
    # the 32-bit DP's per-entry error l (yhat+1) / (2 S n ln min(l, yhat)),
    # maximised by brute force over 2 <= l <= x, 2 <= yhat <= y, against the
    # library's closed form (host arithmetic, no device)
    import math
    for n in (200, 1340, 8000):
        for y in range(2, 60):
            S = math.floor(2.0 ** 32 / (1.02 * n * math.log(y)))
            for x in range(2, 60):
                want = max(l * (yh + 1) / math.log(min(l, yh))
                           for l in range(2, x + 1) for yh in range(2, y + 1)) / (2.0 * S * n)
                got = micx.dp32_bound(n, x, y)
                assert abs(got - want) <= 1e-12 * want, (n, x, y, got, want)
                # never looser than the product of the worst l and the worst normaliser
                assert got <= (y + 1) * x / (2.0 * S * n * math.log(2.0)) * (1 + 1e-12)
    assert micx.dp32_bound(1340, 1, 5) == 0.0 and micx.dp32_bound(1340, 5, 1) == 0.0
