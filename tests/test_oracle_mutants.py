"""The oracle's pins must catch plausible mistakes.

Each case copies mine_oracle.c, plants one mistake (a dropped term, an
off-by-one, a wrong reading of the paper), compiles the copy with gcc on the
CPU and runs the pin battery against it; at least one pin must fail.  The
unmodified source must pass the same battery.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads

SRC = os.path.join(os.path.dirname(oracle.__file__), "mine_oracle.c")

MUTANTS = {
    # h(s,t) loses its last row term
    "drop_row_term": ("for (int r = 0; r < yhat; r++)\n                acc += span_cost",
                      "for (int r = 0; r < yhat - 1; r++)\n                acc += span_cost"),
    # the garbled Algorithm 1: one fresh label per point of a mixed group
    "per_point_label": ("for (int j = 0; j < s; j++) lab[i + j] = fresh;\n            fresh--;",
                        "for (int j = 0; j < s; j++) lab[i + j] = fresh--;"),
    # desiredRowSize reset with the wrong remaining-point count
    "reset_off_by_one": ("desired = (double) (n - i) / (double) (y - row);",
                         "desired = (double) (n - i - 1) / (double) (y - row);"),
    # the DP never tries the source just before the target
    "dp_skip_last_source": ("for (size_t s = 1; s < t; s++)", "for (size_t s = 1; s + 1 < t; s++)"),
    # orientations combined at equal index instead of equal grid shape
    "combine_index": ("double b = (flags & ORC_COMBINE_INDEX)", "double b = !(flags & ORC_COMBINE_INDEX)"),
    # normalised by the requested row count instead of yhat (App. A item 4)
    "norm_by_requested": ("(l < yhat ? l : yhat)", "(l < ry ? l : ry)"),
    # one superclump more than khat (the MINE.jar behaviour of App. A item 7)
    "khat_plus_one": ("int k = (int) floor(c * (double) cx);", "int k = (int) floor(c * (double) cx) + 1;"),
    # Algorithm 2 read as consecutive clumps grouped by count, not by points
    "superclump_equal_count": (
        "int K = oracle_equipartition(d, n, limit, flags & (ORC_TIE_STRICT | ORC_DESIRED_INT), p);",
        "int per = (k + limit - 1) / limit; for (int i = 0; i < n; i++) p[i] = (int) d[i] / per;"
        " int K = p[n - 1] + 1;"),
    # the superclump step alone closes rows on '>' (the row step keeps '>=')
    "superclump_strict_tie": ("flags & (ORC_TIE_STRICT | ORC_DESIRED_INT), p);",
                              "(flags & ORC_DESIRED_INT) | ORC_TIE_STRICT, p);"),
    # no lower bound of one superclump when c x < 1
    "khat_no_floor_guard": ("return k < 1 ? 1 : k;", "return k;"),
}


def _battery() -> bool:
    """True iff every pin holds for the currently loaded oracle build."""
    ok = True
    # Fig. 2
    a, b = workloads.fig2_points()
    order = np.argsort(b, kind="stable")
    q_sorted, _ = oracle.equipartition(b[order], 3)
    q = np.empty(14, dtype=np.int32)
    q[order] = q_sorted
    ok &= list(q + 1) == [1, 1, 2, 2, 2, 2, 3, 3, 3, 3, 3, 2, 1, 1]
    p, _ = oracle.clumps(a, q)
    ok &= list(p + 1) == [1, 1, 1, 1, 2, 2, 3, 3, 3, 3, 3, 4, 5, 5]
    # C++ example
    x, y = workloads.cpp_example()
    st = oracle.score(x, y, 0.6, 15)["stats"]
    for v, want in zip(st, (0.999999, 0.728144, 0.999999, 4.584963)):
        ok &= abs(v - want) <= 5e-7 + 1e-12
    # exhaustive search on tiny inputs
    rng = np.random.default_rng(77)
    for trial in range(6):
        n = 11
        xx = rng.integers(0, 6, n).astype(float) if trial % 2 else rng.uniform(0, 1, n)
        yy = rng.integers(0, 5, n).astype(float) if trial % 3 == 0 else rng.uniform(0, 1, n)
        r = oracle.score(xx, yy, 1.0, 15.0)
        B = r["B"]
        ov, ou = np.argsort(yy, kind="stable"), np.argsort(xx, kind="stable")
        for ry in range(2, B // 2 + 1):
            qv, yhat = oracle.equipartition(yy[ov], ry)
            rowpt = np.empty(n, dtype=np.int32)
            rowpt[ov] = qv
            best = brute.best_partitions(xx[ou], rowpt[ou], B // ry)
            for l in range(2, B // ry + 1):
                norm = min(l, yhat)
                want = best[l] / math.log(norm) if norm >= 2 else 0.0
                ok &= abs(r["Axy"][ry - 2, l - 2] - want) < 1e-12
    # App. A item 4 closed form: a 3-level step observed through 4 requested
    # rows gives yhat = 3 and a pure grid, so the 4x4 entry is exactly 1.
    xs = np.linspace(0, 1, 300)
    ys = np.floor(xs * 3 - 1e-9).clip(0, 2)
    r = oracle.score(xs, ys, 0.6, 15)
    ok &= abs(r["Axy"][2, 2] - 1.0) < 1e-12
    # superclumps never exceed khat (App. A items 6-7)
    x1, y1 = workloads.sine_pair()
    B1 = oracle.grid_bound(len(x1), 0.6)
    for ry in range(2, B1 // 2 + 1):
        it = oracle.item(x1, y1, 0.6, 15, 0, ry)
        ok &= it["K"] <= 15 * (B1 // ry)
    it = oracle.item(x1, y1, 0.6, 1.0, 0, 2)
    ok &= it["K"] <= (B1 // 2)
    # Algorithm 2 worked by hand (tests/golden/superclumps_alg2.txt)
    from test_oracle_pins import clump_input, superclump_ends, superclump_goldens
    for _, khat, sizes, ends in superclump_goldens():
        a, q = clump_input(sizes)
        p, K, k = oracle.superclumps(a, q, khat)
        ok &= k == len(sizes) and K == len(ends) and superclump_ends(p) == ends
    # a bound below one column: one superclump
    for ry in range(2, B1 // 2 + 1):
        if math.floor(0.3 * (B1 // ry)) < 1:
            ok &= oracle.item(x1, y1, 0.6, 0.3, 0, ry)["K"] == 1
    return bool(ok)


def _build_variant(tmp_path, name, text):
    c = tmp_path / (name + ".c")
    c.write_text(text)
    so = tmp_path / (name + ".so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(c),
                    "-lm", "-lpthread"], check=True)
    return str(so)


def test_unmodified_oracle_passes_battery():
    assert _battery()


_CHILD = """
import importlib.util, sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
import oracle
spec = importlib.util.spec_from_file_location("mut", {here!r})
mod = importlib.util.module_from_spec(spec)
spec.loader.exec_module(mod)
with oracle._use_library({so!r}):
    ok = mod._battery()
sys.exit(0 if ok else 3)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    # The battery runs in a child process: a mutant may also corrupt memory,
    # and a crash counts as caught.
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1
    so = _build_variant(tmp_path, name, src.replace(old, new))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = _CHILD.format(root=root, tests=os.path.join(root, "tests"), here=os.path.abspath(__file__),
                         so=so)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode != 0, "pins did not catch mutant " + name
