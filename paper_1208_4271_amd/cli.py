"""Command-line front end in the style of the paper's `mine` application:
the four MINE statistics, Pearson's rho and the non-linearity index for the
variables of a CSV file, computed on the GPU.

    python -m paper_1208_4271_amd.cli data.csv -a 0.6 -c 15 [-m VAR | -p VAR1 VAR2] -o out.tsv

Input: one variable per line, values separated by commas; a first field that
is not a number is the variable's name (else the name is its number).  VAR
numbers count from 1, as in the paper's usage examples.  Modes (the paper's
usage examples): all pairs i < j (default), a master variable against every
other one (-m), or one pair (-p).  Output: a header and one tab-separated line
per pair: X var, Y var, MIC, MAS, MEV, MCN, Pearson, MIC-p^2.
"""
from __future__ import annotations

import argparse
import sys

import numpy as np

HEADER = "X var\tY var\tMIC (strength)\tMAS (non-monotonicity)\tMEV (functionality)\t" \
         "MCN (complexity)\tLinear regression (Pearson)\tMIC-p^2 (nonlinearity)"


def read_csv(path: str):
    """(names, values): one variable per line; float64 array (m, n)."""
    names, rows = [], []
    with open(path) as fh:
        for ln, line in enumerate(fh, 1):
            f = [t.strip() for t in line.strip().split(",")]
            if not f or f == [""]:
                continue
            try:
                float(f[0])
                name, vals = None, f
            except ValueError:
                name, vals = f[0], f[1:]
            try:
                rows.append([float(v) for v in vals])
            except ValueError:
                raise ValueError("%s:%d: a value is not a number" % (path, ln))
            names.append(name if name is not None else str(len(rows)))
    if len(rows) < 2:
        raise ValueError("%s: at least two variables are needed" % path)
    n = len(rows[0])
    if any(len(r) != n for r in rows):
        raise ValueError("%s: every variable needs the same number of values" % path)
    return names, np.asarray(rows, dtype=np.float64)


def parse(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1208_4271_amd.cli",
                                 description="MINE statistics, Pearson and MIC-p^2 of CSV variables")
    ap.add_argument("input", help="CSV file, one variable per line")
    ap.add_argument("-a", "--alpha", type=float, default=0.6, help="grid-size exponent (default 0.6)")
    ap.add_argument("-c", "--clumps", type=float, default=15.0, help="clumping factor (default 15)")
    g = ap.add_mutually_exclusive_group()
    g.add_argument("-m", "--master", type=int, help="variable VAR (from 1) against all others")
    g.add_argument("-p", "--pair", type=int, nargs=2, metavar=("VAR1", "VAR2"), help="one pair")
    ap.add_argument("-o", "--output", help="output file (default: standard output)")
    ap.add_argument("--fp64", action="store_true",
                    help="run the DP in FP64 everywhere (default: the 32-bit form where its bound allows)")
    return ap.parse_args(argv)


def pair_list(m: int, master=None, pair=None):
    """0-based (i, j) pairs of the mode, or None for all pairs i < j."""
    if master is not None:
        if not 1 <= master <= m:
            raise ValueError("master variable %d out of range 1..%d" % (master, m))
        i = master - 1
        return [(i, j) for j in range(m) if j != i]
    if pair is not None:
        a, b = pair
        if not (1 <= a <= m and 1 <= b <= m) or a == b:
            raise ValueError("pair (%d, %d) out of range 1..%d or repeated" % (a, b, m))
        return [(a - 1, b - 1)]
    return None


def main(argv=None) -> int:
    args = parse(argv)
    import torch

    import paper_1208_4271_amd as micx
    names, X = read_csv(args.input)
    m = X.shape[0]
    pl = pair_list(m, args.master, args.pair)
    mode = micx.MODE_FP64 if args.fp64 else micx.MODE_DP32
    Xd = torch.from_numpy(X).cuda()
    if pl is None:
        stats = micx.allpairs(Xd, args.alpha, args.clumps, mode)
        ij = [(i, j) for i in range(m) for j in range(i + 1, m)]
    else:
        stats = micx.pairs(Xd, pl, args.alpha, args.clumps, mode)
        ij = pl
    pr = micx.pearson(Xd, pl, stats).cpu().numpy()
    st = stats.cpu().numpy()
    out = open(args.output, "w") if args.output else sys.stdout
    try:
        out.write(HEADER + "\n")
        for k, (i, j) in enumerate(ij):
            out.write("%s\t%s\t%.6f\t%.6f\t%.6f\t%.6f\t%.6f\t%.6f\n" % (
                names[i], names[j], st[k, 0], st[k, 1], st[k, 2], st[k, 3], pr[k, 0], pr[k, 1]))
    finally:
        if out is not sys.stdout:
            out.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
