"""The oracle against the paper's worked examples (Section 3)."""
import os
from fractions import Fraction

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_table1():
    rows = []
    with open(os.path.join(GOLDEN, "wilkinson20_table1.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return {int(r[0]): r[1:] for r in rows}


def test_wilkinson20_eigenvalue_errors_match_table1_magnitudes():
    """Example 1: refine the double-precision Schur form of the companion matrix,
    stored exactly as double-double, with a double-precision solve and binary128
    products. The errors must be of the order the paper prints for Algorithm 4:
    each at most 10x the 2-double column, the largest at most 10x the largest
    error of the 34-digit column."""
    table = load_table1()
    hi, lo, exact = synth.wilkinson_companion_dd(20)
    qh = synth.hp_schur_start(hi)
    r = oracle.refine((hi, lo), qh, lp="double", maxit=10, tol=1e-33)
    assert r["status"] == "OK"
    thi, tlo = r["T"].to_dd()
    errs = {}
    for i in range(20):
        re = Fraction(thi[i, i].real) + Fraction(tlo[i, i].real)
        im = Fraction(thi[i, i].imag) + Fraction(tlo[i, i].imag)
        k = int(round(float(re)))
        errs[k] = abs(complex(float(re - k), float(im)))
    assert sorted(errs) == list(range(1, 21))
    for k, e in errs.items():
        assert e <= 10 * abs(table[k][3]), (k, e, table[k][3])
    assert max(errs.values()) <= 10 * max(abs(v[1]) for v in table.values())
    # and far better than double-precision root finding (second column)
    assert max(errs.values()) < 1e-10 * max(abs(v[0]) for v in table.values())
