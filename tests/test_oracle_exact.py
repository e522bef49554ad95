"""Pins of the exact row checker (oracle/exact.py): exact reconstruction of
multi-term matrices, brute force in rationals on small inputs, and the closed
forms of an exactly known Schur decomposition."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import exact


def _rand_terms(rng, m, n, terms=3):
    hi = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    out = [hi]
    if terms > 1:
        out.append((rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * 2.0 ** -54)
    if terms > 2:
        out.append((rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * 2.0 ** -108)
    return out


def _frac(terms):
    re = np.zeros(terms[0].shape, dtype=object)
    im = np.zeros(terms[0].shape, dtype=object)
    for t in terms:
        re = re + np.vectorize(Fraction)(np.real(t))
        im = im + np.vectorize(Fraction)(np.imag(t))
    return re, im


def test_to_ints_is_exact():
    rng = np.random.default_rng(1)
    terms = _rand_terms(rng, 6, 5)
    terms[0][0, 0] = 0.0
    terms[1][1, 1] = 5e-324 + 3e-310j  # subnormals
    terms[2][2, 2] = -(2.0 ** -1000)
    re, im, e = exact.to_ints(terms)
    fr, fi = _frac(terms)
    for i in range(6):
        for j in range(5):
            assert Fraction(int(re[i, j]), 1 << e) == fr[i, j]
            assert Fraction(int(im[i, j]), 1 << e) == fi[i, j]
    r2, i2, e2 = exact.to_ints([np.zeros((2, 2))])
    assert e2 == 0 and all(int(v) == 0 for v in np.ravel(r2))


@pytest.mark.parametrize("n", [3, 5])
def test_rows_against_rational_brute_force(n):
    """Every row, against Q^H A Q and Q^H Q - I formed entry by entry in rationals."""
    rng = np.random.default_rng(n)
    a = _rand_terms(rng, n, n, terms=2)
    q = _rand_terms(rng, n, n)
    ar, ai = _frac(a)
    qr, qi = _frac(q)
    stril = Fraction(0)
    orth = Fraction(0)
    rowmax = Fraction(0)
    for i in range(n):
        row = Fraction(0)
        for j in range(n):
            # (Q^H A Q)_ij = sum_k sum_l conj(q_ki) a_kl q_lj
            sr = si = Fraction(0)
            gr = gi = Fraction(0)
            for k in range(n):
                cr, ci = qr[k, i], -qi[k, i]
                gr += cr * qr[k, j] - ci * qi[k, j]
                gi += cr * qi[k, j] + ci * qr[k, j]
                for l in range(n):
                    pr = cr * ar[k, l] - ci * ai[k, l]
                    pi = cr * ai[k, l] + ci * ar[k, l]
                    sr += pr * qr[l, j] - pi * qi[l, j]
                    si += pr * qi[l, j] + pi * qr[l, j]
            if j < i:
                row += sr * sr + si * si
            if i == j:
                gr -= 1
            orth += gr * gr + gi * gi
        stril += row
        rowmax = max(rowmax, row)
    na2 = sum(ar[k, l] ** 2 + ai[k, l] ** 2 for k in range(n) for l in range(n))
    got = exact.residual_rows(a, q, np.arange(n))
    assert got["stril"] == pytest.approx(float(stril / na2) ** 0.5, rel=1e-14)
    assert got["stril_rowmax"] == pytest.approx(float(rowmax / na2) ** 0.5, rel=1e-14)
    assert got["orth"] == pytest.approx(float(orth) ** 0.5, rel=1e-14)
    assert got["normA"] == pytest.approx(float(na2) ** 0.5, rel=1e-15)
    # a subset of rows: the unbiased estimate scales the rows' sum by n / r
    sub = exact.residual_rows(a, q, np.array([n - 1]))
    assert sub["stril"] ** 2 == pytest.approx(sub["stril_rowmax"] ** 2 * n, rel=1e-13)


@pytest.mark.parametrize("n", [16, 64])
def test_exact_hadamard_schur_form(n):
    """A = Q0 T0 Q0^H exactly in binary: Q0 gives exactly zero residual and defect;
    swapping its first two columns moves T0[0, 1] to position (1, 0), and only it."""
    h = synth.hadamard_exact(n, seed=n + 1)
    got = exact.residual_rows([h["A"]], [h["Q0"]], np.arange(n))
    assert got["stril"] == 0.0 and got["orth"] == 0.0
    q = h["Q0"].copy()
    q[:, [0, 1]] = q[:, [1, 0]]
    got = exact.residual_rows([h["A"]], [q], np.arange(n))
    t01 = abs(h["T0"][0, 1])
    assert t01 > 0
    na = np.linalg.norm(h["A"])
    assert got["stril"] == pytest.approx(t01 / na, rel=1e-14)
    assert got["stril_rowmax"] == pytest.approx(t01 / na, rel=1e-14)
    assert got["orth"] == 0.0
