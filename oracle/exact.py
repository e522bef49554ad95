"""Exact checks of a Schur decomposition in Python integers: TEST INFRASTRUCTURE ONLY.

Only the test suite and the benchmark's checks may import this module; the GPU
library never calls it, and the two share no code.

A matrix enters as a list of float64 or complex128 arrays whose sum it is (a
multi-term expansion such as the triple-double tier's three terms, or one array).
Every double is m 2^e with an integer m of at most 53 bits, so one power of two
turns the whole sum into integers without rounding; products and sums of those
integers are exact. That reaches where binary128 (113 bits) cannot: residuals
near 2^-150.

What is evaluated is the plain definition of the two quantities the refinement
drives to zero (Section 2): the strictly lower triangle of Q^H A Q relative to
||A||_F, and Q^H Q - I, on a set of rows (row i of Q^H A Q is (q_i^H A) Q).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

_SHIFT = np.frompyfunc(lambda m, s: int(m) << int(s), 2, 1)


def to_ints(terms):
    """(re, im, e): object arrays of Python ints with sum(terms) = (re + i im) 2^-e
    exactly (e common to every entry and both parts)."""
    parts = []
    for t in terms:
        t = np.asarray(t)
        parts.append(np.real(t).astype(np.float64))
        parts.append(np.imag(t).astype(np.float64) if np.iscomplexobj(t) else np.zeros(t.shape))
    e_min = None
    fr = []
    for p in parts:
        if not np.all(np.isfinite(p)):
            raise ValueError("non-finite entry")
        m, ex = np.frexp(p)  # p = m 2^ex, 0.5 <= |m| < 1 (m = 0 for zeros)
        mant = np.ldexp(m, 53).astype(np.int64)  # exact: m has at most 53 bits
        ex = ex.astype(np.int64) - 53
        nz = mant != 0
        if nz.any():
            lo = int(ex[nz].min())
            e_min = lo if e_min is None else min(e_min, lo)
        fr.append((mant, ex, nz))
    e = 0 if e_min is None else -e_min
    out = []
    for mant, ex, nz in fr:
        shift = np.where(nz, ex + e, 0)
        out.append(_SHIFT(mant, shift))
    re = sum(out[0::2])
    im = sum(out[1::2])
    return re, im, e


def _sq(x):
    return sum(int(v) * int(v) for v in np.ravel(x))


def residual_rows(a_terms, q_terms, rows) -> dict:
    """Exact rows of Q^H A Q and Q^H Q - I.

    Returns floats: `stril` the unbiased estimate sqrt(n / r sum_rows sum_{j<i}
    |(Q^H A Q)_ij|^2) / ||A||_F over the r sampled rows (the full value when every
    row is sampled), `stril_rowmax` the largest row's strictly lower 2-norm over
    ||A||_F, `orth` the same estimate for the rows of Q^H Q - I, and `normA`."""
    ar, ai, ea = to_ints(a_terms)
    qr, qi, eq = to_ints(q_terms)
    n = qr.shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    qrr, qir = qr[:, rows].T, qi[:, rows].T  # the rows of Q^H, before conjugation
    # v = q_i^H A, then row = v Q (scale 2^-(ea + 2 eq))
    vr = qrr.dot(ar) + qir.dot(ai)
    vi = qrr.dot(ai) - qir.dot(ar)
    rr = vr.dot(qr) - vi.dot(qi)
    ri = vr.dot(qi) + vi.dot(qr)
    # g = q_i^H Q - e_i (scale 2^-(2 eq))
    gr = qrr.dot(qr) + qir.dot(qi)
    gi = qrr.dot(qi) - qir.dot(qr)
    one = 1 << (2 * eq)
    for k, i in enumerate(rows):
        gr[k, i] -= one
    s_res = 2 * (ea + 2 * eq)
    row_sq = []
    for k, i in enumerate(rows):
        row_sq.append(_sq(rr[k, :i]) + _sq(ri[k, :i]))
    na2 = Fraction(_sq(ar) + _sq(ai), 1 << (2 * ea))
    norm_a = float(na2) ** 0.5
    tot = Fraction(sum(row_sq), 1 << s_res)
    scale = Fraction(n, len(rows))
    stril = float(tot * scale / na2) ** 0.5 if na2 else 0.0
    rowmax = max(float(Fraction(s, 1 << s_res) / na2) ** 0.5 for s in row_sq) if na2 else 0.0
    o = Fraction(_sq(gr) + _sq(gi), 1 << (4 * eq))
    return {"stril": stril, "stril_rowmax": rowmax, "orth": float(o * scale) ** 0.5, "normA": norm_a}
