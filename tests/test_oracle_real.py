"""Pins of the oracle's real Schur variant (CPU): the block form of the triangular
matrix equation and Algorithm 4 on real data with 2 x 2 diagonal blocks."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from real_util import block_lower_mask as _block_lower_mask
from real_util import exact_real_problem as _exact_real_problem
from real_util import quasi_upper as _quasi_upper
from real_util import rotated as _rotated


def _fraction_block_solve(t, e, blk):
    """The defining equation written out as one linear system over every unknown of
    the block strictly lower L (the Kronecker form of block-stril(T L - L T) = -E),
    solved exactly with rational Gauss-Jordan elimination."""
    n = t.shape[0]
    mask = _block_lower_mask(n, blk)
    unk = [(i, j) for j in range(n) for i in range(n) if mask[i, j]]
    idx = {p: k for k, p in enumerate(unk)}
    F = [[Fraction(float(t[i, j])) for j in range(n)] for i in range(n)]
    rows = []
    for (i, j) in unk:
        # (T L - L T)_ij = sum_k t_ik l_kj - sum_k l_ik t_kj = -e_ij
        row = [Fraction(0)] * (len(unk) + 1)
        for k in range(n):
            if (k, j) in idx:
                row[idx[(k, j)]] += F[i][k]
            if (i, k) in idx:
                row[idx[(i, k)]] -= F[k][j]
        row[-1] = -Fraction(float(e[i, j]))
        rows.append(row)
    m = len(unk)
    for c in range(m):
        piv = next(r for r in range(c, m) if rows[r][c] != 0)
        rows[c], rows[piv] = rows[piv], rows[c]
        for r in range(m):
            if r != c and rows[r][c] != 0:
                f = rows[r][c] / rows[c][c]
                rows[r] = [x - f * y for x, y in zip(rows[r], rows[c])]
    return {(i, j): rows[k][-1] / rows[k][k] for (i, j), k in idx.items()}


@pytest.mark.parametrize("sizes", [[2, 1, 2], [1, 2, 1], [2, 2], [1, 1, 2, 1]])
def test_block_solve_matches_exact_kronecker_system(sizes):
    rng = np.random.default_rng(sum(sizes) * 7 + len(sizes))
    t, blk = _quasi_upper(rng, sizes, dyadic=True)
    n = t.shape[0]
    mask = _block_lower_mask(n, blk)
    e = np.where(mask, np.round(rng.standard_normal((n, n)) * 64) / 64, 0.0)
    exact = _fraction_block_solve(t, e, blk)
    lq, st = oracle.trisolve_real(t.astype(complex), e.astype(complex), blk, lp="quad")
    assert st == "OK"
    hi, lo = lq.to_dd()
    assert not hi.imag.any()
    scale = max(1.0, max(abs(float(v)) for v in exact.values()))
    for (i, j), v in exact.items():
        assert abs(float(Fraction(hi[i, j].real) + Fraction(lo[i, j].real) - v)) <= 1e-30 * scale, (i, j)
    assert not hi[~mask].any()  # block strictly lower


def test_block_solve_on_1x1_blocks_is_the_scalar_solve():
    """With every block of order 1 the block solve is the scalar Algorithm 2 (the
    complex solve on real data): the same L to binary128 rounding."""
    rng = np.random.default_rng(4)
    n = 30
    t = np.triu(rng.standard_normal((n, n)))
    t[np.diag_indices(n)] = np.arange(n) + 1.0
    e = np.tril(rng.standard_normal((n, n)), -1)
    lr, st = oracle.trisolve_real(t.astype(complex), e.astype(complex), None, lp="quad")
    lc, st2 = oracle.trisolve(t.astype(complex), e.astype(complex), lp="quad")
    assert st == st2 == "OK"
    a, b = lr.to_dd(), lc.to_dd()
    scale = np.abs(b[0]).max()
    assert np.abs((a[0] - b[0]) + (a[1] - b[1])).max() <= 1e-30 * scale


def test_block_solve_float_residual_and_breakdown():
    rng = np.random.default_rng(8)
    sizes = [2, 1, 2, 2, 1, 1, 2, 1, 2]
    t, blk = _quasi_upper(rng, sizes)
    n = t.shape[0]
    mask = _block_lower_mask(n, blk)
    e = np.where(mask, 1e-6 * rng.standard_normal((n, n)), 0.0)
    lf, st = oracle.trisolve_real(t.astype(complex), e.astype(complex), blk, lp="float")
    assert st == "OK"
    l = lf.to_c128().real
    t32, e32 = t.astype(np.float32).astype(float), e.astype(np.float32).astype(float)
    r = np.where(mask, t32 @ l - l @ t32 + e32, 0.0)
    assert np.linalg.norm(r) <= 8 * n * 2.0**-24 * (np.linalg.norm(t) * np.linalg.norm(l) + np.linalg.norm(e))
    # the float solve is FP32 arithmetic: its error against the quad solve is of that size
    lq = oracle.trisolve_real(t.astype(complex), e.astype(complex), blk, lp="quad")[0].to_c128().real
    err = np.linalg.norm(l - lq) / np.linalg.norm(lq)
    assert 1e-9 < err < 1e-4
    # two 2 x 2 blocks with the same eigenvalues make the equation singular
    t2, blk2 = _quasi_upper(rng, [2, 2])
    t2[2:, 2:] = t2[:2, :2]
    e2 = np.where(_block_lower_mask(4, blk2), 1.0, 0.0)
    assert oracle.trisolve_real(t2.astype(complex), e2.astype(complex), blk2, lp="quad")[1] == "BREAKDOWN"


@pytest.mark.parametrize("n", [16, 64])
def test_refine_real_recovers_exact_real_schur_form(n):
    a, q0, t0, blk = _exact_real_problem(n, n + 3)
    assert np.array_equal((q0 @ t0) @ q0.T, a)
    ev = oracle.evaluate_real(a.astype(complex), q0.astype(complex), t0.astype(complex), blk)
    assert ev["stril"] == 0 and ev["orth"] == 0 and ev["tdiff"] == 0
    qh = _rotated(q0, 1, 1e-6)
    r = oracle.refine_real(a.astype(complex), qh.astype(complex), blk, lp="quad", maxit=8, tol=1e-30)
    assert r["status"] == "OK" and r["iters"] <= 5, r["hist"]
    # quadratic decrease (Theorem 2)
    h = r["hist"]
    for k in range(1, len(h)):
        if h[k - 1] > 1e-25:
            assert h[k] <= 10 * h[k - 1] ** 2 * 1e6 or h[k] <= 1e-30
    t, _ = r["T"].to_dd()
    # every diagonal block's invariant subspace is recovered: Q0^T Q (binary128) is
    # block diagonal to 1e-28; and each block's eigenvalues
    mh, ml = oracle.gemm(q0.astype(complex), r["Q"], opa=1).to_dd()
    m = np.abs(mh + ml)
    i = 0
    while i < n:
        s = 2 if blk[i] else 1
        off = np.delete(m[:, i:i + s], np.s_[i:i + s], axis=0)
        assert off.max() <= 1e-28, (i, off.max())
        ev_t = np.sort_complex(np.linalg.eigvals(t.real[i:i + s, i:i + s]))
        ev_0 = np.sort_complex(np.linalg.eigvals(t0[i:i + s, i:i + s]))
        assert np.abs(ev_t - ev_0).max() <= 1e-13
        i += s
    assert not np.where(_block_lower_mask(n, blk), t.real, 0.0).any()


def test_refine_real_float_lp_convergence():
    """FP32 lp from the sgees start: every pass above the FP64 floor gains at least
    five decades (the observable law with an lp solve), reaching 1e-15 in <= 4 passes."""
    g = synth.real_schur_test_matrix(48, seed=11)
    qh, blk = synth.lp_real_schur_start(g["A"])
    assert blk.sum() == g["blk"].sum()
    r = oracle.refine_real(g["A"].astype(complex), qh.astype(complex), blk, lp="float", maxit=6, tol=1e-15)
    assert r["status"] == "OK" and r["iters"] <= 4, r["hist"]
    h = r["hist"]
    for k in range(1, len(h)):
        assert h[k] <= 1e-5 * h[k - 1] or h[k] <= 1e-15
    # the eigenvalues of the blocks are those of A
    t = r["T"].to_c128().real
    lam = []
    i = 0
    while i < 48:
        s = 2 if blk[i] else 1
        lam += list(np.linalg.eigvals(t[i:i + s, i:i + s]))
        i += s
    d = np.abs(np.sort_complex(np.array(lam)) - np.sort_complex(g["lam"]))
    assert d.max() <= 1e-12


def test_refine_real_equals_complex_on_real_spectrum():
    """A real matrix with a real spectrum has no 2 x 2 blocks; the real refinement is
    then the complex one on real data (same steps): the same Q to binary128 rounding."""
    g = synth.real_schur_test_matrix(24, seed=5, n_real=24)
    assert not g["blk"].any()
    qh, blk = synth.lp_real_schur_start(g["A"])
    assert not blk.any()
    rr = oracle.refine_real(g["A"].astype(complex), qh.astype(complex), blk, lp="quad", maxit=5, tol=1e-30)
    rc = oracle.refine(g["A"].astype(complex), qh.astype(complex), lp="quad", maxit=5, tol=1e-30)
    assert rr["iters"] == rc["iters"] and np.allclose(rr["hist"], rc["hist"], rtol=1e-6, atol=1e-40)
    a, b = rr["Q"].to_dd(), rc["Q"].to_dd()
    assert np.abs((a[0] - b[0]) + (a[1] - b[1])).max() <= 1e-28
