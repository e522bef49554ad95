"""Double-double tier on the GPU: the double-double Ozaki product, the FP64
solve and the refinement to 1e-28, against the binary128 oracle."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from gpu_util import U64, dev, empty, host, phase_align, rand_c

pytestmark = pytest.mark.gpu

UDD = 2.0 ** -104
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def sr():
    import torch

    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _dd_rand(rng, shape):
    """A double-double matrix hi + lo with a full 106-bit significand."""
    hi = rand_c(rng, shape)
    lo = np.asfortranarray(hi * (U64 * (rng.random(shape) - 0.5)))
    return synth.to_dd(hi, lo)


def _dd_err(c_hi, c_lo, ref: "oracle.QMat"):
    rh, rl = ref.to_dd()
    return np.abs((c_hi - rh) + (c_lo - rl))


@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("shape", [(130, 97, 75), (64, 64, 64), (1, 3, 2), (257, 129, 300)])
def test_dd_product_matches_quad(sr, opa, shape):
    m, n, k = shape
    rng = np.random.default_rng(m + 3 * n + 7 * k + opa)
    ah, al = _dd_rand(rng, (k, m) if opa else (m, k))
    bh, bl = _dd_rand(rng, (k, n))
    ch, cl = empty(m, n), empty(m, n)
    assert sr.sr_ozaki_zgemm_dd(dev(ah), dev(al), dev(bh), dev(bl), ch, cl, opa=opa,
                                slices_a=14, slices_b=14, dmax=15) == 0
    ref = oracle.gemm(oracle.QMat.from_dd(ah, al), oracle.QMat.from_dd(bh, bl), opa=opa)
    err = _dd_err(host(ch), host(cl), ref)
    aa = np.abs(ah.conj().T if opa else ah)
    bound = 4 * (k + 4) * UDD * np.sqrt(2.0) * (aa @ np.abs(bh))
    assert np.all(err <= bound), (err / np.maximum(bound, 1e-300)).max()


def test_dd_product_add_and_exact_integers(sr):
    rng = np.random.default_rng(11)
    m, n, k = 70, 90, 40
    a = np.asfortranarray(rng.integers(-2**20, 2**20, (m, k)) + 1j * rng.integers(-2**20, 2**20, (m, k)))
    b = np.asfortranarray(rng.integers(-2**20, 2**20, (k, n)) + 1j * rng.integers(-2**20, 2**20, (k, n)))
    c0 = np.asfortranarray(rng.integers(-2**40, 2**40, (m, n)) * (1 + 1j))
    ch, cl = empty(m, n), empty(m, n)
    assert sr.sr_ozaki_zgemm_dd(dev(a), None, dev(b), None, ch, cl, slices_a=4, slices_b=4, dmax=8,
                                Cin_hi=dev(c0)) == 0
    # exact result (|entries| < 2^47) is representable: hi holds it, lo is 0
    exact = c0 + a @ b
    assert np.array_equal(host(ch), exact) and not host(cl).any()


@pytest.mark.parametrize("n", [2, 33, 100, 200])
def test_trisolve64_matches_exact_solution(sr, n):
    rng = np.random.default_rng(500 + n)
    g = synth.schur_test_matrix(n, seed=500 + n)
    t = np.asfortranarray(np.triu(g["T0"]))
    e = np.asfortranarray(1e-12 * np.tril(rand_c(rng, (n, n)), -1))
    l = empty(n, n)
    assert sr.sr_trisolve64(dev(t), dev(e), l, sr.workspace(n)) == 0
    lg = host(l)
    assert not np.triu(lg).any()
    lx = oracle.trisolve(t, e, lp="quad")[0].to_c128()
    ld = oracle.trisolve(t, e, lp="double")[0].to_c128()  # Algorithm 2 in FP64
    assert np.linalg.norm(lg - lx) <= 10 * np.linalg.norm(ld - lx) + 10 * U64 * np.linalg.norm(lx)


def _phase_aligned_diff(ah, al, bh, bl) -> float:
    """max over columns j of ||a_j d_j - b_j||, d_j the unimodular phase that
    matches a_j to b_j at the largest entry of b_j, all in decimal arithmetic."""
    from decimal import Decimal, getcontext

    getcontext().prec = 40
    D = lambda h, l: Decimal(float(h)) + Decimal(float(l))
    worst = Decimal(0)
    for j in range(ah.shape[1]):
        r = int(np.argmax(np.abs(bh[:, j])))
        ar, ai = D(ah[r, j].real, al[r, j].real), D(ah[r, j].imag, al[r, j].imag)
        br, bi = D(bh[r, j].real, bl[r, j].real), D(bh[r, j].imag, bl[r, j].imag)
        # d = (b / a) / |b / a| = b conj(a) / |b conj(a)|
        zr, zi = br * ar + bi * ai, bi * ar - br * ai
        m = (zr * zr + zi * zi).sqrt()
        dr, di = zr / m, zi / m
        s = Decimal(0)
        for i in range(ah.shape[0]):
            xr, xi = D(ah[i, j].real, al[i, j].real), D(ah[i, j].imag, al[i, j].imag)
            yr, yi = D(bh[i, j].real, bl[i, j].real), D(bh[i, j].imag, bl[i, j].imag)
            er, ei = xr * dr - xi * di - yr, xr * di + xi * dr - yi
            s += er * er + ei * ei
        worst = max(worst, s.sqrt())
    return float(worst)


def _refine_dd(sr, ah, al, qh, ql, iters=8, tol=1e-28, **kw):
    n = ah.shape[0]
    qhd, qld = dev(qh), dev(ql)
    th, tl = empty(n, n), empty(n, n)
    info = sr.schur_refine_dd(dev(ah), dev(al), qhd, qld, th, tl, iters=iters, tol=tol, **kw)
    return host(qhd), host(qld), host(th), host(tl), info


def test_dd_refine_n64_against_oracle(sr):
    g = synth.schur_test_matrix(64, seed=0)
    a = g["A"]
    al = np.zeros_like(a)
    qh = synth.hp_schur_start(a)
    q_hi, q_lo, t_hi, t_lo, info = _refine_dd(sr, a, al, qh, np.zeros_like(qh))
    assert info["status"] == "OK" and info["iters"] <= 4, info
    ev = oracle.evaluate(oracle.QMat.from_dd(a), oracle.QMat.from_dd(q_hi, q_lo),
                         oracle.QMat.from_dd(t_hi, t_lo))
    assert ev["stril"] <= 1e-28 and ev["orth"] <= 1e-26 and ev["tdiff"] <= 1e-26 * ev["normA"], ev
    # (double lp, quad hp) oracle mirrors the iteration
    ref = oracle.refine(a, qh, lp="double", maxit=8, tol=1e-28)
    for k, (eg, eo) in enumerate(zip(info["resid_hist"], ref["hist"])):
        if eo > 1e-27:
            assert 0.1 * eo <= eg <= 10 * eo, (k, eg, eo)
    # Schur vectors agree with the quad ground truth up to column phases, aligned
    # in 40-digit decimal arithmetic (a double-precision phase is too coarse)
    qq = oracle.refine(a, qh, lp="quad", maxit=8, tol=1e-32)["Q"]
    qqh, qql = qq.to_dd()
    assert _phase_aligned_diff(q_hi, q_lo, qqh, qql) <= 1e-25


@pytest.mark.parametrize("n", [1, 17, 130])
def test_dd_refine_ragged_and_float_start(sr, n):
    g = synth.schur_test_matrix(n, seed=70 + n)
    a = g["A"]
    qh = synth.lp_schur_start(a)  # a complex64 start still converges, in more passes
    q_hi, q_lo, t_hi, t_lo, info = _refine_dd(sr, a, np.zeros_like(a), qh, np.zeros_like(qh))
    assert info["status"] == "OK", info
    ev = oracle.evaluate(oracle.QMat.from_dd(a), oracle.QMat.from_dd(q_hi, q_lo),
                         oracle.QMat.from_dd(t_hi, t_lo))
    assert ev["stril"] <= 1e-28 and ev["orth"] <= 1e-26, ev


def _table1():
    rows = {}
    with open(os.path.join(GOLDEN, "wilkinson20_table1.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                r = [float(x) for x in line.split()]
                rows[int(r[0])] = r[1:]
    return rows


def test_dd_wilkinson20_table1(sr):
    """Example 1: the companion matrix of prod (x - i), i = 1..20, stored exactly as
    double-double, refined from its double-precision Schur form. The eigenvalue
    errors must be of the order of the paper's Algorithm 4 columns."""
    table = _table1()
    hi, lo, exact = synth.wilkinson_companion_dd(20)
    qh = synth.hp_schur_start(hi)
    # the first row holds the coefficients (up to 20! ~ 2^61) and the other rows
    # ones: 23 digits per operand keep the small entries of P = A Q to 2^-106 (the
    # updates Q Delta take the same count by default)
    # The normwise residual of the double-precision start is already below 1e-28
    # (the entries span 1 .. 20!, and ||A||_F ~ 2e19 is carried by the first row),
    # while the ill-conditioned eigenvalues are far from their double-double values:
    # the strict rule also waits for an update whose correction is negligible to
    # second order (||W||^2 <= 2^-104).
    _, _, _, _, info_n = _refine_dd(sr, hi, lo, qh, np.zeros_like(qh), iters=8, tol=1e-28, slices=23)
    q_hi, q_lo, t_hi, t_lo, info = _refine_dd(sr, hi, lo, qh, np.zeros_like(qh), iters=8, tol=1e-28,
                                              slices=23, strict_stop=True)
    assert info_n["status"] == "OK" and info_n["iters"] <= 2, info_n
    assert info["status"] == "OK" and info_n["iters"] < info["iters"] <= 7, info
    assert info["norm_w_hist"][info["updates"] - 1] ** 2 <= UDD, info
    errs = {}
    for i in range(20):
        re = Fraction(t_hi[i, i].real) + Fraction(t_lo[i, i].real)
        im = Fraction(t_hi[i, i].imag) + Fraction(t_lo[i, i].imag)
        k = int(round(float(re)))
        errs[k] = abs(complex(float(re - k), float(im)))
    assert sorted(errs) == list(range(1, 21))
    worst_paper = max(abs(r[3]) for r in table.values())  # the 2-double Algorithm 4 column
    for k, err in errs.items():
        assert err <= max(10 * abs(table[k][3]), 1e-27), (k, err, table[k])
    assert max(errs.values()) <= 10 * worst_paper


def test_dd_continuation_warm_start(sr):
    """Two steps of the continuation A(t) = A0 + t A1 at a reduced size: the second
    matrix is warm-started from the refined Schur form of the first."""
    n = 96
    g = synth.schur_test_matrix(n, seed=12)
    a1 = synth.continuation_perturbation(n, seed=13)
    ah0, al0 = synth.continuation_step_dd(g["A"], a1, 0)
    q0 = synth.hp_schur_start(g["A"])
    q_hi, q_lo, _, _, i0 = _refine_dd(sr, ah0, al0, q0, np.zeros_like(q0))
    assert i0["status"] == "OK", i0
    ah1, al1 = synth.continuation_step_dd(g["A"], a1, 1)
    q_hi1, q_lo1, t_hi1, t_lo1, i1 = _refine_dd(sr, ah1, al1, q_hi, q_lo, update_slices=-1)
    assert i1["status"] == "OK" and i1["iters"] <= 5, i1
    ev = oracle.evaluate(oracle.QMat.from_dd(ah1, al1), oracle.QMat.from_dd(q_hi1, q_lo1),
                         oracle.QMat.from_dd(t_hi1, t_lo1))
    assert ev["stril"] <= 1e-28, ev


def test_dd_continuation_config4_n2048(sr):
    """The double-double continuation at its full size for three steps: A(t_k) =
    A0 + (k/64) A1, n = 2048 (A0 seed 4, A1 = 1e-3 CN(0,1) seed 5, both exact in
    double-double), the first step from the zgees Schur form of A0, the next two
    warm-started from the refined Q of the step before (digits of Q Delta from
    ||Delta||). Each step reaches 1e-28 within 5 passes and its binary128 residual
    and orthogonality on 8 sampled rows meet the tier's targets."""
    n = 2048
    g = synth.schur_test_matrix(n, seed=4, gap=0.05)
    a1 = synth.continuation_perturbation(n, seed=5)
    q0 = synth.hp_schur_start(g["A"])
    ws = sr.workspace_dd(n, update_slices=-1)
    qh, ql = dev(q0), dev(np.zeros_like(q0))
    th, tl = empty(n, n), empty(n, n)
    rows = np.random.default_rng(9).choice(n, 8, replace=False)
    for k in range(3):
        ah, al = synth.continuation_step_dd(g["A"], a1, k)
        info = sr.schur_refine_dd(dev(ah), dev(al), qh, ql, th, tl, iters=8, tol=1e-28, workspace=ws,
                                  update_slices=-1)
        assert info["status"] == "OK" and info["iters"] <= 5, (k, info)
        ev = oracle.evaluate_rows(oracle.QMat.from_dd(ah, al), oracle.QMat.from_dd(host(qh), host(ql)), rows)
        assert ev["stril"] <= 1e-28 and ev["stril_rowmax"] <= 1e-28, (k, ev)
        assert ev["orth"] <= 4 * UDD * np.sqrt(n), (k, ev)


def test_dd_validation(sr):
    a = np.eye(8, dtype=np.complex128)
    q, t = dev(a), empty(8, 8)
    z = dev(np.zeros_like(a))
    assert sr.schur_refine_dd(dev(a), z, q, dev(np.zeros_like(a)), t, empty(8, 8), slices=33)["rc"] == -1
    assert sr.schur_refine_dd(dev(a), z, q, dev(np.zeros_like(a)), t, empty(8, 8), iters=0)["rc"] == -1


# Outputs with a 64 x 64 tile per CU and the tier's digit sets (S digits per
# operand, pairs up to s + t = S + 1) take the windowed kernel: 4 x 4 windows of
# slices, a three-term FP64 expansion per output between windows.

def _ints(rng, shape, lim):
    return np.asfortranarray(rng.integers(-lim, lim + 1, shape) + 1j * rng.integers(-lim, lim + 1, shape))


@pytest.mark.parametrize("add", [False, True])
@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("S", [2, 6, 14])
def test_dd_windows_exact_on_integers(sr, S, opa, add):
    # op(A) of 9-bit integers (two digits), B of 6-bit ones (one digit): the pairs
    # (s, 1), s <= 2, give the exact product, which FP64 holds (lo = 0)
    m, n, k = 2085, 2048, 130  # ragged rows, a ragged K-tile
    rng = np.random.default_rng(900 + 10 * S + 2 * opa + add)
    a = _ints(rng, (k, m) if opa else (m, k), 256)
    b = _ints(rng, (k, n), 63)
    c0 = _ints(rng, (m, n), 2**30) if add else None
    ch, cl = empty(m, n), empty(m, n)
    assert sr.sr_ozaki_zgemm_dd(dev(a), None, dev(b), None, ch, cl, opa=opa, slices_a=S, slices_b=S, dmax=S + 1,
                                Cin_hi=dev(c0) if add else None) == 0
    exact = (a.conj().T if opa else a) @ b
    if add:
        exact = exact + c0
    assert np.array_equal(host(ch), exact) and not host(cl).any()


@pytest.mark.parametrize("opa", [0, 1])
def test_dd_windows_matches_quad(sr, opa):
    m = n = 2048
    k = 192
    rng = np.random.default_rng(77 + opa)
    ah, al = _dd_rand(rng, (k, m) if opa else (m, k))
    bh, bl = _dd_rand(rng, (k, n))
    ch, cl = empty(m, n), empty(m, n)
    assert sr.sr_ozaki_zgemm_dd(dev(ah), dev(al), dev(bh), dev(bl), ch, cl, opa=opa,
                                slices_a=14, slices_b=14, dmax=15) == 0
    rows = np.random.default_rng(5).choice(m, 24, replace=False)
    sub_h = np.asfortranarray(ah[:, rows] if opa else ah[rows])
    sub_l = np.asfortranarray(al[:, rows] if opa else al[rows])
    ref = oracle.gemm(oracle.QMat.from_dd(sub_h, sub_l), oracle.QMat.from_dd(bh, bl), opa=opa)
    err = _dd_err(host(ch)[rows], host(cl)[rows], ref)
    aa = np.abs(sub_h.conj().T if opa else sub_h)
    bound = 4 * (k + 4) * UDD * np.sqrt(2.0) * (aa @ np.abs(bh))
    assert np.all(err <= bound), (err / np.maximum(bound, 1e-300)).max()


def test_dd_refine_n1024_windows(sr):
    """n = 1024: every double-double product takes the windowed kernel."""
    g = synth.schur_test_matrix(1024, seed=12)
    a = g["A"]
    qh = synth.hp_schur_start(a)
    q_hi, q_lo, _, _, info = _refine_dd(sr, a, np.zeros_like(a), qh, np.zeros_like(qh))
    assert info["status"] == "OK" and info["iters"] <= 4, info
    rows = np.random.default_rng(31).choice(1024, 24, replace=False)
    ev = oracle.evaluate_rows(oracle.QMat.from_dd(a), oracle.QMat.from_dd(q_hi, q_lo), rows)
    assert ev["stril"] <= 1e-28 and ev["orth"] <= 1e-26, ev
