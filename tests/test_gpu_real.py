"""The real Schur variant on the GPU (schur_refine_real and its stages through the
C interface) against the binary128 oracle: real FP64 products, the FP32 block solve
and the refinement of a real quasi-triangular Schur form."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import U32, U64
from real_util import block_lower_mask, block_sizes, exact_real_problem, quasi_upper, rotated

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sr():
    import torch

    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def dev(x, dtype=np.float64):
    import paper_2203_10879_amd as m

    return m.colmajor(np.asfortranarray(np.asarray(x, dtype=dtype)))


def host(t):
    import paper_2203_10879_amd as m

    return m.to_numpy(t)


def empty(m, n, f32=False):
    import torch

    import paper_2203_10879_amd as sr

    return sr.colmajor_empty(m, n, torch.float32 if f32 else torch.float64)


def quad_real(q):
    """(hi, lo) real parts of an oracle QMat."""
    hi, lo = q.to_dd()
    assert not hi.imag.any()
    return hi.real, lo.real


# ------------------------------------------------------------------ products

@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("comp", [False, True])
@pytest.mark.parametrize("shape", [(130, 97, 75), (64, 64, 64), (1, 1, 1), (5, 200, 33)])
def test_dgemm_exact_on_integers(sr, opa, comp, shape):
    m, n, k = shape
    rng = np.random.default_rng(m * 1000 + n + k + 7)
    a = rng.integers(-4096, 4097, (k, m) if opa else (m, k)).astype(np.float64)
    b = rng.integers(-4096, 4097, (k, n)).astype(np.float64)
    c = empty(m, n)
    assert sr.sr_dgemm(dev(a), dev(b), c, opa=opa, compensated=comp) == 0
    ref = (a.T if opa else a) @ b  # every partial sum is an integer below 2^53
    assert np.array_equal(host(c), ref)


@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("comp", [False, True])
def test_dgemm_random_within_bound_of_quad(sr, opa, comp):
    rng = np.random.default_rng(17 + opa)
    m, n, k = 150, 131, 260
    a = rng.standard_normal((k, m) if opa else (m, k))
    b = rng.standard_normal((k, n))
    c = empty(m, n)
    assert sr.sr_dgemm(dev(a), dev(b), c, opa=opa, compensated=comp) == 0
    chi, clo = quad_real(oracle.gemm(a.astype(complex), b.astype(complex), opa=opa))
    err = np.abs((host(c) - chi) - clo)
    aa = np.abs(a.T if opa else a)
    assert np.all(err <= (k + 4) * U64 * (aa @ np.abs(b)))
    assert np.linalg.norm(err) <= 4 * U64 * np.sqrt(k) * np.linalg.norm(aa @ np.abs(b))


def test_dgemm_two_level_sum_is_more_accurate(sr):
    """The two-level (chunked) accumulation of the compensated form lowers the error
    of long dot products (k = 1024) against the binary128 product."""
    rng = np.random.default_rng(12)
    n = 1024
    a = rng.standard_normal((n, n))
    b = rng.standard_normal((n, 64))
    chi, clo = quad_real(oracle.gemm(a.astype(complex), b.astype(complex)))
    errs = []
    for comp in (False, True):
        c = empty(n, 64)
        assert sr.sr_dgemm(dev(a), dev(b), c, compensated=comp) == 0
        errs.append(np.linalg.norm((host(c) - chi) - clo))
    assert errs[1] < 0.7 * errs[0], errs


@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("comp", [False, True])
def test_dgemm_large_tile_exact_on_integers(sr, opa, comp):
    """Products with at least one 128 x 128 tile per CU take the large-tile kernel:
    bit-exact on integers (ragged M), and with an added C."""
    m, n, k = 2048 + 37, 2048, 300
    rng = np.random.default_rng(90 + opa + 2 * comp)
    a = rng.integers(-4096, 4097, (k, m) if opa else (m, k)).astype(np.float64)
    b = rng.integers(-4096, 4097, (k, n)).astype(np.float64)
    c0 = rng.integers(-2**20, 2**20, (m, n)).astype(np.float64)
    c = empty(m, n)
    assert sr.sr_dgemm(dev(a), dev(b), c, opa=opa, compensated=comp) == 0
    ref = (a.T if opa else a) @ b
    assert np.array_equal(host(c), ref)
    assert sr.sr_dgemm(dev(a), dev(b), c, opa=opa, Cin=dev(c0), compensated=comp) == 0
    assert np.array_equal(host(c), ref + c0)


def test_dgemm_add_epilogue(sr):
    rng = np.random.default_rng(3)
    m, n, k = 70, 90, 40
    a, b, c0 = rng.standard_normal((m, k)), rng.standard_normal((k, n)), rng.standard_normal((m, n))
    c = empty(m, n)
    assert sr.sr_dgemm(dev(a), dev(b), c, Cin=dev(c0), compensated=True) == 0
    chi, clo = quad_real(oracle.gemm(a.astype(complex), b.astype(complex)))
    ref = c0 + chi + clo
    assert np.abs(host(c) - ref).max() <= 4 * U64 * np.abs(ref).max()


# ------------------------------------------------------------------ block solve

def _solve_case(n, seed, scale=1e-6, pair_frac=0.5):
    rng = np.random.default_rng(seed)
    sizes = []
    while sum(sizes) < n:
        sizes.append(2 if sum(sizes) + 2 <= n and rng.random() < pair_frac else 1)
    t, blk = quasi_upper(rng, sizes)
    t = (t / np.sqrt(n)).astype(np.float32)
    mask = block_lower_mask(n, blk)
    e = np.where(mask, scale * rng.standard_normal((n, n)), 0.0).astype(np.float32)
    return np.asfortranarray(t), np.asfortranarray(e), blk, mask


@pytest.mark.parametrize("n", [2, 3, 31, 33, 64, 65, 130, 300])
def test_trisolve_real_matches_exact_solution(sr, n):
    """The FP32 block solve against the exact (binary128) solution of the same FP32
    data: block strictly lower, the forward error within 10x that of the oracle's
    FP32 block solve, and a small normwise residual of the defining equation."""
    t, e, blk, mask = _solve_case(n, 400 + n)
    l = empty(n, n, f32=True)
    assert sr.sr_trisolve_real(dev(t, np.float32), dev(e, np.float32), l, blk) == 0
    lg = host(l).astype(np.float64)
    assert not lg[~mask].any()
    t64, e64 = t.astype(np.float64), e.astype(np.float64)
    lx = oracle.trisolve_real(t64.astype(complex), e64.astype(complex), blk, lp="quad")[0].to_c128().real
    lf = oracle.trisolve_real(t64.astype(complex), e64.astype(complex), blk, lp="float")[0].to_c128().real
    err_gpu = np.linalg.norm(lg - lx)
    err_ref = np.linalg.norm(lf - lx)
    assert err_gpu <= 10 * err_ref + 10 * U32 * np.linalg.norm(lx), (err_gpu, err_ref)
    # block by block, the backward error of a correct FP32 solve: the solve runs in the
    # basis of the 2 x 2 unitaries, which mixes the rows (columns) of a block, so each
    # block (I, J) of the residual R = block-stril(T L - L T) + E is bounded by its
    # largest entry of sqrt(2)(n + 8) u (|T||L| + |L||T| + |E|)
    r = np.abs(np.where(mask, t64 @ lg - lg @ t64 + e64, 0.0))
    b = np.sqrt(2) * (n + 8) * U32 * (np.abs(t64) @ np.abs(lg) + np.abs(lg) @ np.abs(t64) + np.abs(e64))
    for i, p in block_sizes(blk):
        for j, q in block_sizes(blk):
            if i > j:
                assert r[i:i + p, j:j + q].max() <= b[i:i + p, j:j + q].max(), (i, j)


def test_trisolve_real_without_blocks_is_the_complex_solve(sr):
    """With no 2 x 2 block the unitary transform is the identity and the block solve
    is the complex FP32 sweep on real data: bit for bit the real part of sr_trisolve."""
    n = 97
    t, e, blk, _ = _solve_case(n, 11, pair_frac=0.0)
    assert not blk.any()
    l = empty(n, n, f32=True)
    assert sr.sr_trisolve_real(dev(t, np.float32), dev(e, np.float32), l, None) == 0
    import torch

    lc = sr.colmajor_empty(n, n, torch.complex64)
    tc, ec = dev(t.astype(np.complex64), np.complex64), dev(e.astype(np.complex64), np.complex64)
    assert sr.sr_trisolve(tc, ec, lc, sr.workspace(n)) == 0
    lcc = host(lc)
    assert not lcc.imag.any()
    assert np.array_equal(host(l), lcc.real)


def test_trisolve_real_breakdown_and_invalid_markers(sr):
    rng = np.random.default_rng(21)
    t, blk = quasi_upper(rng, [2, 1, 2])
    t[3:, 3:] = t[:2, :2]  # two blocks with the same pair of eigenvalues
    n = 5
    e = np.where(block_lower_mask(n, blk), 1e-3, 0.0)
    l = empty(n, n, f32=True)
    assert sr.sr_trisolve_real(dev(t, np.float32), dev(e, np.float32), l, blk) == 3  # SR_BREAKDOWN
    bad = np.array([1, 1, 0, 0, 0], dtype=np.int32)  # overlapping blocks
    assert sr.sr_trisolve_real(dev(t, np.float32), dev(e, np.float32), l, bad) == -1
    last = np.array([0, 0, 0, 0, 1], dtype=np.int32)  # a block at the last row
    assert sr.sr_trisolve_real(dev(t, np.float32), dev(e, np.float32), l, last) == -1


# ------------------------------------------------------------------ refinement

def _refine_real(sr, a, qh, blk, iters=6, tol=1e-15, **kw):
    n = a.shape[0]
    q, t = dev(qh), empty(n, n)
    info = sr.schur_refine_real(dev(a), q, t, blk, iters=iters, tol=tol, **kw)
    return host(q), host(t), info


def _block_eigs(t, blk):
    lam = []
    for i, s in block_sizes(blk):
        lam += list(np.linalg.eigvals(t[i:i + s, i:i + s]))
    return np.array(lam)


@pytest.mark.parametrize("n", [16, 64, 256])
def test_exact_walsh_hadamard_real_schur_form(sr, n):
    """A = Q0 T0 Q0^T exact in binary, started from Q0 rotated by 1e-6: every diagonal
    block's invariant subspace and eigenvalues are recovered to FP64 accuracy."""
    a, q0, t0, blk = exact_real_problem(n, n + 3)
    qh = rotated(q0, 1, 1e-6)
    q, t, info = _refine_real(sr, a, qh, blk)
    assert info["status"] == "OK" and info["iters"] <= 4, info
    assert not t[block_lower_mask(n, blk)].any()
    c = q0.T @ q
    for i, s in block_sizes(blk):
        off = np.delete(c[:, i:i + s], np.s_[i:i + s], axis=0)
        assert np.abs(off).max() <= 1e-13, (i, np.abs(off).max())
        d = np.sort_complex(np.linalg.eigvals(t[i:i + s, i:i + s])) - np.sort_complex(
            np.linalg.eigvals(t0[i:i + s, i:i + s]))
        assert np.abs(d).max() <= 1e-13


def test_n48_sgees_start_against_oracle_mirror(sr):
    """n = 48 from the real Schur vectors of float32(A) (LAPACK sgees): the FP64 tier
    reaches 1e-15; each pass's residual tracks the (float lp, quad hp) oracle above
    the FP64 floor; Q matches the oracle's binary128 fixed point block by block."""
    g = synth.real_schur_test_matrix(48, seed=11)
    qh, blk = synth.lp_real_schur_start(g["A"])
    q, t, info = _refine_real(sr, g["A"], qh, blk)
    assert info["status"] == "OK" and info["iters"] <= 5, info
    assert info["hp_gemms"] == 4 * info["iters"]
    ev = oracle.evaluate_real(g["A"].astype(complex), q.astype(complex), t.astype(complex), blk)
    assert ev["stril"] <= 1e-15 and ev["orth"] <= 1e-13 and ev["tdiff"] <= 1e-13 * ev["normA"], ev
    ref = oracle.refine_real(g["A"].astype(complex), qh.astype(complex), blk, lp="float", maxit=6, tol=1e-15)
    for k, (eg, eo) in enumerate(zip(info["resid_hist"], ref["hist"])):
        if eo > 1e-14:
            assert 0.1 * eo <= eg <= 10 * eo, (k, eg, eo)
    qq = oracle.refine_real(g["A"].astype(complex), qh.astype(complex), blk, lp="quad", maxit=8,
                            tol=1e-30)["Q"].to_c128().real
    # the real Schur vectors are unique up to an orthogonal map within each block
    # (a sign for a 1 x 1 block): compare the projectors onto each block's columns
    for i, s in block_sizes(blk):
        pg = q[:, i:i + s] @ q[:, i:i + s].T
        pq = qq[:, i:i + s] @ qq[:, i:i + s].T
        assert np.abs(pg - pq).max() <= 1e-13, i
    lam = _block_eigs(t, blk)
    assert np.abs(np.sort_complex(lam) - np.sort_complex(g["lam"])).max() <= 1e-12


@pytest.mark.parametrize("n", [1, 2, 3, 17, 100, 257])
def test_ragged_sizes_converge(sr, n):
    g = synth.real_schur_test_matrix(n, seed=70 + n)
    qh, blk = synth.lp_real_schur_start(g["A"])
    q, t, info = _refine_real(sr, g["A"], qh, blk)
    assert info["status"] == "OK", info
    ev = oracle.evaluate_real(g["A"].astype(complex), q.astype(complex), t.astype(complex), blk)
    assert ev["stril"] <= 1e-15 and ev["orth"] <= 1e-12, ev


def test_n1024_quad_rows(sr):
    """n = 1024 real matrix with complex pairs (about half), the sgees start: at most 5
    passes to 1e-15; binary128 residual (block strictly lower entries) and
    orthogonality on 32 sampled rows of Q^T A Q and Q^T Q."""
    n = 1024
    g = synth.real_schur_test_matrix(n, seed=12)
    a = g["A"]
    qh, blk = synth.lp_real_schur_start(a)
    assert blk.sum() > 100
    q, t, info = _refine_real(sr, a, qh, blk, timing=True)
    assert info["status"] == "OK" and info["iters"] <= 5, info
    rows = np.sort(np.random.default_rng(20003).choice(n, 32, replace=False))
    qr = np.asfortranarray(q[:, rows]).astype(complex)
    ra_hi, ra_lo = oracle.gemm(qr, a.astype(complex), opa=1).to_dd()  # Q_r^T A (quad, rounded to dd)
    # (Q_r^T A) Q, the double-double left operand taken as two FP64 products in quad
    m_hi, m_lo = oracle.gemm(np.asfortranarray(ra_hi), q.astype(complex)).to_dd()
    m2_hi, m2_lo = oracle.gemm(np.asfortranarray(ra_lo), q.astype(complex)).to_dd()
    m = (m_hi.real + m2_hi.real) + (m_lo.real + m2_lo.real)
    mask = block_lower_mask(n, blk)[rows]
    na = np.linalg.norm(a)
    stril = np.sqrt(np.sum(m[mask] ** 2) * n / len(rows)) / na
    assert stril <= 1e-15, stril
    o_hi, o_lo = oracle.gemm(qr, q.astype(complex), opa=1).to_dd()
    o = o_hi.real.copy()
    o[np.arange(len(rows)), rows] -= 1.0
    o += o_lo.real
    orth = np.sqrt(np.sum(o ** 2) * n / len(rows))
    assert orth <= 4 * U64 * np.sqrt(n) * 10, orth
    # T is the block upper part of Q^T A Q: on the sampled rows, within FP64 rounding
    tt = np.where(mask, 0.0, m)
    assert np.abs(t[rows] - tt).max() <= 1e-13 * na
    lam = _block_eigs(t, blk)
    assert np.abs(np.sort_complex(lam) - np.sort_complex(g["lam"])).max() <= 1e-10


def test_n2048_large_tiles_quad_rows(sr):
    """n = 2048 (the real benchmark size: every FP64 product on the 128 x 128 tile
    kernel, the symmetric Y over its upper tiles): at most 5 passes to 1e-15 and the
    binary128 residual and orthogonality on 16 sampled rows."""
    n = 2048
    g = synth.real_schur_test_matrix(n, seed=3)
    a = g["A"]
    qh, blk = synth.lp_real_schur_start(a)
    q, t, info = _refine_real(sr, a, qh, blk)
    assert info["status"] == "OK" and info["iters"] <= 5, info
    rows = np.sort(np.random.default_rng(20004).choice(n, 16, replace=False))
    qr = np.asfortranarray(q[:, rows]).astype(complex)
    ra_hi, ra_lo = oracle.gemm(qr, a.astype(complex), opa=1).to_dd()
    m_hi, m_lo = oracle.gemm(np.asfortranarray(ra_hi), q.astype(complex)).to_dd()
    m2_hi, m2_lo = oracle.gemm(np.asfortranarray(ra_lo), q.astype(complex)).to_dd()
    m = (m_hi.real + m2_hi.real) + (m_lo.real + m2_lo.real)
    mask = block_lower_mask(n, blk)[rows]
    stril = np.sqrt(np.sum(m[mask] ** 2) * n / len(rows)) / np.linalg.norm(a)
    assert stril <= 1e-15, stril
    o_hi, o_lo = oracle.gemm(qr, q.astype(complex), opa=1).to_dd()
    o = o_hi.real.copy()
    o[np.arange(len(rows)), rows] -= 1.0
    o += o_lo.real
    assert np.sqrt(np.sum(o ** 2) * n / len(rows)) <= 4 * U64 * np.sqrt(n) * 10
    assert np.abs(t[rows] - np.where(mask, 0.0, m)).max() <= 1e-13 * np.linalg.norm(a)


def test_real_status_codes(sr):
    g = synth.real_schur_test_matrix(24, seed=31)
    qh, blk = synth.lp_real_schur_start(g["A"])
    a = dev(g["A"])
    q, t = dev(qh), empty(24, 24)
    assert sr.schur_refine_real(a, q, t, blk, gemm="ozaki_i8")["rc"] == -4  # SR_ENOSYS
    bad = blk.copy()
    bad[-1] = 1
    assert sr.schur_refine_real(a, q, t, bad)["rc"] == -1  # SR_EINVAL
    info = sr.schur_refine_real(a, q, t, blk, iters=1)
    assert info["rc"] == 1 and info["iters"] == 1  # SR_NOT_CONVERGED: one evaluation only
