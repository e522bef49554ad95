"""GPU parity of each step of a refinement pass against the CPU oracle, through
the C interface (include/schur_refine.h)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import U32, U64, dev, empty, gemm_bound, host, rand_c

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sr():
    import torch

    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


@pytest.mark.parametrize("kind", [0, 1])
def test_mfma_operand_layout(sr, kind):
    rng = np.random.default_rng(kind)
    a = rng.integers(-9, 10, (16, 4)).astype(np.float64)
    b = rng.integers(-9, 10, (4, 16)).astype(np.float64)
    d = sr.sr_diag_mfma(a, b, kind=kind)
    assert np.array_equal(d, a @ b)


def _gauss_int(rng, shape, lim=256):
    return np.asfortranarray(rng.integers(-lim, lim + 1, shape) + 1j * rng.integers(-lim, lim + 1, shape))


@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("comp", [False, True])
@pytest.mark.parametrize("shape", [(130, 97, 75), (64, 64, 64), (1, 1, 1), (5, 200, 33)])
def test_zgemm_exact_on_integers(sr, opa, comp, shape):
    m, n, k = shape
    rng = np.random.default_rng(m * 1000 + n + k)
    a = _gauss_int(rng, (k, m) if opa else (m, k))
    b = _gauss_int(rng, (k, n))
    c = empty(m, n)
    assert sr.sr_zgemm(dev(a), dev(b), c, opa=opa, compensated=comp) == 0
    ref = (a.conj().T if opa else a) @ b  # every partial sum is an integer below 2^53
    assert np.array_equal(host(c), ref)


@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("comp", [False, True])
def test_zgemm_random_within_bound_of_quad(sr, opa, comp):
    rng = np.random.default_rng(7 + opa)
    m, n, k = 150, 131, 260
    a = rand_c(rng, (k, m) if opa else (m, k))
    b = rand_c(rng, (k, n))
    c = empty(m, n)
    assert sr.sr_zgemm(dev(a), dev(b), c, opa=opa, compensated=comp) == 0
    chi, clo = oracle.gemm(a, b, opa=opa).to_dd()
    err = np.abs((host(c) - chi) - clo)
    aa = np.abs(a.conj().T if opa else a)
    assert np.all(err <= gemm_bound(aa, np.abs(b), k, U64))
    # typical error: u * sqrt(k) relative to the entries
    assert np.linalg.norm(err) <= 4 * U64 * np.sqrt(k) * np.linalg.norm(aa @ np.abs(b))


def test_zgemm_compensated_is_more_accurate(sr):
    rng = np.random.default_rng(12)
    n = 1024
    a = rand_c(rng, (n, n))
    b = rand_c(rng, (n, 64))
    chi, clo = oracle.gemm(a, b).to_dd()
    errs = []
    for comp in (False, True):
        c = empty(n, 64)
        assert sr.sr_zgemm(dev(a), dev(b), c, compensated=comp) == 0
        errs.append(np.linalg.norm((host(c) - chi) - clo))
    assert errs[1] < 0.7 * errs[0]


def test_zgemm_add_epilogue(sr):
    rng = np.random.default_rng(3)
    m, n, k = 70, 90, 40
    a, b, c0 = _gauss_int(rng, (m, k)), _gauss_int(rng, (k, n)), _gauss_int(rng, (m, n))
    c = empty(m, n)
    assert sr.sr_zgemm(dev(a), dev(b), c, Cin=dev(c0)) == 0
    assert np.array_equal(host(c), c0 + a @ b)


def test_cgemm_fp32_within_bound(sr):
    import torch

    rng = np.random.default_rng(5)
    m, n, k = 100, 77, 129
    a = rand_c(rng, (m, k)).astype(np.complex64)
    b = rand_c(rng, (k, n)).astype(np.complex64)
    c = empty(m, n, c64=True)
    assert sr.sr_cgemm(dev(a), dev(b), c) == 0
    ref = a.astype(np.complex128) @ b.astype(np.complex128)
    err = np.abs(host(c).astype(np.complex128) - ref)
    assert np.all(err <= gemm_bound(np.abs(a).astype(np.float64), np.abs(b).astype(np.float64), k, U32))
    assert host(c).dtype == np.complex64 and torch.cuda.is_available()


@pytest.mark.parametrize("n", [64, 200])
def test_residual_split_matches_quad(sr, n):
    g = synth.schur_test_matrix(n, seed=n)
    a = g["A"]
    q = synth.lp_schur_start(a)
    ws = sr.workspace(n)
    t, tlp, elp = empty(n, n), empty(n, n, True), empty(n, n, True)
    rc, eps = sr.sr_residual(dev(a), dev(q), t, tlp, elp, ws)
    assert rc == 0
    aq = oracle.gemm(a, q)
    th_hi, th_lo = oracle.gemm(q, aq, opa=1).to_dd()
    th = th_hi + th_lo
    # T = triu(That) to FP64 accuracy, zero below
    tg = host(t)
    bound = 2 * gemm_bound(np.abs(q).T, np.abs(a) @ np.abs(q), n, U64)
    assert np.all(np.abs(np.triu(tg) - np.triu(th)) <= np.triu(bound))
    assert not np.tril(tg, -1).any()
    # lp copies are the FP32 roundings of the split (up to one FP64 error)
    tl, el = host(tlp), host(elp)
    assert not np.tril(tl, -1).any() and not np.triu(el).any()
    # E_lp is the FP32 rounding of the FP64 stril(That): per entry at most one FP32
    # rounding of the exact value plus the FP64 product bound (carried through it)
    e_exact = np.tril(th, -1)
    lower = np.tril(np.ones((n, n), dtype=bool), -1)
    e_err = np.abs(el.astype(np.complex128) - e_exact)
    e_bound = np.sqrt(2) * U32 * np.abs(e_exact) + (1 + 2 * U32) * bound
    assert np.all(e_err[lower] <= e_bound[lower])
    t_err = np.abs(tl.astype(np.complex128) - np.triu(th))
    t_bound = np.sqrt(2) * U32 * np.abs(np.triu(th)) + (1 + 2 * U32) * bound
    upper = np.triu(np.ones((n, n), dtype=bool))
    assert np.all(t_err[upper] <= t_bound[upper])
    ev = oracle.evaluate(a, q)
    assert abs(eps - ev["stril"]) <= 1e-6 * ev["stril"]


def _residual_entrywise_ok(t, e, lg, u):
    """Componentwise backward error of a substitution solve of the equation
    stril(T L - L T) = -E (eq. (7)): every entry (i, j), i > j, of the residual
    R = stril(T L - L T) + E satisfies |r_ij| <= c u (|T||L| + |L||T|)_ij + u |e_ij|
    with c = sqrt(2)(n + 8) (dot products of at most n terms in any summation order,
    complex products, the division), for a correct solve in precision u. Returns the
    largest ratio |r_ij| / bound_ij (evaluated in FP64, far below u32 / u64 bounds)."""
    n = t.shape[0]
    lower = np.tril(np.ones((n, n), dtype=bool), -1)
    r = np.abs(np.tril(t @ lg - lg @ t, -1) + e)
    at, al = np.abs(t), np.abs(lg)
    b = np.sqrt(2) * (n + 8) * u * (at @ al + al @ at) + u * np.abs(e)
    return float(np.max(r[lower] / b[lower])) if lower.any() else 0.0


def _sweep_case(n, seed, scale=1e-6):
    rng = np.random.default_rng(seed)
    g = synth.schur_test_matrix(n, seed=seed)
    t = np.triu(g["T0"]).astype(np.complex64)
    e = (scale * np.tril(rand_c(rng, (n, n)), -1)).astype(np.complex64)
    return np.asfortranarray(t), np.asfortranarray(e)


@pytest.mark.parametrize("n", [2, 31, 33, 64, 65, 130, 300])
def test_trisolve_matches_exact_solution(sr, n):
    t, e = _sweep_case(n, 100 + n)
    ws = sr.workspace(n)
    l = empty(n, n, True)
    assert sr.sr_trisolve(dev(t), dev(e), l, ws) == 0
    lg = host(l).astype(np.complex128)
    assert not np.triu(lg).any()
    t64, e64 = t.astype(np.complex128), e.astype(np.complex128)
    lx = oracle.trisolve(t64, e64, lp="quad")[0].to_c128()  # exact solve of the same lp data
    lf = oracle.trisolve(t64, e64, lp="float")[0].to_c128()  # Algorithm 2 in FP32
    err_gpu = np.linalg.norm(lg - lx)
    err_alg2 = np.linalg.norm(lf - lx)
    assert err_gpu <= 10 * err_alg2 + 10 * U32 * np.linalg.norm(lx)
    # entry by entry: the componentwise backward error of a correct FP32 solve
    assert _residual_entrywise_ok(t64, e64, lg, U32) <= 1.0
    # and per column, the forward error within 10x the oracle's FP32 Algorithm 2
    ecol_gpu = np.abs(lg - lx).max(axis=0)
    ecol_alg2 = np.abs(lf - lx).max(axis=0)
    assert np.all(ecol_gpu <= 10 * ecol_alg2 + 10 * U32 * np.abs(lx).max(axis=0) + 1e-300)


def test_trisolve_32_wide_tiles(sr):
    """Above n = 2048 the level solve runs on 32-wide tiles (66 tile rows here, the
    last one ragged), in FP32 and in FP64. The quad solve is out of reach at this
    size, so the oracle's Algorithm 2 in FP64 is the reference: the FP32 solve must
    stay within 10x of the oracle's FP32 error, the FP64 solve within 10x of that
    error scaled by u64/u32, and both must meet the backward-error bound of the
    defining equation (eq. (7))."""
    n = 2100
    t, e = _sweep_case(n, 100 + n)
    t64, e64 = t.astype(np.complex128), e.astype(np.complex128)
    ld = oracle.trisolve(t64, e64, lp="double")[0].to_c128()
    lf = oracle.trisolve(t64, e64, lp="float")[0].to_c128()
    err_alg2 = np.linalg.norm(lf - ld)
    nt, nl = np.linalg.norm(t64), np.linalg.norm(ld)
    l32 = empty(n, n, True)
    assert sr.sr_trisolve(dev(t), dev(e), l32, sr.workspace(n)) == 0
    l64 = empty(n, n)
    assert sr.sr_trisolve64(dev(t64), dev(e64), l64, sr.workspace(n)) == 0
    for lg, u, bound in [(host(l32).astype(np.complex128), U32, 10 * err_alg2 + 10 * U32 * nl),
                         (host(l64), U64, 10 * err_alg2 * U64 / U32 + 10 * U64 * nl)]:
        assert not np.triu(lg).any()
        assert np.linalg.norm(lg - ld) <= bound
        res = np.linalg.norm(np.tril(t64 @ lg - lg @ t64, -1) + e64)
        assert res <= 8 * n * u * (nt * np.linalg.norm(lg) + np.linalg.norm(e64))
        assert _residual_entrywise_ok(t64, e64, lg, u) <= 1.0


def test_trisolve_one_by_one_and_breakdown(sr):
    ws = sr.workspace(4)
    l = empty(1, 1, True)
    one = np.ones((1, 1), dtype=np.complex64)
    assert sr.sr_trisolve(dev(one), dev(np.zeros((1, 1), np.complex64)), l, ws) == 0
    assert host(l)[0, 0] == 0
    t = np.triu(np.ones((40, 40), dtype=np.complex64))
    t[np.diag_indices(40)] = np.arange(40)
    t[35, 35] = t[3, 3]  # Theorem 1: equal diagonal entries make the equation singular
    e = np.tril(np.ones((40, 40), dtype=np.complex64), -1)
    l = empty(40, 40, True)
    assert sr.sr_trisolve(dev(t), dev(e), l, sr.workspace(40)) == 3  # SR_BREAKDOWN


def test_trisolve_truncation(sr):
    t, e = _sweep_case(70, 9, scale=1.0)
    l = empty(70, 70, True)
    assert sr.sr_trisolve(dev(t), dev(e), l, sr.workspace(70), trunc=1e-5) == 0
    assert np.abs(host(l)).max() <= 1e-5


@pytest.mark.parametrize("n,ref_lp", [(70, "quad"), (600, "double"), (2100, "double")])
def test_trisolve_truncation_as_computed_against_oracle(sr, n, ref_lp):
    """The large-entry device of Example 4 zeroes an entry of L as it is computed,
    so later entries see the zero. On a case whose few large entries (far above
    1e-5) feed every later entry, the GPU takes the same zeroing decisions as the
    oracle (the same zero pattern) and the surviving entries match the oracle's
    truncating solve entry by entry: 16- and 32-wide tiles, ragged edges."""
    from test_oracle_pins import truncation_case

    trunc = 1e-5
    t, e = truncation_case(n, 3)
    t32, e32 = t.astype(np.complex64), e.astype(np.complex64)
    t64, e64 = t32.astype(np.complex128), e32.astype(np.complex128)
    lr, st = oracle.trisolve(t64, e64, lp=ref_lp, trunc=trunc)
    assert st == "OK"
    lr = lr.to_c128()
    lower = np.tril(np.ones((n, n), dtype=bool), -1)
    ar = np.abs(lr[lower])
    assert np.all((ar == 0) | (ar < 0.1 * trunc))  # no decision close to the threshold
    assert np.count_nonzero(ar == 0) >= 3
    l = empty(n, n, True)
    assert sr.sr_trisolve(dev(t32), dev(e32), l, sr.workspace(n), trunc=trunc) == 0
    lg = host(l).astype(np.complex128)
    assert np.array_equal(lg == 0, lr == 0)
    # surviving entries: FP32 forward error, entry by entry relative to the largest
    # entry of their column (the entries are O(1e-8), the zeroed ones left out)
    scale = np.abs(lr).max(axis=0)[None, :]
    assert np.all(np.abs(lg - lr) <= 1e-3 * scale + 1e-30)
    # zeroing only after the sweep would give another L
    full = oracle.trisolve(t64, e64, lp="double")[0].to_c128()
    after = np.where(np.abs(full) > trunc, 0, full)
    assert np.abs(after - lr).max() >= 10 * np.abs(lr).max()


def test_ns_init_matches_quad(sr):
    n = 150
    g = synth.schur_test_matrix(n, seed=4)
    qh = synth.lp_schur_start(g["A"])
    q = empty(n, n)
    assert sr.sr_ns_init(dev(qh), q, sr.workspace(n)) == 0
    hi, lo = oracle.ns(qh).to_dd()
    err = np.linalg.norm((host(q) - hi) - lo)
    assert err <= 8 * U64 * n  # ||Q|| ~ sqrt(n); error ~ u sqrt(n) per column
    # entry by entry: first-order bound of Q = Qh + Qh (-Y0 / 2) with Y0 = Qh^H Qh - I
    # formed in FP64 (dot products of length n), the product Qh (Y0 / 2) and the sum
    aq = np.abs(qh)
    y0 = qh.conj().T @ qh - np.eye(n)
    bound = np.sqrt(2) * (n + 8) * U64 * (aq @ (aq.conj().T @ aq) / 2 + aq @ np.abs(y0) / 2) + U64 * np.abs(hi)
    assert np.all(np.abs((host(q) - hi) - lo) <= bound)
    # Lemma 2: the defect after the step is -3/4 Y0^2 + 1/4 Y0^3
    y0 = qh.conj().T @ qh - np.eye(n)
    y = host(q).conj().T @ host(q) - np.eye(n)
    pred = -0.75 * y0 @ y0 + 0.25 * y0 @ y0 @ y0
    assert np.linalg.norm(y - pred) <= 1e-2 * np.linalg.norm(pred) + 1e-13


def test_update_matches_oracle_merged_step(sr):
    n = 96
    g = synth.schur_test_matrix(n, seed=5)
    q = np.asfortranarray(oracle.ns(synth.lp_schur_start(g["A"])).to_c128())
    rng = np.random.default_rng(1)
    lmat = (1e-4 * np.tril(rand_c(rng, (n, n)), -1)).astype(np.complex64)
    w = lmat.astype(np.complex128) - lmat.astype(np.complex128).conj().T
    qo = empty(n, n)
    rc, (nw, ny) = sr.sr_update(dev(q), dev(lmat), qo, sr.workspace(n), gate=False)
    assert rc == 0
    assert abs(nw - np.linalg.norm(w)) <= 1e-6 * np.linalg.norm(w)
    hi, lo = oracle.ns_merged(q, w, lp="float", full=False).to_dd()
    err = np.linalg.norm((host(qo) - hi) - lo)
    # FP64 rounding of Q + Q Delta, plus FP32 rounding of the (1e-8 sized) lp products
    assert err <= 16 * U64 * n + 1e-7 * np.linalg.norm(w @ w) * np.sqrt(n)
    assert np.all(np.abs((host(qo) - hi) - lo) <= _update_bound(q, w, hi))


@pytest.mark.parametrize("n", [64, 200])
def test_update_hermitian_defect(sr, n):
    """Y = Q^H Q - I is formed from the tiles on and above the diagonal and mirrored;
    with a Q far from unitary (Y of order 0.1) its norm and the update built from
    it are checked against FP64 and the binary128 merged step (n = 200 leaves a
    ragged diagonal tile)."""
    rng = np.random.default_rng(70 + n)
    q = np.asfortranarray(np.eye(n) + 0.3 * rand_c(rng, (n, n)) / np.sqrt(n))
    lmat = (1e-4 * np.tril(rand_c(rng, (n, n)), -1)).astype(np.complex64)
    w = lmat.astype(np.complex128) - lmat.astype(np.complex128).conj().T
    qo = empty(n, n)
    rc, (nw, ny) = sr.sr_update(dev(q), dev(lmat), qo, sr.workspace(n), gate=False)
    assert rc == 0
    y = q.conj().T @ q - np.eye(n)
    assert abs(ny - np.linalg.norm(y)) <= 1e-12 * np.linalg.norm(y)
    hi, lo = oracle.ns_merged(q, w, lp="float", full=False).to_dd()
    # FP64 products plus FP32 lp products YW, W^2, W^3 (Y ~ 0.1, W ~ 1e-4)
    err = np.linalg.norm((host(qo) - hi) - lo)
    assert err <= 1e-9 * np.linalg.norm(hi)
    assert np.all(np.abs((host(qo) - hi) - lo) <= _update_bound(q, w, hi))


def _update_bound(q, w, qout):
    """Entrywise first-order bound for the GPU form Q + Q Delta of the merged
    update against the oracle's (float lp, binary128 hp) step: Y = Q^H Q - I in FP64
    (length-n dot products), the FP32 products YW, W^2, W^3 and their operands
    rounded to FP32 (operands rounded once; (W^2 - Y) W formed as one product when
    both terms are present), Delta in FP64, the FP64 product Q Delta and the sum."""
    n = q.shape[0]
    aq, aw = np.abs(q), np.abs(w)
    y = q.conj().T @ q - np.eye(n)
    ay = np.abs(y)
    c64 = np.sqrt(2) * (n + 8) * U64
    c32 = np.sqrt(2) * (n + 8) * U32
    d_y = c64 * (aq.conj().T @ aq) / 2
    d_lp = c32 * (ay @ aw + aw @ aw + aw @ aw @ aw + (aw @ aw + ay) @ aw) + U32 * (ay + aw @ aw) @ aw
    delta = np.abs(w) + ay / 2 + (ay @ aw + aw @ aw + aw @ aw @ aw) / 2
    return aq @ (d_y + d_lp + 4 * U64 * delta) + c64 * (aq @ delta) + 2 * U64 * np.abs(qout)

