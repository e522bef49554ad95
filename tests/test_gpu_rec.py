"""The recursive block solve (Algorithm 3) on the GPU: sr_trisolve_rec against the
binary128 oracle's exact solve of the same FP32 data, against the tile wavefront
(Theorem 1: the solution does not depend on the order), and inside the refinement
(sr_opts.solver)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import U32, U64, dev, empty, host, rand_c
from test_gpu_kernels import _residual_entrywise_ok, _sweep_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sr():
    import torch

    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


@pytest.mark.parametrize("n,leaf", [(2, 0), (31, 16), (33, 16), (64, 0), (65, 16), (130, 32), (300, 0),
                                    (300, 16), (513, 64), (513, 200)])
def test_rec_matches_exact_solution(sr, n, leaf):
    """Every entry within the componentwise backward-error bound of eq. (7) for an
    FP32 solve, and the forward error within 10x that of the oracle's FP32 Algorithm 2
    against the exact (binary128) solve of the same data, column by column."""
    t, e = _sweep_case(n, 700 + n)
    l = empty(n, n, True)
    e_dev = dev(e)
    assert sr.sr_trisolve_rec(dev(t), e_dev, l, leaf_rows=leaf) == 0
    assert np.array_equal(host(e_dev), e)  # E is not modified
    lg = host(l).astype(np.complex128)
    assert not np.triu(lg).any()
    t64, e64 = t.astype(np.complex128), e.astype(np.complex128)
    lx = oracle.trisolve(t64, e64, lp="quad")[0].to_c128()
    lf = oracle.trisolve(t64, e64, lp="float")[0].to_c128()
    assert _residual_entrywise_ok(t64, e64, lg, U32) <= 1.0
    assert np.linalg.norm(lg - lx) <= 10 * np.linalg.norm(lf - lx) + 10 * U32 * np.linalg.norm(lx)
    ecol = np.abs(lg - lx).max(axis=0)
    assert np.all(ecol <= 10 * np.abs(lf - lx).max(axis=0) + 10 * U32 * np.abs(lx).max(axis=0) + 1e-300)


@pytest.mark.parametrize("n", [1000, 2100])
def test_rec_agrees_with_wavefront(sr, n):
    """Theorem 1: the equation has one solution, whatever the order of the unknowns.
    The recursive solve and the wavefront solve (32-wide tiles above n = 2048) of the
    same FP32 data agree within the sum of their forward-error bounds, measured
    against the oracle's Algorithm 2 in FP64, and both meet the entrywise bound."""
    t, e = _sweep_case(n, 900 + n)
    t64, e64 = t.astype(np.complex128), e.astype(np.complex128)
    ld = oracle.trisolve(t64, e64, lp="double")[0].to_c128()
    lf = oracle.trisolve(t64, e64, lp="float")[0].to_c128()
    err_alg2 = np.linalg.norm(lf - ld)
    lr, lw = empty(n, n, True), empty(n, n, True)
    assert sr.sr_trisolve_rec(dev(t), dev(e), lr) == 0
    assert sr.sr_trisolve(dev(t), dev(e), lw, sr.workspace(n)) == 0
    a, b = host(lr).astype(np.complex128), host(lw).astype(np.complex128)
    for lg in (a, b):
        assert np.linalg.norm(lg - ld) <= 10 * err_alg2 + 10 * U32 * np.linalg.norm(ld)
        assert _residual_entrywise_ok(t64, e64, lg, U32) <= 1.0
    assert np.linalg.norm(a - b) <= 20 * err_alg2 + 20 * U32 * np.linalg.norm(ld)


def test_rec_breakdown_truncation_and_arguments(sr):
    t = np.triu(np.ones((40, 40), dtype=np.complex64))
    t[np.diag_indices(40)] = np.arange(40)
    t[35, 35] = t[3, 3]  # Theorem 1: equal diagonal entries make the equation singular
    e = np.tril(np.ones((40, 40), dtype=np.complex64), -1)
    l = empty(40, 40, True)
    assert sr.sr_trisolve_rec(dev(t), dev(e), l, leaf_rows=16) == 3  # SR_BREAKDOWN
    t2, e2 = _sweep_case(70, 9, scale=1.0)
    l2 = empty(70, 70, True)
    assert sr.sr_trisolve_rec(dev(t2), dev(e2), l2, trunc=1e-5) == 0
    assert np.abs(host(l2)).max() <= 1e-5
    import torch

    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    assert sr.sr_trisolve_rec(dev(t2), dev(e2), l2, ws=small) == -3  # SR_ENOMEM
    assert sr.sr_trisolve_rec(dev(t2), dev(e2), l2, leaf_rows=-1) == -1  # SR_EINVAL


def _refine(sr, a, qh, iters=6, tol=1e-15, **kw):
    n = a.shape[0]
    q, t = dev(qh), empty(n, n)
    info = sr.schur_refine(dev(a), q, t, iters=iters, tol=tol, **kw)
    return host(q), host(t), info


@pytest.mark.parametrize("n,leaf", [(64, 16), (257, 0), (1024, 0), (1024, 256)])
def test_refine_with_recursive_solver(sr, n, leaf):
    """The FP64 tier with the recursive solve converges like the wavefront (the same
    pass count within one), to a binary128-checked residual <= 1e-15."""
    g = synth.schur_test_matrix(n, seed=60 + n)
    qh = synth.lp_schur_start(g["A"])
    q, t, info = _refine(sr, g["A"], qh, solver="recursive", rec_leaf=leaf)
    _, _, ref = _refine(sr, g["A"], qh)
    assert info["status"] == "OK" and abs(info["iters"] - ref["iters"]) <= 1, (info, ref)
    rows = np.random.default_rng(5).choice(n, min(n, 32), replace=False)
    ev = oracle.evaluate_rows(g["A"], q, rows)
    assert ev["stril"] <= 1e-15 and ev["orth"] <= 4 * U64 * np.sqrt(n) * 10, ev


def test_recursive_solver_option_scope(sr):
    """The recursive solve is an option of the FP32 tier only."""
    g = synth.schur_test_matrix(32, seed=3)
    qh = synth.lp_schur_start(g["A"])
    a = dev(g["A"])
    q, t = dev(qh), empty(32, 32)
    assert sr.schur_refine(a, q, t, solver=2)["status"] == "EINVAL"
    gr = synth.real_schur_test_matrix(32, seed=3)
    qr, blk = synth.lp_real_schur_start(gr["A"])
    import torch

    assert sr.schur_refine_real(dev(gr["A"]), dev(qr), sr.colmajor_empty(32, 32, torch.float64), blk,
                                solver="recursive")["rc"] == -4  # SR_ENOSYS


@pytest.mark.parametrize("n,mode", [(257, "fp64"), (1024, "fp64"), (1024, "ozaki_crt")])
def test_skip_orth(sr, n, mode):
    """Section 2.4: with Q (I + W) already unitary in hp the product Y of an update can
    be left out. Four passes with a tolerance below reach (three updates): from the
    cgees start the first correction is ||W|| = 1e-4 .. 4e-4, so the predicted ||Y||
    before the second update is 3/4 ||W_1||^4 (7e-17 at n = 257: skipped there, 2e-14
    at n = 1024: formed); before the third it is below 1e-27 (skipped at n = 1024,
    formed at n = 257 right after a skip). Either way one hp product fewer, the same
    passes, and Q unitary to the rounding level on binary128 rows. Off by default."""
    g = synth.schur_test_matrix(n, seed=80 + n)
    a, qh = g["A"], synth.lp_schur_start(g["A"])
    kw = dict(gemm=mode, iters=4, tol=1e-30)
    q0, _, ref = _refine(sr, a, qh, **kw)
    q1, _, info = _refine(sr, a, qh, skip_orth=True, **kw)
    assert info["iters"] == ref["iters"] == 4 and info["status"] == ref["status"], (info, ref)
    assert ref["hp_gemms"] == 4 * ref["iters"]
    assert info["hp_gemms"] == ref["hp_gemms"] - 1, (info["hp_gemms"], ref["hp_gemms"], info["norm_w_hist"])
    rows = np.random.default_rng(6).choice(n, 32, replace=False)
    for q in (q0, q1):
        ev = oracle.evaluate_rows(a, q, rows)
        assert ev["stril"] <= 1e-15 and ev["orth"] <= 4 * U64 * np.sqrt(n) * 10, ev
    ad = dev(a)
    assert sr.schur_refine_dd(ad, dev(np.zeros_like(a)), dev(qh), dev(np.zeros_like(qh)), empty(n, n),
                              empty(n, n), skip_orth=True)["rc"] == -4  # SR_ENOSYS
