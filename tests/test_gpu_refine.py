"""End-to-end GPU refinement (schur_refine through the C interface) against the
binary128 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import U64, dev, empty, host, phase_align

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sr():
    import torch

    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _refine(sr, a, qh, iters=6, tol=1e-15, **kw):
    n = a.shape[0]
    q, t = dev(qh), empty(n, n)
    info = sr.schur_refine(dev(a), q, t, iters=iters, tol=tol, **kw)
    return host(q), host(t), info


def test_config0_n64_against_oracle_mirror(sr):
    """n = 64, gaps 0.05, start = complex64 Schur form from the oracle's QR
    algorithm; FP64 tier, tol 1e-15, at most 6 passes."""
    g = synth.schur_test_matrix(64, seed=0)
    a = g["A"]
    z, _ = oracle.schur_qr(a.astype(np.complex64).astype(np.complex128), lp="float")
    qh = np.asfortranarray(z.astype(np.complex64).astype(np.complex128))
    q, t, info = _refine(sr, a, qh)
    assert info["status"] == "OK" and info["iters"] <= 5, info
    assert info["hp_gemms"] == 4 * info["iters"]
    ev = oracle.evaluate(a, q, t)
    assert ev["stril"] <= 1e-15 and ev["orth"] <= 1e-13 and ev["tdiff"] <= 1e-13 * ev["normA"]
    # the (float lp, quad hp) oracle mirrors the iteration: same eps per pass
    # while above the FP64 floor (within a factor 10)
    ref = oracle.refine(a, qh, lp="float", maxit=6, tol=1e-15)
    for k, (eg, eo) in enumerate(zip(info["resid_hist"], ref["hist"])):
        if eo > 1e-14:
            assert 0.1 * eo <= eg <= 10 * eo, (k, eg, eo)
    # the Schur form itself: diag(T) recovers diag(T0), Q matches the oracle's
    assert np.max(np.min(np.abs(np.diag(t)[:, None] - g["lam"][None, :]), axis=1)) <= 1e-12
    qq = oracle.refine(a, qh, lp="quad", maxit=8, tol=1e-30)["Q"].to_c128()
    assert np.linalg.norm(phase_align(q, qq) - qq) <= 1e-13


@pytest.mark.parametrize("n", [16, 64, 256])
def test_exact_hadamard_schur_form(sr, n):
    h = synth.hadamard_exact(n, seed=n + 1)
    qh = synth.perturbed_start(h["Q0"], seed=2, delta=1e-6)
    q, t, info = _refine(sr, h["A"], qh)
    assert info["status"] == "OK", info
    assert np.abs(np.diag(t) - h["lam"]).max() <= 1e-13
    c = h["Q0"].real.T @ q  # must be diagonal unitary
    assert np.abs(c - np.diag(np.diag(c))).max() <= 1e-13
    assert np.abs(np.abs(np.diag(c)) - 1).max() <= 1e-13


@pytest.mark.parametrize("n", [1, 2, 17, 100, 257])
def test_ragged_sizes_converge(sr, n):
    g = synth.schur_test_matrix(n, seed=50 + n)
    qh = synth.lp_schur_start(g["A"])
    q, t, info = _refine(sr, g["A"], qh)
    assert info["status"] == "OK", info
    ev = oracle.evaluate(g["A"], q, t)
    assert ev["stril"] <= 1e-15 and ev["orth"] <= 1e-12


def test_config1_n1024_quad_rows(sr):
    """n = 1024 (the benchmark workload): passes to 1e-15, quad error on 64 rows."""
    g = synth.schur_test_matrix(1024, seed=1)
    a = g["A"]
    qh = synth.lp_schur_start(a)
    q, t, info = _refine(sr, a, qh)
    assert info["status"] == "OK" and info["iters"] <= 5, info
    rows = np.random.default_rng(20001).choice(1024, 64, replace=False)
    ev = oracle.evaluate_rows(a, q, rows)
    assert ev["stril"] <= 1e-15, ev
    assert ev["orth"] <= 4 * U64 * np.sqrt(1024) * 10, ev
    assert np.max(np.min(np.abs(np.diag(t)[:, None] - g["lam"][None, :]), axis=1)) <= 1e-10


@pytest.fixture(scope="module")
def config2():
    """n = 4096, eigenvalue gaps >= 1e-3 (seed 2), started from the complex64 Schur
    basis of complex64(A) (LAPACK cgees): the benchmark's workload (about 17 s of
    host work, made once for the three forms)."""
    g = synth.schur_test_matrix(4096, seed=2, gap=1e-3)
    return g["A"], synth.lp_schur_start(g["A"])


@pytest.mark.parametrize("mode", ["fp64", "ozaki_i8", "ozaki_i8_all", "ozaki_crt", "ozaki_i8_all/lp4",
                                  "ozaki_crt/lp4"])
def test_config2_n4096_quad_rows(sr, config2, mode):
    """The precision comparison at n = 4096 in each form of the hp products (native
    FP64; INT8 digits for P, the start and Q Delta; INT8 digits for every hp
    product; residues for every hp product; "/lp4": the lp products from 4 INT8
    digits as well): at most 5 passes to 1e-15 (the paper's count, That evaluations),
    and the binary128 residual and orthogonality on 32 sampled rows."""
    a, qh = config2
    n = a.shape[0]
    form, _, lp = mode.partition("/lp")
    q, t, info = _refine(sr, a, qh, iters=8, gemm=form, lp_digits=int(lp or 0))
    assert info["status"] == "OK" and info["iters"] <= 5, (mode, info)
    assert info["hp_gemms"] == 4 * info["iters"]
    rows = np.random.default_rng(20002).choice(n, 32, replace=False)
    ev = oracle.evaluate_rows(a, q, rows)
    assert ev["stril"] <= 1e-15 and ev["stril_rowmax"] <= 1e-15, (mode, ev)
    assert ev["orth"] <= 4 * U64 * np.sqrt(n), (mode, ev)
    # T is triu(Q^H A Q) of the returned Q (checked on the sampled rows' diagonal)
    assert not np.tril(t[:64, :64], -1).any()


def test_status_codes(sr):
    g = synth.schur_test_matrix(40, seed=3)
    qh = synth.lp_schur_start(g["A"])
    _, _, info = _refine(sr, g["A"], qh, iters=1)
    assert info["status"] == "NOT_CONVERGED" and info["iters"] == 1 and info["rc"] == 1
    a = g["A"].copy()
    a[5, 7] = np.nan
    _, _, info = _refine(sr, a, qh)
    assert info["status"] == "BREAKDOWN"
    # invalid arguments are rejected without touching the outputs
    q, t = dev(qh), empty(40, 40)
    info = sr.schur_refine(dev(g["A"]), q, t, iters=0)
    assert info["rc"] == -1
    assert np.array_equal(host(q), qh)


def test_resume_from_saved_iterate(sr):
    """Checkpoint/resume: a second call from the first call's Q continues the
    iteration (the method accepts any nearly unitary start)."""
    g = synth.schur_test_matrix(128, seed=8)
    qh = synth.lp_schur_start(g["A"])
    q1, _, i1 = _refine(sr, g["A"], qh, iters=2, tol=1e-15)
    q2, t2, i2 = _refine(sr, g["A"], q1, iters=4, tol=1e-15)
    assert i1["status"] == "NOT_CONVERGED" and i2["status"] == "OK"
    assert oracle.evaluate(g["A"], q2, t2)["stril"] <= 1e-15


@pytest.mark.parametrize("sizes", [[20, 50, 90, 1, 2, 130], [2, 17, 32, 5, 31]])
def test_batched_matches_single(sr, sizes):
    """The batched driver (grouped launches, device-side loop control, graph
    replays) reaches the same passes and, up to rounding, the same Q and T as
    single calls. The first batch solves by tile diagonal across the matrices, the
    second (no matrix with more than two 16-wide tile rows) one block per matrix."""
    mats = [synth.schur_test_matrix(n, seed=200 + n) for n in sizes]
    starts = [synth.lp_schur_start(m["A"]) for m in mats]
    As = [dev(m["A"]) for m in mats]
    Qs = [dev(s) for s in starts]
    Ts = [empty(n, n) for n in sizes]
    rc, infos = sr.schur_refine_batched(As, Qs, Ts)
    assert rc == 0
    for m, s, qd, td, inf in zip(mats, starts, Qs, Ts, infos):
        q1, t1, i1 = _refine(sr, m["A"], s)
        assert inf["status"] == "OK" and inf["iters"] == i1["iters"], (inf, i1)
        assert inf["hp_gemms"] == i1["hp_gemms"] or m["A"].shape[0] == 1
        qb, tb = host(qd), host(td)
        assert np.linalg.norm(qb - q1) <= 1e-12 * np.sqrt(qb.shape[0])
        assert np.linalg.norm(tb - t1) <= 1e-12 * np.linalg.norm(t1)
        ev = oracle.evaluate(m["A"], qb, tb)
        assert ev["stril"] <= 1e-15 and ev["orth"] <= 1e-12, ev


def test_batched_uneven_sizes_and_outcomes(sr):
    """A batch of uneven sizes (16..256) with one broken matrix: the others still
    converge, the broken one reports BREAKDOWN, the batch the worst outcome."""
    rng = np.random.default_rng(31)
    sizes = [int(x) for x in rng.integers(16, 257, 24)]
    mats = [synth.schur_test_matrix(n, seed=400 + i) for i, n in enumerate(sizes)]
    starts = [synth.lp_schur_start(m["A"]) for m in mats]
    bad = mats[5]["A"].copy()
    bad[3, 4] = np.nan
    As = [dev(bad if i == 5 else m["A"]) for i, m in enumerate(mats)]
    Qs = [dev(s) for s in starts]
    Ts = [empty(n, n) for n in sizes]
    rc, infos = sr.schur_refine_batched(As, Qs, Ts)
    assert rc == 3  # SR_BREAKDOWN, the worst outcome
    for i, (m, qd, td, inf) in enumerate(zip(mats, Qs, Ts, infos)):
        if i == 5:
            assert inf["status"] == "BREAKDOWN"
            continue
        assert inf["status"] == "OK" and inf["iters"] <= 5, (i, inf)
        if i % 6 == 0:
            ev = oracle.evaluate(m["A"], host(qd), host(td))
            assert ev["stril"] <= 1e-15 and ev["orth"] <= 1e-12, (i, ev)
    for n in sizes:
        assert sr.lib().sr_batched_tile_edge(n) in (32, 64)


def test_batched_pass_limit_and_workspace(sr):
    sizes = [40, 70, 33]
    mats = [synth.schur_test_matrix(n, seed=600 + n) for n in sizes]
    starts = [synth.lp_schur_start(m["A"]) for m in mats]
    ws = sr.workspace_batched(sizes)
    As = [dev(m["A"]) for m in mats]
    Qs = [dev(s) for s in starts]
    Ts = [empty(n, n) for n in sizes]
    rc, infos = sr.schur_refine_batched(As, Qs, Ts, iters=1, workspace=ws)
    assert rc == 1 and all(i["status"] == "NOT_CONVERGED" and i["iters"] == 1 for i in infos)
    # resume from the saved iterates with an odd pass limit
    rc, infos = sr.schur_refine_batched(As, Qs, Ts, iters=3, workspace=ws)
    assert rc == 0, infos
    for m, qd, td in zip(mats, Qs, Ts):
        assert oracle.evaluate(m["A"], host(qd), host(td))["stril"] <= 1e-15


@pytest.mark.parametrize("mode", ["ozaki_i8", "ozaki_i8_all", "ozaki_crt"])
@pytest.mark.parametrize("n", [64, 257])
def test_ozaki_mode_converges(sr, n, mode):
    """Ozaki modes (P = A Q, the start's products and Q Delta on INT8 digits; That and
    Y native FP64, or from digits too) reach the same tolerance in the same number of
    passes."""
    g = synth.schur_test_matrix(n, seed=300 + n)
    qh = synth.lp_schur_start(g["A"])
    q, t, info = _refine(sr, g["A"], qh, gemm=mode)
    _, _, ref = _refine(sr, g["A"], qh)
    assert info["status"] == "OK", info
    assert abs(info["iters"] - ref["iters"]) <= 1, (info, ref)
    ev = oracle.evaluate(g["A"], q, t)
    assert ev["stril"] <= 1e-15 and ev["orth"] <= 1e-12, ev
    su = info["update_slices_hist"]
    lo, hi = (12, 55) if mode == "ozaki_crt" else (2, 8)
    assert all(lo <= s <= hi for s in su[: info["updates"] + 1]), su
    # later updates need fewer digits (Delta shrinks quadratically)
    assert su[info["updates"]] <= su[0], su


def test_ozaki_mode_exact_hadamard(sr):
    h = synth.hadamard_exact(256, seed=9)
    qh = synth.perturbed_start(h["Q0"], seed=4, delta=1e-6)
    q, t, info = _refine(sr, h["A"], qh, gemm="ozaki_i8", update_slices=4)
    assert info["status"] == "OK", info
    assert np.abs(np.diag(t) - h["lam"]).max() <= 1e-13
    c = h["Q0"].real.T @ q
    assert np.abs(c - np.diag(np.diag(c))).max() <= 1e-13


@pytest.mark.parametrize("mode", ["ozaki_i8", "ozaki_i8_all", "ozaki_crt"])
def test_ozaki_mode_n1024_quad_rows(sr, mode):
    g = synth.schur_test_matrix(1024, seed=1)
    a = g["A"]
    qh = synth.lp_schur_start(a)
    q, t, info = _refine(sr, a, qh, gemm=mode)
    assert info["status"] == "OK" and info["iters"] <= 5, info
    rows = np.random.default_rng(20001).choice(1024, 64, replace=False)
    ev = oracle.evaluate_rows(a, q, rows)
    assert ev["stril"] <= 1e-15, ev
    assert ev["orth"] <= 4 * U64 * np.sqrt(1024) * 10, ev


def test_gemm_mode_validation(sr):
    g = synth.schur_test_matrix(32, seed=5)
    qh = synth.lp_schur_start(g["A"])
    q, t = dev(qh), empty(32, 32)
    assert sr.schur_refine(dev(g["A"]), q, t, gemm="ozaki_bf16")["rc"] == -4
    assert sr.schur_refine(dev(g["A"]), q, t, gemm=7)["rc"] == -1
    assert sr.schur_refine(dev(g["A"]), q, t, gemm="ozaki_i8", slices=17)["rc"] == -1
    assert sr.schur_refine(dev(g["A"]), q, t, gemm="ozaki_i8", update_slices=9)["rc"] == -1
    assert np.array_equal(host(q), qh)


def test_ozaki_mode_n2048_large_tiles(sr):
    """n = 2048: every Ozaki product takes the all-pairs kernel (64 x 64 tiles)."""
    g = synth.schur_test_matrix(2048, seed=6, gap=0.01)
    a = g["A"]
    qh = synth.lp_schur_start(a)
    q, t, info = _refine(sr, a, qh, gemm="ozaki_i8")
    assert info["status"] == "OK" and info["iters"] <= 6, info
    rows = np.random.default_rng(20002).choice(2048, 24, replace=False)
    ev = oracle.evaluate_rows(a, q, rows)
    assert ev["stril"] <= 1e-15, ev
    assert ev["orth"] <= 4 * U64 * np.sqrt(2048) * 10, ev


def test_batched_config3_full_batch(sr):
    """The batched workload at full size: 2000 matrices, n uniform in [16, 256]
    (seed 3), each from its own seed with a cgees start, refined in one call. Every
    matrix converges within 5 passes; the binary128 residual and orthogonality of 12
    sampled matrices are checked in full, and their passes and results agree with
    single calls."""
    import os

    sizes = [int(x) for x in synth.batched_sizes(2000, seed=3)]
    data = synth.batched_inputs(sizes, 10000, workers=min(16, os.cpu_count() or 1))
    As = [dev(a) for a, _ in data]
    Qs = [dev(q) for _, q in data]
    Ts = [empty(n, n) for n in sizes]
    rc, infos = sr.schur_refine_batched(As, Qs, Ts, iters=8)
    assert rc == 0
    passes = np.array([i["iters"] for i in infos])
    assert passes.max() <= 5 and all(i["status"] == "OK" for i in infos)
    for i in np.random.default_rng(5).choice(2000, 12, replace=False):
        a, qh = data[i]
        qb, tb = host(Qs[i]), host(Ts[i])
        ev = oracle.evaluate(a, qb, tb)
        assert ev["stril"] <= 1e-15 and ev["orth"] <= 4 * U64 * np.sqrt(sizes[i]) * 10, (i, ev)
        q1, t1, i1 = _refine(sr, a, qh)
        assert i1["iters"] == infos[i]["iters"]
        assert np.linalg.norm(qb - q1) <= 1e-12 * np.sqrt(sizes[i])


def test_batched_graph_kept_across_calls(sr):
    """With a caller-owned workspace, a second call on the same sizes, pass limit
    and tolerance replays the graph captured by the first (no new capture), also
    for other matrices of those sizes; a change of size captures anew."""
    sizes = [24, 61, 130, 7]
    ws = sr.workspace_batched(sizes)
    builds = sr.lib().sr_batched_graph_builds

    def run(seed0, szs, wsp):
        mats = [synth.schur_test_matrix(n, seed=seed0 + n) for n in szs]
        As = [dev(m["A"]) for m in mats]
        Qs = [dev(synth.lp_schur_start(m["A"])) for m in mats]
        Ts = [empty(n, n) for n in szs]
        rc, infos = sr.schur_refine_batched(As, Qs, Ts, workspace=wsp)
        assert rc == 0, infos
        for m, qd, td in zip(mats, Qs, Ts):
            assert oracle.evaluate(m["A"], host(qd), host(td))["stril"] <= 1e-15

    run(700, sizes, ws)
    b1 = builds()
    run(800, sizes, ws)
    assert builds() == b1
    sizes2 = [24, 61, 131, 7]
    run(900, sizes2, sr.workspace_batched(sizes2))
    assert builds() == b1 + 1
