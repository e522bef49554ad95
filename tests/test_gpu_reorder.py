"""Reordering of the start on the GPU (Section 2.4, the paragraph on the reordering
of Algorithm 4) against the binary128 oracle, and the clustered-spectrum example
(Section 3, Example 3) as an acceptance test of the double-double tier."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, empty, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sr():
    import torch

    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _gpu_reorder(sr, a, q, theta):
    import torch

    n = a.shape[0]
    qd = dev(q)
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    assert sr.reorder_start(dev(a), qd, theta, perm=perm) == 0
    return host(qd), perm.cpu().numpy()


@pytest.mark.parametrize("n,theta,seed", [(2, 0.5, 1), (3, 2.0, 2), (33, -0.8, 3), (150, 1.1, 4), (257, 2.9, 5)])
def test_reorder_matches_oracle(sr, n, theta, seed):
    g = synth.schur_test_matrix(n, seed=seed)
    a = g["A"]
    qh = synth.lp_schur_start(a)
    q, perm = _gpu_reorder(sr, a, qh, theta)
    qo, permo = oracle.reorder(a, qh, theta)
    hi, lo = qo.to_dd()
    # the same swaps in the same order: the same permutation, and the bases agree to
    # the FP64 rounding of the rotations
    assert np.array_equal(perm, permo)
    assert np.max(np.abs(q - (hi + lo))) <= 1e-13 * np.sqrt(n)
    # properties of the result itself
    s = q.conj().T @ a @ q
    key = (np.diag(s) * np.exp(-1j * theta)).real
    assert np.all(np.diff(key) > 0)
    nrm = np.linalg.norm(a)
    r0 = np.linalg.norm(np.tril(qh.conj().T @ a @ qh, -1)) / nrm
    assert np.linalg.norm(np.tril(s, -1)) / nrm <= 10 * r0


def test_reorder_sorted_start_and_validation(sr):
    import torch

    g = synth.schur_test_matrix(20, seed=9)
    a, q0 = g["A"], g["Q0"]
    lam = np.diag(q0.conj().T @ a @ q0)
    theta = 0.3
    order = np.argsort((lam * np.exp(-1j * theta)).real, kind="stable")
    q, perm = _gpu_reorder(sr, a, q0, theta)
    assert list(perm) == list(order)
    # already in key order: nothing moves
    q2, perm2 = _gpu_reorder(sr, a, q, theta)
    assert list(perm2) == list(range(20)) and np.array_equal(q2, q)
    # n = 1 and argument checks
    one = dev(np.array([[2.0 + 1j]]))
    p1 = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    assert sr.reorder_start(one, dev(np.array([[1.0 + 0j]])), 0.0, perm=p1) == 0 and int(p1[0]) == 0
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    assert sr.reorder_start(dev(a), dev(q0), 0.0, ws=ws) == -1
    assert sr.reorder_start(dev(a), dev(q0), float("nan")) == -1


def _refine_dd(sr, a, q):
    n = a.shape[0]
    qhd, qld = dev(q), dev(np.zeros_like(q))
    th, tl = empty(n, n), empty(n, n)
    info = sr.schur_refine_dd(dev(a), dev(np.zeros_like(a)), qhd, qld, th, tl, iters=10, tol=1e-28)
    return host(qhd), host(qld), info


def test_example3_clusters_fail_and_softened_converges(sr):
    """Example 3 (n = 150, A = X D X^{-1}, two clusters of 10 eigenvalues within
    1e-5): from a reordered double Schur start the double-double refinement fails,
    as the oracle does and as the paper reports; with cond(X) = 1e4 instead of 1e5
    it converges to 1e-28 (the paper: in 6 iterations)."""
    theta = 1.1
    g = synth.example3_matrix(150, seed=0, cond_x=1e5, radius=1e-5)
    q, _ = _gpu_reorder(sr, g["A"], synth.hp_schur_start(g["A"]), theta)
    _, _, info = _refine_dd(sr, g["A"], q)
    assert info["status"] != "OK", info
    ref = oracle.refine(g["A"], np.asfortranarray(q), lp="double", maxit=10, tol=1e-28)
    assert ref["status"] != "OK", ref["status"]

    g = synth.example3_matrix(150, seed=0, cond_x=1e4, radius=1e-5)
    q, _ = _gpu_reorder(sr, g["A"], synth.hp_schur_start(g["A"]), theta)
    q_hi, q_lo, info = _refine_dd(sr, g["A"], q)
    assert info["status"] == "OK" and info["iters"] <= 7, info
    ev = oracle.evaluate(oracle.QMat.from_dd(g["A"]), oracle.QMat.from_dd(q_hi, q_lo))
    assert ev["stril"] <= 1e-28 and ev["orth"] <= 1e-26, ev
    ref = oracle.refine(g["A"], np.asfortranarray(q), lp="double", maxit=10, tol=1e-28)
    assert ref["status"] == "OK" and abs(ref["iters"] - info["iters"]) <= 1, (ref["iters"], info["iters"])
