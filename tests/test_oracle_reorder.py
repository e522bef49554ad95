"""Pins of the oracle's reordering of the start (Section 2.4, the paragraph on the
first step of Algorithm 4: the lp Schur form is reordered so that clustered
eigenvalues sit next to each other, in the order of their projections onto a
random line). The reordered Schur form with a given diagonal order is unique up
to column phases, so the checks fix the result without following the swaps:
Q unitary, Q^H A Q upper triangular, its diagonal in key order, and closed forms.
"""
import numpy as np
import pytest

import oracle
import synth


def _reordered(a, qh, theta):
    q, perm = oracle.reorder(np.asfortranarray(a), np.asfortranarray(qh), theta)
    hi, lo = q.to_dd()
    return hi + lo, perm


def _keys(lam, theta):
    return (lam * np.exp(-1j * theta)).real


def test_two_by_two_closed_form():
    # [[a, b], [0, d]] with key(a) > key(d): the unitary whose first column is the
    # eigenvector (b, d - a) of d gives [[d, *], [0, a]]
    a, b, d = 3 + 1j, 0.5 - 0.2j, -1 + 0.5j
    t = np.array([[a, b], [0, d]], dtype=complex)
    q, perm = _reordered(t, np.eye(2, dtype=complex), 0.0)
    x = np.array([b, d - a])
    assert np.allclose(q[:, 0], x / np.linalg.norm(x), atol=1e-15)
    s = q.conj().T @ t @ q
    assert abs(s[0, 0] - d) < 1e-15 and abs(s[1, 1] - a) < 1e-15 and abs(s[1, 0]) < 1e-15
    assert list(perm) == [1, 0]


@pytest.mark.parametrize("n,theta", [(5, 0.3), (30, 2.1), (64, -1.2)])
def test_reordered_schur_form_properties(n, theta):
    g = synth.schur_test_matrix(n, seed=40 + n)
    a, q0 = g["A"], g["Q0"]
    lam = np.diag(q0.conj().T @ a @ q0)  # the known spectrum, in the start's order
    q, perm = _reordered(a, q0, theta)
    s = q.conj().T @ a @ q
    nrm = np.linalg.norm(a)
    assert np.linalg.norm(q.conj().T @ q - np.eye(n)) < 1e-13 * n
    assert np.linalg.norm(np.tril(s, -1)) / nrm < 1e-13
    # the diagonal is the spectrum in increasing key order, and perm records it
    order = np.argsort(_keys(lam, theta), kind="stable")
    assert list(perm) == list(order)
    assert np.max(np.abs(np.diag(s) - lam[order])) < 1e-12 * np.max(np.abs(lam))
    assert np.all(np.diff(_keys(np.diag(s), theta)) > 0)


def test_first_schur_vector_is_the_eigenvector():
    # brute force at n = 4: column 0 of the reordered basis spans the eigenvector
    # of the eigenvalue with the smallest key
    g = synth.schur_test_matrix(4, seed=7)
    a = g["A"]
    theta = 0.9
    q, _ = _reordered(a, g["Q0"], theta)
    w, v = np.linalg.eig(a)
    k = np.argmin(_keys(w, theta))
    vk = v[:, k] / np.linalg.norm(v[:, k])
    assert abs(abs(np.vdot(q[:, 0], vk)) - 1) < 1e-13


def test_sorted_start_is_unchanged_and_opposite_line_reverses():
    g = synth.schur_test_matrix(12, seed=3)
    a, q0 = g["A"], g["Q0"]
    lam = np.diag(q0.conj().T @ a @ q0)
    theta = 0.4
    q, perm = _reordered(a, q0, theta)
    # the result in key order is a fixed point
    q2, perm2 = _reordered(a, q, theta)
    assert list(perm2) == list(range(12)) and np.array_equal(q2, q)
    # the opposite direction reverses the order
    _, perm3 = _reordered(a, q0, theta + np.pi)
    assert list(perm3) == list(np.argsort(_keys(lam, theta + np.pi), kind="stable"))
    assert list(np.asarray(perm3)[::-1]) == list(perm)


def test_lp_start_keeps_its_residual():
    # from an FP32 Schur start the swaps leave the residual at its level
    g = synth.schur_test_matrix(48, seed=5)
    a = g["A"]
    qh = synth.lp_schur_start(a)
    q, _ = _reordered(a, qh, 1.3)
    nrm = np.linalg.norm(a)
    r0 = np.linalg.norm(np.tril(qh.conj().T @ a @ qh, -1)) / nrm
    r1 = np.linalg.norm(np.tril(q.conj().T @ a @ q, -1)) / nrm
    assert r1 < 10 * r0
    assert np.linalg.norm(q.conj().T @ q - np.eye(48)) < 10 * np.linalg.norm(qh.conj().T @ qh - np.eye(48))
