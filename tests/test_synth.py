"""Invariants of the seeded generators (shared by the oracle tests and the GPU tests)."""
from fractions import Fraction

import numpy as np

import synth


def test_schur_test_matrix_invariants():
    g = synth.schur_test_matrix(48, seed=0, gap=0.05)
    n = 48
    assert g["A"].flags.f_contiguous and g["A"].dtype == np.complex128
    assert np.linalg.norm(g["Q0"].conj().T @ g["Q0"] - np.eye(n)) < 1e-13
    lam = g["lam"]
    d = np.abs(lam[:, None] - lam[None, :]) + np.eye(n) * 10
    assert d.min() > 0.05
    assert np.allclose(np.diag(g["T0"]), lam) and not np.tril(g["T0"], -1).any()
    w = np.linalg.eigvals(g["A"])
    for x in lam:
        assert np.min(np.abs(w - x)) < 1e-10
    g2 = synth.schur_test_matrix(48, seed=0, gap=0.05)
    assert np.array_equal(g["A"], g2["A"])


def test_hadamard_matrix_is_exact():
    h = synth.hadamard_exact(16, seed=4)
    a, q0, t0 = h["A"], h["Q0"].real, h["T0"]
    s = Fraction(1, 4)
    for i in range(0, 16, 5):
        for j in range(16):
            exact_re = sum(s * s * int(np.sign(q0[i, k])) * int(np.sign(q0[j, l])) * Fraction(t0[k, l].real)
                           for k in range(16) for l in range(16))
            exact_im = sum(s * s * int(np.sign(q0[i, k])) * int(np.sign(q0[j, l])) * Fraction(t0[k, l].imag)
                           for k in range(16) for l in range(16))
            assert Fraction(a[i, j].real) == exact_re and Fraction(a[i, j].imag) == exact_im


def test_lp_start_is_complex64_schur_basis():
    g = synth.schur_test_matrix(32, seed=1)
    q = synth.lp_schur_start(g["A"])
    assert np.array_equal(q, q.astype(np.complex64).astype(np.complex128))
    th = q.conj().T @ g["A"] @ q
    assert np.linalg.norm(np.tril(th, -1)) / np.linalg.norm(g["A"]) < 1e-5


def test_continuation_dd_is_exact():
    a0 = synth.schur_test_matrix(8, seed=4)["A"]
    a1 = synth.continuation_perturbation(8, seed=5)
    for k in (0, 1, 37, 63):
        hi, lo = synth.continuation_step_dd(a0, a1, k)
        for (i, j) in [(0, 0), (3, 5), (7, 2)]:
            exact = Fraction(a0[i, j].real) + Fraction(k, 64) * Fraction(a1[i, j].real)
            assert Fraction(hi[i, j].real) + Fraction(lo[i, j].real) == exact


def test_batched_sizes_range():
    s = synth.batched_sizes()
    assert s.size == 2000 and s.min() >= 16 and s.max() <= 256
