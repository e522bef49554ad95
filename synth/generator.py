"""Seeded test-matrix generators.

Every generator is deterministic in its seed. Matrices come back as complex128
numpy arrays in column-major (Fortran) order, which is the storage order of the
library's C interface.

Workloads follow the shape of the paper's dense random experiments (Section 3,
Example 2): A = Q0 T0 Q0^H with a Haar-random unitary Q0 and an upper
triangular T0 whose diagonal holds gap-separated complex normal eigenvalues.
The starting basis is the Schur basis of the matrix rounded to a lower
precision, computed by LAPACK (cgees for complex64, zgees for complex128).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def cn(rng: np.random.Generator, shape) -> np.ndarray:
    """Standard complex normal draws, (N(0,1) + i N(0,1)) / sqrt(2), so E|z|^2 = 1."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / math.sqrt(2.0)


def _cn_square(rng: np.random.Generator, n: int) -> np.ndarray:
    """n x n complex normal matrix, filled column by column."""
    return np.asfortranarray(cn(rng, n * n).reshape((n, n), order="F"))


def haar_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed unitary: QR of a complex normal matrix with the phases of
    diag(R) moved into Q (Mezzadri's correction)."""
    z = _cn_square(rng, n)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    ph = d / np.abs(d)
    return np.asfortranarray(q * ph[None, :])


def gapped_eigenvalues(rng: np.random.Generator, n: int, gap: float,
                       grid: float | None = None) -> np.ndarray:
    """Complex normal eigenvalues drawn one at a time; a draw is rejected while it
    lies within `gap` of an earlier accepted one. With `grid`, each draw is first
    rounded to that grid (used for exactly representable test matrices)."""
    lam = np.empty(n, dtype=np.complex128)
    for i in range(n):
        while True:
            z = cn(rng, 1)[0]
            if grid is not None:
                z = complex(round(z.real / grid) * grid, round(z.imag / grid) * grid)
            if i == 0 or float(np.min(np.abs(lam[:i] - z))) > gap:
                break
        lam[i] = z
    return lam


def schur_test_matrix(n: int, seed: int, gap: float = 0.05) -> dict:
    """A = Q0 T0 Q0^H with known eigenvalues diag(T0).

    Draw order from numpy's PCG64 stream `default_rng(seed)`: the n x n complex
    normal matrix behind Q0 (column by column), then the eigenvalues with
    sequential gap rejection, then an n x n complex normal matrix whose strictly
    upper part, scaled by 1/sqrt(n), becomes the strictly upper part of T0.
    A is formed in float64 arithmetic.
    """
    rng = np.random.default_rng(seed)
    q0 = haar_unitary(rng, n)
    lam = gapped_eigenvalues(rng, n, gap)
    u = _cn_square(rng, n) / math.sqrt(n)
    t0 = np.triu(u, 1) + np.diag(lam)
    a = (q0 @ t0) @ q0.conj().T
    return {"A": np.asfortranarray(a), "Q0": q0, "T0": np.asfortranarray(t0),
            "lam": lam, "n": n, "seed": seed, "gap": gap}


def lp_schur_start(a: np.ndarray) -> np.ndarray:
    """Schur vectors of complex64(A) from LAPACK cgees, widened to complex128.

    These are the low-precision starting basis Q-hat of the refinement; the
    eigenvalue order is whatever cgees returns."""
    import scipy.linalg as sl

    _, z = sl.schur(np.asarray(a, dtype=np.complex64), output="complex")
    return np.asfortranarray(z.astype(np.complex128))


def hp_schur_start(a: np.ndarray) -> np.ndarray:
    """Schur vectors of A from LAPACK zgees (complex128)."""
    import scipy.linalg as sl

    _, z = sl.schur(np.asarray(a, dtype=np.complex128), output="complex")
    return np.asfortranarray(z)


def _walsh_hadamard(n: int) -> np.ndarray:
    h = np.ones((1, 1))
    while h.shape[0] < n:
        h = np.block([[h, h], [h, -h]])
    return h


def hadamard_exact(n: int, seed: int, gap: float = 0.05) -> dict:
    """A test matrix whose Schur decomposition is known exactly in binary.

    n must be 4**k. Q0 = H_n / sqrt(n) is the real orthogonal Walsh-Hadamard
    matrix; its entries are +-2**(-k), exact in binary. T0 has its entries on the
    grid 2**-12 (eigenvalues gap-separated on that grid). Every partial sum of
    Q0 T0 Q0^T lies on the grid 2**(-12-2k) and is bounded by about 5 * 2**(2k),
    which needs at most 15 + 4k bits, so float64 forms A exactly: the stored
    complex128 A equals Q0 T0 Q0^H with no rounding, and (Q0, T0) is its Schur
    decomposition up to column phases."""
    k = int(round(math.log(n, 4)))
    if 4 ** k != n:
        raise ValueError("n must be a power of 4")
    rng = np.random.default_rng(seed)
    grid = 2.0 ** -12
    lam = gapped_eigenvalues(rng, n, gap, grid=grid)
    u = _cn_square(rng, n) / math.sqrt(n)
    u = (np.round(u.real / grid) + 1j * np.round(u.imag / grid)) * grid
    t0 = np.triu(u, 1) + np.diag(lam)
    q0 = _walsh_hadamard(n) * (2.0 ** -k)
    a = (q0 @ t0) @ q0.T
    return {"A": np.asfortranarray(a), "Q0": np.asfortranarray(q0.astype(np.complex128)),
            "T0": np.asfortranarray(t0), "lam": lam, "n": n, "seed": seed}


def perturbed_start(q0: np.ndarray, seed: int, delta: float,
                    to_complex64: bool = True) -> np.ndarray:
    """Q0 + delta * CN(0,1), optionally rounded to complex64: a nearly unitary
    start whose Q^H A Q is nearly upper triangular."""
    rng = np.random.default_rng(seed)
    n = q0.shape[0]
    q = q0 + delta * _cn_square(rng, n)
    if to_complex64:
        q = q.astype(np.complex64).astype(np.complex128)
    return np.asfortranarray(q)


def to_dd(x: np.ndarray, y: np.ndarray):
    """Exact double-double (hi, lo) of x + y for complex128 arrays (Knuth's TwoSum
    on the real and imaginary parts)."""
    def two_sum(a, b):
        s = a + b
        bb = s - a
        err = (a - (s - bb)) + (b - bb)
        return s, err

    hr, lr = two_sum(np.real(x), np.real(y))
    hi_, li = two_sum(np.imag(x), np.imag(y))
    return (np.asfortranarray(hr + 1j * hi_), np.asfortranarray(lr + 1j * li))


def round_mantissa(x: np.ndarray, bits: int) -> np.ndarray:
    """Round the real and imaginary parts of x to `bits` significant bits."""
    def r(v):
        m, e = np.frexp(v)
        return np.ldexp(np.round(m * 2.0 ** bits) / 2.0 ** bits, e)

    return np.asfortranarray(r(np.real(x)) + 1j * r(np.imag(x)))


def wilkinson_companion_dd(n: int = 20):
    """Companion matrix of prod_{i=1..n} (x - i) (Section 3, Example 1), first row
    -c[1:], ones on the subdiagonal. The integer coefficients reach 20! > 2**53,
    so the matrix is returned exactly as a double-double pair (hi, lo)."""
    coeffs = [1]
    for r in range(1, n + 1):
        nxt = coeffs + [0]
        for i in range(1, len(nxt)):
            nxt[i] -= r * coeffs[i - 1]
        coeffs = nxt
    hi = np.zeros((n, n), dtype=np.complex128, order="F")
    lo = np.zeros((n, n), dtype=np.complex128, order="F")
    for j in range(n):
        v = -coeffs[j + 1]
        h = float(v)
        rest = v - int(Fraction(h))
        hi[0, j] = h
        lo[0, j] = float(rest)
        assert int(Fraction(float(rest))) == rest
    for i in range(1, n):
        hi[i, i - 1] = 1.0
    return hi, lo, np.arange(1, n + 1, dtype=np.float64)


def example3_matrix(n: int = 150, seed: int = 0, cond_x: float = 1e5,
                    radius: float = 1e-5, clusters: int = 2, size: int = 10) -> dict:
    """A = X D X^{-1} (Section 3, Example 3): X random with condition number
    cond_x (singular values log-spaced), D real diagonal uniform in [-10, 10]
    except for `clusters` groups of `size` eigenvalues within `radius` of a
    random centre."""
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((n, n)))
    v, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0.0, -math.log10(cond_x), n)
    x = (u * s[None, :]) @ v.T
    d = rng.uniform(-10.0, 10.0, n)
    pos = 0
    for _ in range(clusters):
        c = rng.uniform(-10.0, 10.0)
        d[pos:pos + size] = c + radius * rng.uniform(-1.0, 1.0, size)
        pos += size
    a = x @ np.diag(d) @ np.linalg.inv(x)
    return {"A": np.asfortranarray(a.astype(np.complex128)), "eig": d, "n": n}


def batched_sizes(count: int = 2000, seed: int = 3, lo: int = 16, hi: int = 256) -> np.ndarray:
    """Matrix sizes of the batched workload: lo + integers(0, hi - lo + 1)."""
    return lo + np.random.default_rng(seed).integers(0, hi - lo + 1, size=count)


def real_schur_test_matrix(n: int, seed: int, gap: float = 0.05, n_real: int | None = None) -> dict:
    """Real A = Q0 T0 Q0^T with a real quasi-triangular T0 (the real Schur form).

    The spectrum has the structure of a real Gaussian matrix's: about sqrt(2n/pi)
    real eigenvalues (n_real; n - n_real is made even), the rest in conjugate pairs.
    Draws from `default_rng(seed)`: the n x n real normal matrix behind the Haar
    orthogonal Q0 (QR with the signs of diag(R) moved into Q), the order of the 1 x 1
    and 2 x 2 blocks (a random permutation), then the spectrum (sequential gap
    rejection on complex normal draws, as for the complex generator: a real
    eigenvalue is the real part of a draw, a pair a +- ib needs |b| >= gap / 2), then
    the strictly upper part N(0,1)/sqrt(n). A pair sits in a standardized 2 x 2 block
    [[a, b c], [-b / c, a]] (c drawn in [0.5, 2]); blk[i] = 1 marks a block at rows and
    columns i, i + 1."""
    if n_real is None:
        n_real = min(n, max(1, int(round(math.sqrt(2 * n / math.pi)))))
    if (n - n_real) % 2:
        n_real += 1 if n_real < n else -1
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    q0 = np.asfortranarray(q * np.sign(np.diag(r))[None, :])
    kinds = rng.permutation(np.array([1] * n_real + [2] * ((n - n_real) // 2)))
    lam = []  # eigenvalues in block order
    blk = np.zeros(n, dtype=np.int32)
    t0 = np.zeros((n, n))
    i = 0
    for kind in kinds:
        pair = kind == 2
        while True:
            w = cn(rng, 1)[0]
            cand = [complex(w.real, abs(w.imag)), complex(w.real, -abs(w.imag))] if pair else [complex(w.real, 0.0)]
            if pair and abs(w.imag) < gap / 2:
                continue
            if all(min((abs(c - l) for l in lam), default=np.inf) > gap for c in cand):
                break
        if pair:
            a, b = w.real, abs(w.imag)
            c = 0.5 + 1.5 * rng.random()
            t0[i, i] = t0[i + 1, i + 1] = a
            t0[i, i + 1] = b * c
            t0[i + 1, i] = -b / c
            blk[i] = 1
            lam += cand
            i += 2
        else:
            t0[i, i] = w.real
            lam += cand
            i += 1
    u = rng.standard_normal((n, n)) / math.sqrt(n)
    for j in range(n):
        for k in range(j):
            if not (j == k + 1 and blk[k]):
                t0[k, j] = u[k, j]
    a = (q0 @ t0) @ q0.T
    return {"A": np.asfortranarray(a), "Q0": q0, "T0": np.asfortranarray(t0), "blk": blk,
            "lam": np.array(lam), "n": n, "seed": seed, "gap": gap}


def real_blocks_of(t: np.ndarray) -> np.ndarray:
    """2 x 2 block markers of a real quasi-triangular T (nonzero subdiagonal entries)."""
    n = t.shape[0]
    blk = np.zeros(n, dtype=np.int32)
    i = 0
    while i < n - 1:
        if t[i + 1, i] != 0:
            blk[i] = 1
            i += 2
        else:
            i += 1
    return blk


def lp_real_schur_start(a: np.ndarray):
    """Real Schur vectors of float32(A) from LAPACK sgees, widened to float64, and the
    2 x 2 block markers of the float32 quasi-triangular factor."""
    import scipy.linalg as sl

    t, z = sl.schur(np.asarray(a, dtype=np.float32), output="real")
    return np.asfortranarray(z.astype(np.float64)), real_blocks_of(t)


def _batched_one(item):
    n, seed = item
    g = schur_test_matrix(n, seed=seed)
    return g["A"], lp_schur_start(g["A"])


def batched_inputs(sizes, seed0: int = 10000, workers: int = 16):
    """Matrices and cgees starts of a batch: matrix i is schur_test_matrix(sizes[i],
    seed0 + i) (gaps 0.05) with its complex64 Schur basis. Made in `workers`
    processes (spawned, each with single-threaded BLAS: many small factorizations
    are faster side by side than threaded one by one). Returns [(A, Q-hat)]."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os

    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"
    try:
        items = [(int(n), seed0 + i) for i, n in enumerate(sizes)]
        with cf.ProcessPoolExecutor(max_workers=max(1, workers), mp_context=mp.get_context("spawn")) as ex:
            return list(ex.map(_batched_one, items, chunksize=25))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def continuation_step_dd(a0: np.ndarray, a1: np.ndarray, k: int, steps: int = 64):
    """A(t_k) = A0 + (k/steps) A1 as an exact double-double pair. a1 must carry at
    most 46 significant bits so that (k/steps) * a1 is exact for k < 64."""
    p = (k / steps) * a1
    return to_dd(a0, p)


def continuation_perturbation(n: int, seed: int, scale: float = 1e-3) -> np.ndarray:
    """A1 = scale * CN(0,1), rounded to 46 significant bits."""
    rng = np.random.default_rng(seed)
    return round_mantissa(scale * _cn_square(rng, n), 46)
