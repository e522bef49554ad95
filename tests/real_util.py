"""Test inputs for the real Schur variant (shared by the oracle pins and the GPU
tests): quasi-upper-triangular matrices with 2 x 2 blocks, the block strictly lower
mask, and exactly representable real Schur problems."""
import numpy as np

import synth


def quasi_upper(rng, sizes, dyadic=False):
    """A real block upper triangular T with diagonal blocks of the given orders:
    2 x 2 blocks [[a, b], [c, a]] with b c < 0 (a complex pair), distinct eigenvalues."""
    n = sum(sizes)
    t = np.triu(rng.standard_normal((n, n)))
    blk = np.zeros(n, dtype=np.int32)
    i = 0
    for k, s in enumerate(sizes):
        if s == 2:
            a, b, c = float(k + 1), 0.5 + rng.random(), -(0.5 + rng.random())
            t[i, i] = t[i + 1, i + 1] = a
            t[i, i + 1], t[i + 1, i] = b, c
            blk[i] = 1
        else:
            t[i, i] = k + 1.5
        i += s
    if dyadic:
        t = np.round(t * 64) / 64
    return t, blk


def block_lower_mask(n, blk):
    """Entries of the block strictly lower part: below the diagonal, minus the
    subdiagonal entry of each 2 x 2 block."""
    m = np.tril(np.ones((n, n), dtype=bool), -1)
    if blk is not None:
        for i in range(n - 1):
            if blk[i]:
                m[i + 1, i] = False
    return m


def block_sizes(blk):
    n = len(blk)
    out, i = [], 0
    while i < n:
        s = 2 if blk[i] else 1
        out.append((i, s))
        i += s
    return out


def exact_real_problem(n, seed):
    """A = Q0 T0 Q0^T exact in binary: Q0 the scaled Walsh-Hadamard matrix (entries
    +-2^-k), T0 real quasi-triangular on the grid 2^-8 with 2 x 2 blocks for complex
    pairs; every product stays on a fine dyadic grid with few bits."""
    rng = np.random.default_rng(seed)
    sizes = []
    while sum(sizes) < n:
        sizes.append(2 if sum(sizes) + 2 <= n and rng.random() < 0.5 else 1)
    t0, blk = quasi_upper(rng, sizes, dyadic=True)
    t0 = t0 * 0.25  # eigenvalues spread less
    h = synth.hadamard_exact(n, seed=seed)["Q0"].real
    a = (h @ t0) @ h.T
    return a, h, t0, blk


def rotated(q0, seed, delta):
    """q0 exp(K) for a random skew-symmetric K of size delta (a real orthogonal
    perturbation of the start)."""
    rng = np.random.default_rng(seed)
    n = q0.shape[0]
    x = delta * rng.standard_normal((n, n))
    k = (x - x.T) / 2
    w, v = np.linalg.eigh(1j * k)
    return np.asfortranarray((q0 @ (v @ np.diag(np.exp(-1j * w)) @ v.conj().T)).real)
