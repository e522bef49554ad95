"""The lp products on INT8 digits (sr_opts.lp_digits, stage call sr_ozaki_cgemm):
complex64 operands split into balanced 8-bit digits, exact int32 pair sums, FP64
fold, one rounding to complex64; Hermitian and skew-Hermitian outputs over the
upper tiles."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import U64, dev, empty, host

pytestmark = pytest.mark.gpu

N = 1024  # the kernel takes at least 256 output tiles of 64 x 64


@pytest.fixture(scope="module")
def sr():
    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _c64(x):
    return np.asfortranarray(x.astype(np.complex64))


def _prod(sr, a, b, slices, herm=0):
    c = empty(a.shape[0], b.shape[1], c64=True)
    rc = sr.sr_ozaki_cgemm(dev(a), dev(b), c, slices=slices, herm=herm)
    torch.cuda.synchronize()
    assert rc == 0, rc
    return host(c)


@pytest.mark.parametrize("slices", [1, 3])
def test_exact_on_small_integers(sr, slices):
    """Entries below 126 in magnitude are one digit each, and every sum stays below
    2^24: the product is exact in complex64."""
    rng = np.random.default_rng(slices)
    shape = (N, 1040)
    a = _c64(rng.integers(-63, 64, shape) + 1j * rng.integers(-63, 64, shape))
    b = _c64(rng.integers(-63, 64, shape[::-1]) + 1j * rng.integers(-63, 64, shape[::-1]))
    c = _prod(sr, a, b, slices)
    exact = a.astype(np.complex128) @ b.astype(np.complex128)
    assert np.array_equal(c.astype(np.complex128), exact)


def _bound(a, b, S):
    """Digit truncation of both operands and the dropped pairs s + t > S + 1, per
    entry, plus the final rounding to complex64 (applied by the caller)."""
    ma = np.max(np.maximum(np.abs(a.real), np.abs(a.imag)), axis=1).astype(np.float64)
    mb = np.max(np.maximum(np.abs(b.real), np.abs(b.imag)), axis=0).astype(np.float64)
    k = a.shape[1]
    return (16 + 8 * S) * k * 2.0 ** (-8 * S) * np.outer(ma, mb)


def test_random_within_digit_bound(sr):
    rng = np.random.default_rng(5)
    a = _c64(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    b = _c64(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    exact = a.astype(np.complex128) @ b.astype(np.complex128)
    errs = {}
    for S in (2, 3, 4):
        c = _prod(sr, a, b, S).astype(np.complex128)
        err = np.abs(c - exact)
        assert np.all(err <= _bound(a, b, S) + 2.0 ** -23 * np.abs(exact)), S
        errs[S] = float(err.max())
    # 8 bits per digit until the complex64 rounding floor
    assert errs[3] <= errs[2] * 2.0 ** -6
    assert errs[4] <= errs[3]
    # three digits: within a small factor of the FP32 MFMA product's error
    c32 = empty(N, N, c64=True)
    assert sr.sr_cgemm(dev(a), dev(b), c32) == 0
    e32 = float(np.abs(host(c32).astype(np.complex128) - exact).max())
    assert errs[3] <= 4 * e32, (errs, e32)


def _mirrored(c, sign):
    """Off the diagonal c[j, i] = sign conj(c[i, j]) bit for bit."""
    off = ~np.eye(c.shape[0], dtype=bool)
    return np.array_equal(c[off], (sign * c.conj().T)[off])


def test_hermitian_and_skew_outputs(sr):
    """W skew-Hermitian: W^2 (herm = 1) is Hermitian and W^2 W (herm = -1)
    skew-Hermitian, off the diagonal exactly (each element of the upper triangle
    stored with its mirror); the diagonal keeps its computed value, whose imaginary
    (real) part is rounding; the upper triangles equal the full products' bit for
    bit (the same digits and sums per element)."""
    rng = np.random.default_rng(6)
    l = np.tril(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)), -1) * 1e-3
    w = _c64(l - l.conj().T)
    iu = np.triu_indices(N)
    w2 = _prod(sr, w, w, 3, herm=1)
    assert _mirrored(w2, 1)
    d2 = np.diag(w2)
    assert np.all(np.abs(d2.imag) <= np.diag(_bound(w, w, 3)))
    full = _prod(sr, w, w, 3)
    assert np.array_equal(w2[iu], full[iu])
    w3 = _prod(sr, w2, w, 3, herm=-1)
    assert _mirrored(w3, -1)
    d3 = np.diag(w3)
    assert np.all(np.abs(d3.real) <= np.diag(_bound(w2, w, 3)))
    full3 = _prod(sr, w2, w, 3)
    assert np.array_equal(w3[iu], full3[iu])


def test_arguments(sr):
    import ctypes

    L = sr.lib()
    a = dev(_c64(np.eye(N)))
    c = empty(N, N, c64=True)
    need = int(L.sr_ozaki_ws_bytes(N, N, N, 3, 3))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    w = ctypes.c_void_p(ws.data_ptr())
    p = lambda t: ctypes.c_void_p(t.data_ptr())

    def call(m=N, n=N, k=N, S=3, herm=0, nb=need):
        return L.sr_ozaki_cgemm(m, n, k, p(a), N, p(a), N, p(c), N, S, herm, w, nb, None)

    assert call() == 0
    assert call(m=512, n=512) == -1  # below 256 output tiles
    assert call(S=0) == -1 and call(S=8) == -1
    assert call(herm=2) == -1 and call(m=N, n=N - 64, herm=1) == -1
    assert call(nb=need - 1) == -3


@pytest.mark.parametrize("mode", ["ozaki_i8_all", "ozaki_crt"])
def test_refinement_with_lp_digits(sr, mode):
    """n = 1024 (gaps 0.05, cgees start): the same passes as with FP32 lp products,
    binary128 residual and orthogonality on 64 rows."""
    g = synth.schur_test_matrix(N, seed=1)
    a = g["A"]
    qh = synth.lp_schur_start(a)
    infos = {}
    for lp in (0, 4):
        q, t = dev(qh), empty(N, N)
        infos[lp] = sr.schur_refine(dev(a), q, t, iters=6, tol=1e-15, gemm=mode, lp_digits=lp)
        assert infos[lp]["status"] == "OK" and infos[lp]["iters"] <= 5, (lp, infos[lp])
        rows = np.random.default_rng(20001).choice(N, 64, replace=False)
        ev = oracle.evaluate_rows(a, host(q), rows)
        assert ev["stril"] <= 1e-15, (lp, ev)
        assert ev["orth"] <= 4 * U64 * np.sqrt(N) * 10, (lp, ev)
    assert infos[4]["iters"] == infos[0]["iters"], infos
    assert infos[4]["lp_products"] == infos[0]["lp_products"]


def test_option_validation(sr):
    g = synth.schur_test_matrix(64, seed=2)
    a, qh = g["A"], synth.lp_schur_start(g["A"])
    run = lambda **kw: sr.schur_refine(dev(a), dev(qh), empty(64, 64), iters=2, tol=1e-15, **kw)["status"]
    assert run(gemm="fp64", lp_digits=3) == "EINVAL"  # the native form keeps FP32
    assert run(gemm="ozaki_crt", lp_digits=8) == "EINVAL"
    # below the kernel's size the FP32 products are used
    assert run(gemm="ozaki_crt", lp_digits=3) in ("OK", "NOT_CONVERGED")
