"""GPU parity of the Ozaki split product (INT8 MFMA) against exact arithmetic and
the binary128 oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import U64, dev, empty, gemm_bound, host, rand_c

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sr():
    import torch

    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _gauss_int(rng, shape, lim=256):
    return np.asfortranarray(rng.integers(-lim, lim + 1, shape) + 1j * rng.integers(-lim, lim + 1, shape))


@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("shape", [(130, 97, 75), (64, 64, 64), (1, 1, 1), (200, 33, 129)])
def test_ozaki_exact_on_integers(sr, opa, shape):
    # 9-bit integers fit in two 8-bit digits (the row scale leaves the top digit
    # below 127); with every slice pair kept the product is exact and so is its
    # FP64 combination
    m, n, k = shape
    rng = np.random.default_rng(m + 7 * n + 13 * k)
    a = _gauss_int(rng, (k, m) if opa else (m, k))
    b = _gauss_int(rng, (k, n))
    c = empty(m, n)
    assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, opa=opa, slices_a=2, slices_b=2, dmax=4) == 0
    ref = (a.conj().T if opa else a) @ b
    assert np.array_equal(host(c), ref)


@pytest.mark.parametrize("opa", [0, 1])
def test_ozaki_fp64_faithful_with_7_slices(sr, opa):
    rng = np.random.default_rng(21 + opa)
    m, n, k = 150, 131, 260
    a = rand_c(rng, (k, m) if opa else (m, k))
    b = rand_c(rng, (k, n))
    c = empty(m, n)
    assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, opa=opa, slices_a=7, slices_b=7, dmax=8) == 0
    chi, clo = oracle.gemm(a, b, opa=opa).to_dd()
    err = np.abs((host(c) - chi) - clo)
    aa = np.abs(a.conj().T if opa else a)
    assert np.all(err <= gemm_bound(aa, np.abs(b), k, U64))


def test_ozaki_error_decreases_with_slices(sr):
    rng = np.random.default_rng(5)
    n = 256
    a, b = rand_c(rng, (n, n)), rand_c(rng, (n, n))
    chi, clo = oracle.gemm(a, b).to_dd()
    scale = np.linalg.norm(np.abs(a) @ np.abs(b))
    errs = []
    for s in (3, 4, 5, 6):
        c = empty(n, n)
        assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, slices_a=s, slices_b=s, dmax=s + 1) == 0
        errs.append(np.linalg.norm((host(c) - chi) - clo) / scale)
    for e_prev, e_next in zip(errs[:-1], errs[1:]):
        assert e_next < e_prev / 60  # about 8 bits per slice
    assert errs[0] < 2.0 ** -(8 * 3 - 6)


def _carry_ints(rng, shape):
    """Integers k 2^14 + r up to 2^20 + 8160 in magnitude. With that maximum in every
    row and column the scale is 2^22, the first raw digit is about k and the second
    r / 64 rounded to nearest even: r = 8160 gives 127.5 -> 128 (a carry into the
    first digit), r = -8192 and -8160 give -128 (a carry of the negated digits),
    r = 8128 gives 127."""
    k = rng.integers(-64, 64, shape) * 2**14
    r = rng.choice([8160, 8128, 8144, 8159, -8192, -8160, 8136, 0, 63], shape)
    return k + r


@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("shape", [(96, 80, 70), (2085, 2048, 66)])
def test_ozaki_exact_with_digit_carries(sr, opa, shape):
    m, n, k = shape
    rng = np.random.default_rng(11 + opa + m)
    ar, ai = _carry_ints(rng, (k, m) if opa else (m, k)), _carry_ints(rng, (k, m) if opa else (m, k))
    br, bi = _carry_ints(rng, (k, n)), _carry_ints(rng, (k, n))
    # every row of op(A) and column of B holds the maximum 2^20 + 8160 once
    big = 2**20 + 8160
    if opa:
        ar[0, :] = big
    else:
        ar[:, 0] = big
    br[0, :] = big
    a = np.asfortranarray(ar + 1j * ai)
    b = np.asfortranarray(br + 1j * bi)
    c = empty(m, n)
    assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, opa=opa, slices_a=3, slices_b=3, dmax=6) == 0
    ref = (a.conj().T if opa else a) @ b  # |entries| < 2^47: exact in FP64
    rows = np.arange(m) if m < 200 else np.random.default_rng(2).choice(m, 40, replace=False)
    assert np.array_equal(host(c)[rows], ref[rows])


def test_ozaki_add_epilogue_and_validation(sr):
    rng = np.random.default_rng(3)
    m, n, k = 70, 90, 40
    a, b, c0 = _gauss_int(rng, (m, k)), _gauss_int(rng, (k, n)), _gauss_int(rng, (m, n))
    c = empty(m, n)
    assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, slices_a=2, slices_b=2, dmax=4, Cin=dev(c0)) == 0
    assert np.array_equal(host(c), c0 + a @ b)
    assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, slices_a=0, slices_b=2) == -1


# Outputs with at least one 128 x 128 tile per CU (256 tiles) and digit sets
# other than the FP64 tier's take the large-tile kernel (two int32 accumulators
# per output, FP64 partial sums in scratch between folds).

@pytest.mark.parametrize("opa", [0, 1])
def test_ozaki_large_tiles_exact_on_integers(sr, opa):
    m, n, k = 2085, 2048, 130  # ragged rows, a ragged K-tile
    rng = np.random.default_rng(90 + opa)
    a = _gauss_int(rng, (k, m) if opa else (m, k))
    b = _gauss_int(rng, (k, n))
    c0 = _gauss_int(rng, (m, n))
    c = empty(m, n)
    assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, opa=opa, slices_a=2, slices_b=2, dmax=4, Cin=dev(c0)) == 0
    ref = c0 + (a.conj().T if opa else a) @ b
    assert np.array_equal(host(c), ref)


def test_ozaki_large_tiles_segmented_diagonal(sr):
    # k = 8256: 258 K-steps of 32 in the all-pairs kernel, folded in two
    # segments of at most 256
    m = n = 2048
    k = 8256
    rng = np.random.default_rng(17)
    a = _gauss_int(rng, (m, k))
    b = _gauss_int(rng, (k, n))
    c = empty(m, n)
    assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, slices_a=7, slices_b=7, dmax=8) == 0
    rows = np.random.default_rng(3).choice(m, 48, replace=False)
    assert np.array_equal(host(c)[rows], a[rows] @ b)


# slices 7 (pairs up to s + t = 8) take the all-pairs kernel, 8 the large-tile one
@pytest.mark.parametrize("slices", [7, 8])
@pytest.mark.parametrize("opa", [0, 1])
def test_ozaki_large_tiles_fp64_faithful(sr, opa, slices):
    m = n = 2048
    k = 192
    rng = np.random.default_rng(40 + opa)
    a = rand_c(rng, (k, m) if opa else (m, k))
    b = rand_c(rng, (k, n))
    c = empty(m, n)
    assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, opa=opa, slices_a=slices, slices_b=slices, dmax=slices + 1) == 0
    rows = np.random.default_rng(4).choice(m, 32, replace=False)
    asub = np.asfortranarray(a[:, rows] if opa else a[rows])
    chi, clo = oracle.gemm(asub, b, opa=opa).to_dd()
    err = np.abs((host(c)[rows] - chi) - clo)
    aa = np.abs(asub.conj().T if opa else asub)
    assert np.all(err <= gemm_bound(aa, np.abs(b), k, U64))


# The FP64 tier's digit sets (S digits per operand, pairs up to s + t = S + 1) on
# outputs with a 64 x 64 tile per CU take the all-pairs kernel: every slice of a
# K-step staged at once, one int32 accumulator pair per diagonal.

def _one_digit_ints(rng, shape):
    # |x| <= 63: the scale leaves x 2^(8-e) an integer below 126, a single digit
    return rng.integers(-63, 64, shape)


@pytest.mark.parametrize("add", [False, True])
@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("S", [1, 3, 7])
def test_ozaki_allpairs_exact_on_integers(sr, S, opa, add):
    # op(A) of 9-bit integers needs two digits (one for S = 1: 6-bit), B one, so
    # the pairs (s, 1), s <= 2, that the triangle keeps give the exact product
    m, n, k = 2085, 2048, 130  # ragged rows, a ragged K-tile
    rng = np.random.default_rng(500 + 10 * S + 2 * opa + add)
    shp = (k, m) if opa else (m, k)
    if S == 1:
        a = np.asfortranarray(_one_digit_ints(rng, shp) + 1j * _one_digit_ints(rng, shp))
    else:
        a = _gauss_int(rng, shp)
    b = np.asfortranarray(_one_digit_ints(rng, (k, n)) + 1j * _one_digit_ints(rng, (k, n)))
    c0 = _gauss_int(rng, (m, n)) if add else None
    c = empty(m, n)
    rc = sr.sr_ozaki_zgemm(dev(a), dev(b), c, opa=opa, slices_a=S, slices_b=S, dmax=S + 1,
                           Cin=dev(c0) if add else None)
    assert rc == 0
    ref = (a.conj().T if opa else a) @ b
    if add:
        ref = ref + c0
    assert np.array_equal(host(c), ref)


@pytest.mark.parametrize("opa", [0, 1])
def test_ozaki_allpairs_exact_with_digit_carries(sr, opa):
    # op(A) with three digits and carries (see _carry_ints), B with one digit:
    # S = 3 keeps the pairs (s, 1) the product needs
    m, n, k = 1100, 1030, 66
    rng = np.random.default_rng(77 + opa)
    shp = (k, m) if opa else (m, k)
    ar, ai = _carry_ints(rng, shp), _carry_ints(rng, shp)
    big = 2**20 + 8160
    if opa:
        ar[0, :] = big
    else:
        ar[:, 0] = big
    a = np.asfortranarray(ar + 1j * ai)
    b = np.asfortranarray(_one_digit_ints(rng, (k, n)) + 1j * _one_digit_ints(rng, (k, n)))
    c = empty(m, n)
    assert sr.sr_ozaki_zgemm(dev(a), dev(b), c, opa=opa, slices_a=3, slices_b=3, dmax=4) == 0
    ref = (a.conj().T if opa else a) @ b
    assert np.array_equal(host(c), ref)
