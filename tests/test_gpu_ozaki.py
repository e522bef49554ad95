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


# ------------------------------------------------------------ Ozaki scheme II (CRT)

def test_crt_moduli_count(sr):
    """N is the least count of the moduli 256, 255, 253, 251, ... whose product M
    exceeds 8 K 2^(2 bits) (host call, no GPU work)."""
    mods = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193, 191, 181, 179, 173]
    for k, bits in [(4096, 55), (8192, 55), (64, 55), (1000, 30), (100, 12), (65535, 55)]:
        n = sr.lib().sr_crt_moduli(k, bits)
        prod = 1
        for m in mods[:n]:
            prod *= m
        lk = (k - 1).bit_length()
        assert prod >= 2 ** (2 * bits + lk + 3)
        assert n == 1 or prod // mods[n - 1] < 2 ** (2 * bits + lk + 3)
    assert sr.lib().sr_crt_moduli(4096, 55) == 16
    assert sr.lib().sr_crt_moduli(65536, 55) == 0  # int32 sums would not stay exact
    assert sr.lib().sr_crt_moduli(4096, 80) == 0  # more than 20 moduli


@pytest.mark.parametrize("add", [False, True])
@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("shape", [(130, 97, 75), (128, 128, 64), (1, 1, 1), (257, 33, 200)])
def test_crt_exact_on_integers(sr, opa, shape, add):
    """Gaussian integers of at most 21 bits are scaled exactly (55 bits per entry
    hold them), so the residue products and the reconstruction give the exact
    product, which FP64 holds (|sum| < 2^52): bit-exact, ragged tiles, op(A) = A
    and A^H, with and without the added C."""
    m, n, k = shape
    rng = np.random.default_rng(3 * m + 5 * n + 7 * k + opa + 11 * add)
    a = _gauss_int(rng, (k, m) if opa else (m, k), 2**20)
    b = _gauss_int(rng, (k, n), 2**20)
    c0 = _gauss_int(rng, (m, n), 2**30) if add else None
    c = empty(m, n)
    assert sr.sr_crt_zgemm(dev(a), dev(b), c, opa=opa, bits=55, Cin=dev(c0) if add else None) == 0
    ref = (a.conj().T if opa else a) @ b
    if add:
        ref = ref + c0
    assert np.array_equal(host(c), ref)


@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("shape", [(2176, 4096, 64), (4224, 4096, 32), (1024, 1024, 64), (2048, 2048, 32)])
def test_crt_split_tiles_exact_on_integers(sr, opa, shape):
    """Output tiles of 128 x 128 against rounds of block slots (2 per CU): 544 tiles
    (32 past 512) and 1056 (32 past 1024), and launches with no full round, 64 tiles
    (n = 1024, 8 shares each) and 256 (n = 2048, 2 shares). The split tiles go to
    blocks of consecutive moduli whose residues meet in the tile's scratch, and the
    last share reconstructs; the product stays bit-exact."""
    m, n, k = shape
    rng = np.random.default_rng(m + n + k + opa)
    a = _gauss_int(rng, (k, m) if opa else (m, k), 2**20)
    b = _gauss_int(rng, (k, n), 2**20)
    c = empty(m, n)
    assert sr.sr_crt_zgemm(dev(a), dev(b), c, opa=opa, bits=55) == 0
    ref = (a.conj().T if opa else a) @ b
    assert np.array_equal(host(c), ref)


def _crt_bound(a_op, b, bits):
    """Entrywise bound of the CRT product: each entry of a row (column) is rounded to
    a multiple of 2^t with 2^t <= 2^-bits of twice the row (column) maximum (an
    error of 2^(t-1) in re and in im), plus the final rounding to FP64."""
    def scale(mx):
        e = np.where(mx > 0, np.frexp(mx)[1], 0)
        return np.ldexp(1.0, e - bits)  # 2^t
    ra = scale(np.maximum(np.abs(a_op.real), np.abs(a_op.imag)).max(axis=1))
    cb = scale(np.maximum(np.abs(b.real), np.abs(b.imag)).max(axis=0))
    da = np.sqrt(2) * 0.5 * ra[:, None] * np.ones_like(a_op.real)
    db = np.sqrt(2) * 0.5 * cb[None, :] * np.ones_like(b.real)
    return da @ np.abs(b) + np.abs(a_op) @ db + da @ db


@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("bits", [55, 30])
def test_crt_random_within_bound_of_quad(sr, opa, bits):
    rng = np.random.default_rng(41 + opa + bits)
    m, n, k = 150, 131, 260
    a = rand_c(rng, (k, m) if opa else (m, k))
    a[3] *= 1e-9  # rows and columns of very different scales
    b = rand_c(rng, (k, n))
    b[:, 7] *= 1e12
    c = empty(m, n)
    assert sr.sr_crt_zgemm(dev(a), dev(b), c, opa=opa, bits=bits) == 0
    chi, clo = oracle.gemm(a, b, opa=opa).to_dd()
    err = np.abs((host(c) - chi) - clo)
    a_op = a.conj().T if opa else a
    bound = _crt_bound(a_op, b, bits) + 1.01 * U64 * np.abs(chi)
    assert np.all(err <= bound), (err / bound).max()
    # the bound is met with little room: the error is of the order of the input rounding
    if bits == 30:
        assert np.median(err / bound) >= 1e-3


def test_crt_n2048_rows_against_quad(sr):
    """A product with 256 output tiles of 128 x 128 (every CU busy): sampled rows
    against the binary128 product, and more accurate than native FP64."""
    rng = np.random.default_rng(9)
    n = 2048
    a, b = rand_c(rng, (n, n)), rand_c(rng, (n, n))
    c = empty(n, n)
    assert sr.sr_crt_zgemm(dev(a), dev(b), c, bits=55) == 0
    rows = np.sort(rng.choice(n, 6, replace=False))
    chi, clo = oracle.gemm(np.asfortranarray(a[rows]), b).to_dd()
    err = np.abs((host(c)[rows] - chi) - clo)
    bound = _crt_bound(a[rows], b, 55) + 1.01 * U64 * np.abs(chi)
    assert np.all(err <= bound)
    cf = empty(n, n)
    assert sr.sr_zgemm(dev(a), dev(b), cf) == 0
    err64 = np.abs((host(cf)[rows] - chi) - clo)
    assert np.linalg.norm(err) < np.linalg.norm(err64)
