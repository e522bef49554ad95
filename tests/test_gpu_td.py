"""The triple-double tier (schur_refine_td: three doubles per number, FP64 lp)
against exact rational arithmetic, which reaches past the binary128 oracle."""
from fractions import Fraction

import numpy as np
import pytest

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


def _exact(parts):
    """Entries of a sum of float64 arrays as exact rationals (real, imag) lists."""
    re = np.zeros(parts[0].shape, dtype=object)
    im = np.zeros(parts[0].shape, dtype=object)
    for p in parts:
        re = re + np.vectorize(Fraction)(p.real)
        im = im + np.vectorize(Fraction)(p.imag)
    return re, im


def _cmatmul(ar, ai, br, bi):
    """Exact complex product of object (Fraction) matrices."""
    return ar.dot(br) - ai.dot(bi), ar.dot(bi) + ai.dot(br)


def _refine(sr, a, qh, **kw):
    n = a.shape[0]
    z = np.zeros_like(a)
    As = [dev(a), dev(z), dev(z)]
    Qs = [dev(qh), dev(z), dev(z)]
    Ts = [empty(n, n), empty(n, n), empty(n, n)]
    info = sr.schur_refine_td(As, Qs, Ts, **kw)
    return [host(q) for q in Qs], [host(t) for t in Ts], info


@pytest.mark.parametrize("n", [16, 64])
def test_td_exact_hadamard_schur_form(sr, n):
    """A = Q0 T0 Q0^H exact in binary, started 1e-6 from Q0: Q0^H Q is diagonal and
    unimodular, and diag(T) equals diag(T0), to 1e-40 in exact arithmetic."""
    h = synth.hadamard_exact(n, seed=n + 5)
    qh = synth.perturbed_start(h["Q0"], seed=4, delta=1e-6, to_complex64=False)
    q, t, info = _refine(sr, h["A"], qh, iters=6, tol=1e-40)
    assert info["status"] == "OK" and info["iters"] <= 5, info
    q0 = h["Q0"].real  # entries +-2^-k: exact
    qr, qi = _exact(q)
    q0f = np.vectorize(Fraction)(q0)
    cr, ci = q0f.T.dot(qr), q0f.T.dot(qi)
    off = max(abs(float(cr[i, j])) + abs(float(ci[i, j])) for i in range(n) for j in range(n) if i != j)
    assert off <= 1e-40, off
    dev1 = max(abs(float(cr[i, i] * cr[i, i] + ci[i, i] * ci[i, i] - 1)) for i in range(n))
    assert dev1 <= 1e-40, dev1
    tr, ti = _exact(t)
    lam = h["lam"]
    err = max(abs(float(tr[i, i] - Fraction(lam[i].real))) + abs(float(ti[i, i] - Fraction(lam[i].imag)))
              for i in range(n))
    assert err <= 1e-40, err
    assert not any(t[0][i, j] for i in range(n) for j in range(i))


def test_td_random_n32_exact_residual(sr):
    """n = 32 (gaps 0.05) from the complex128 Schur basis of A (LAPACK zgees): at most
    4 passes to 1e-40, each pass gaining at least 12 decades; the exact residual
    ||stril(Q^H A Q)||_F / ||A||_F and ||Q^H Q - I||_F below 1e-40."""
    n = 32
    g = synth.schur_test_matrix(n, seed=77)
    a = g["A"]
    qh = synth.hp_schur_start(a)
    q, t, info = _refine(sr, a, qh, iters=6, tol=1e-40)
    assert info["status"] == "OK" and info["iters"] <= 4, info
    h = info["resid_hist"]
    for k in range(1, len(h)):
        assert h[k] <= 1e-12 * h[k - 1] or h[k] <= 1e-40, h
    qr, qi = _exact(q)
    ar, ai = _exact([a])
    pr, pi = _cmatmul(ar, ai, qr, qi)
    # Q^H P
    mr = qr.T.dot(pr) + qi.T.dot(pi)
    mi = qr.T.dot(pi) - qi.T.dot(pr)
    stril = sum(float(mr[i, j] ** 2 + mi[i, j] ** 2) for i in range(n) for j in range(i))
    assert np.sqrt(stril) / np.linalg.norm(a) <= 1e-40
    gr = qr.T.dot(qr) + qi.T.dot(qi)
    gi = qr.T.dot(qi) - qi.T.dot(qr)
    orth = sum(float((gr[i, j] - (1 if i == j else 0)) ** 2 + gi[i, j] ** 2) for i in range(n) for j in range(n))
    assert np.sqrt(orth) <= 1e-40, np.sqrt(orth)
    # T holds triu(Q^H A Q): its entries match to the triple-double rounding
    tr, ti = _exact(t)
    terr = max(abs(float(tr[i, j] - mr[i, j])) + abs(float(ti[i, j] - mi[i, j])) for i in range(n) for j in range(i, n))
    assert terr <= 1e-42 * np.linalg.norm(a), terr


def test_td_arguments(sr):
    g = synth.schur_test_matrix(8, seed=3)
    z = np.zeros_like(g["A"])
    As = [dev(g["A"]), dev(z), dev(z)]
    Qs = [dev(synth.hp_schur_start(g["A"])), dev(z), dev(z)]
    Ts = [empty(8, 8), empty(8, 8), empty(8, 8)]
    assert sr.schur_refine_td(As, Qs, Ts, gemm="ozaki_i8")["rc"] == -4  # SR_ENOSYS
    assert sr.schur_refine_td(As, Qs, Ts, slices=12)["rc"] == -1  # SR_EINVAL: too few digits
    # past the product kernel's 32-bit plane offsets (rejected before any access)
    import ctypes

    arr = lambda xs: (ctypes.c_void_p * 3)(*[x.data_ptr() for x in xs])
    info = sr.SrInfo()
    # n = 6000: (20 + 4) 3 n^2 > 2^31 (20 digits), and (22 + 4) 3 n^2 too (22 digits)
    assert sr.lib().schur_refine_td(arr(As), arr(Qs), arr(Ts), 6000, 2, 1e-40, None, ctypes.byref(info)) == -1
    ws = sr.lib().sr_ozaki_ws_bytes(8, 8, 8, 22, 22)
    assert sr.lib().sr_ozaki_zgemm_td(0, 6000, 6000, 6000, arr(As), 6000, arr(As), 6000, None, 1, arr(Ts), 6000,
                                      22, ctypes.c_void_p(Ts[0].data_ptr()), ws, None) == -1


# ---------------------------------------------------------------- the product stage call

def _td_rand(rng, m, n, terms=3):
    """Three-term operands: a complex128 leading term, then terms below its ulp."""
    hi = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    z = np.zeros_like(hi)
    if terms == 1:
        return [hi, z, z]
    mid = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * 2.0 ** -54
    lo = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * 2.0 ** -108
    return [hi, mid, lo]


def _td_product(sr, As, Bs, opa, m, n, cins=None, slices=22):
    import torch

    Cs = [empty(m, n) for _ in range(3)]
    rc = sr.sr_ozaki_zgemm_td([dev(a) for a in As], [dev(b) for b in Bs], Cs, opa=opa, slices=slices,
                              Cins=[dev(c) for c in cins] if cins is not None else None)
    torch.cuda.synchronize()
    assert rc == 0, rc
    return [host(c) for c in Cs]


def _op_exact(parts, opa):
    r, i = _exact(parts)
    return (r.T, -i.T) if opa else (r, i)


def _scale_bound(As, Bs, opa, k):
    """2^-150 k max_row |op(A)| max_col |B| per entry (the digits' and the three-term
    accumulation's reach)."""
    a = np.abs(As[0].real) + np.abs(As[0].imag)
    if opa:
        a = a.T
    b = np.abs(Bs[0].real) + np.abs(Bs[0].imag)
    return 2.0 ** -150 * k * np.outer(a.max(axis=1), b.max(axis=0))


@pytest.mark.parametrize("shape", [(16, 16, 16), (70, 65, 33)])
@pytest.mark.parametrize("opa", [0, 1])
def test_td_product_exact_on_doubles(sr, shape, opa):
    """Operands that are plain doubles: every digit product and pair sum is exact and
    22 digits hold every double of a row, so the three-term result is the exact product."""
    m, n, k = shape
    rng = np.random.default_rng(m + 7 * opa)
    As = _td_rand(rng, k if opa else m, m if opa else k, terms=1)
    Bs = _td_rand(rng, k, n, terms=1)
    C = _td_product(sr, As, Bs, opa, m, n)
    ar, ai = _op_exact(As, opa)
    br, bi = _exact(Bs)
    er, ei = _cmatmul(ar, ai, br, bi)
    cr, ci = _exact(C)
    assert (cr == er).all() and (ci == ei).all()


@pytest.mark.parametrize("shape", [(16, 16, 16), (70, 65, 33)])
@pytest.mark.parametrize("opa", [0, 1])
def test_td_product_three_term_operands(sr, shape, opa):
    m, n, k = shape
    rng = np.random.default_rng(100 + m + opa)
    As = _td_rand(rng, k if opa else m, m if opa else k)
    Bs = _td_rand(rng, k, n)
    C = _td_product(sr, As, Bs, opa, m, n)
    ar, ai = _op_exact(As, opa)
    br, bi = _exact(Bs)
    er, ei = _cmatmul(ar, ai, br, bi)
    cr, ci = _exact(C)
    bound = _scale_bound(As, Bs, opa, k)
    err = np.vectorize(lambda x: abs(float(x)))(cr - er) + np.vectorize(lambda x: abs(float(x)))(ci - ei)
    assert (err <= bound).all(), float((err / bound).max())


@pytest.mark.parametrize("where", [1, 2])
def test_td_product_cancellation_leading_term(sr, where):
    """A = [X X], B = [Y; -Y + D] with D in the middle (2^-60) or lowest (2^-115) term:
    the pair sums cancel down to X D. The result's terms must still be renormalized:
    C[0] is X D rounded to double and C[1] the remainder rounded, each up to the
    accumulation bound 2^-150 k max|A| max|B| (below 2^-30 of |X D| here), and the sum
    of all three is exact up to the same bound."""
    rng = np.random.default_rng(40 + where)
    m, h, n = 24, 12, 20
    X = rng.standard_normal((m, h)) + 1j * rng.standard_normal((m, h))
    Y = rng.standard_normal((h, n)) + 1j * rng.standard_normal((h, n))
    Dm = (rng.standard_normal((h, n)) + 1j * rng.standard_normal((h, n))) * (2.0 ** -60 if where == 1 else 2.0 ** -115)
    z = np.zeros((m, 2 * h), dtype=np.complex128)
    As = [np.hstack([X, X]), z, z]
    b0 = np.vstack([Y, -Y])
    zb = np.zeros_like(b0)
    bd = np.vstack([np.zeros_like(Y), Dm])
    Bs = [b0, bd, zb] if where == 1 else [b0, zb, bd]
    C = _td_product(sr, As, Bs, 0, m, n)
    xr, xi = _exact([X])
    dr, di = _exact([Dm])
    vr, vi = _cmatmul(xr, xi, dr, di)  # the exact value X D
    bound = _scale_bound(As, Bs, 0, 2 * h)
    for part, vv in ((0, vr), (1, vi)):
        v = np.vectorize(float)(vv)
        c0 = C[0].real if part == 0 else C[0].imag
        c1 = C[1].real if part == 0 else C[1].imag
        assert np.all(np.abs(c0 - v) <= 2.0 ** -52 * np.abs(v) + bound), float(np.max(np.abs(c0 - v) / np.abs(v)))
        rem = np.vectorize(float)(vv - np.vectorize(Fraction)(c0))
        assert np.all(np.abs(c1 - rem) <= 2.0 ** -50 * np.abs(rem) + bound)
    cr, ci = _exact(C)
    err = np.vectorize(lambda x: abs(float(x)))(cr - vr) + np.vectorize(lambda x: abs(float(x)))(ci - vi)
    assert (err <= bound).all()


def test_td_product_add_epilogue(sr):
    """C = A B + Cin with a three-term Cin equal to -(A B) in its leading terms: the
    sum keeps the exact difference."""
    rng = np.random.default_rng(9)
    m, n, k = 33, 31, 20
    As = _td_rand(rng, m, k)
    Bs = _td_rand(rng, k, n)
    ar, ai = _exact(As)
    br, bi = _exact(Bs)
    er, ei = _cmatmul(ar, ai, br, bi)
    # Cin: minus the product rounded to double-double, plus a third term of its own
    c_hi = -(np.vectorize(float)(er) + 1j * np.vectorize(float)(ei))
    rr = er + np.vectorize(Fraction)(c_hi.real)
    ri = ei + np.vectorize(Fraction)(c_hi.imag)
    c_mid = -(np.vectorize(float)(rr) + 1j * np.vectorize(float)(ri))
    c_lo = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * 2.0 ** -120
    cins = [c_hi, c_mid, c_lo]
    C = _td_product(sr, As, Bs, 0, m, n, cins=cins)
    cinr, cini = _exact(cins)
    vr, vi = er + cinr, ei + cini
    cr, ci = _exact(C)
    bound = _scale_bound(As, Bs, 0, k) + 2.0 ** -155 * np.abs(c_hi)
    err = np.vectorize(lambda x: abs(float(x)))(cr - vr) + np.vectorize(lambda x: abs(float(x)))(ci - vi)
    assert (err <= bound).all(), float((err / bound).max())
    # the leading term is the difference rounded to double
    v = np.vectorize(float)(vr)
    assert np.all(np.abs(C[0].real - v) <= 2.0 ** -52 * np.abs(v) + 2.0 ** -150 * np.abs(c_hi.real) * 64)


def test_td_product_arguments(sr):
    import ctypes

    import torch

    lib = sr.lib()
    t = [dev(np.eye(8, dtype=np.complex128)) for _ in range(3)]
    ptrs = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in t])
    need = int(lib.sr_ozaki_ws_bytes(8, 8, 8, 22, 22))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    w = ctypes.c_void_p(ws.data_ptr())
    call = lambda k=8, s=22, nb=need, C=ptrs: lib.sr_ozaki_zgemm_td(0, 8, 8, k, ptrs, 8, ptrs, 8, None, 1, C, 8,
                                                                    s, w, nb, None)
    assert call(k=0) == -1  # SR_EINVAL: k >= 1
    assert call(s=0) == -1 and call(s=33) == -1
    assert call(nb=need - 1) == -3  # SR_ENOMEM
    assert call(C=None) == -1
    assert call() == 0


# ---------------------------------------------------------- sizes, checked in integers

@pytest.mark.parametrize("n", [2, 3, 17, 100, 130, 256])
def test_td_ragged_sizes_exact_rows(sr, n):
    """Gaps 0.05 from the complex128 Schur basis (zgees): converged to 1e-42 within 5
    passes; the exact residual and orthogonality defect (every row up to n = 130,
    16 sampled rows above) meet it, and T's upper triangle equals Q^H A Q's there."""
    from oracle import exact

    g = synth.schur_test_matrix(n, seed=300 + n, gap=0.05)
    a = g["A"]
    qh = synth.hp_schur_start(a)
    q, t, info = _refine(sr, a, qh, iters=6, tol=1e-42)
    assert info["status"] == "OK" and info["iters"] <= 5, info
    rows = np.arange(n) if n <= 130 else np.sort(np.random.default_rng(n).choice(n, 16, replace=False))
    ev = exact.residual_rows([a], q, rows)
    assert ev["stril"] <= 1e-42, ev
    assert ev["orth"] <= 1e-42, ev
    # T: the upper triangle of the same exact rows
    qr, qi, eq = exact.to_ints(q)
    ar, ai, ea = exact.to_ints([a])
    tr, ti, et = exact.to_ints(t)
    r = rows[: min(len(rows), 4)]
    vr = qr[:, r].T.dot(ar) + qi[:, r].T.dot(ai)
    vi = qr[:, r].T.dot(ai) - qi[:, r].T.dot(ar)
    mr = vr.dot(qr) - vi.dot(qi)
    mi = vr.dot(qi) + vi.dot(qr)
    s = ea + 2 * eq
    worst = 0.0
    for k, i in enumerate(r):
        for j in range(i, n):
            d = abs(Fraction(int(mr[k, j]), 1 << s) - Fraction(int(tr[i, j]), 1 << et)) + \
                abs(Fraction(int(mi[k, j]), 1 << s) - Fraction(int(ti[i, j]), 1 << et))
            worst = max(worst, float(d))
        assert not any(t[0][i, :i])  # T is upper triangular
    assert worst <= 1e-44 * ev["normA"], worst
