"""Pins of the CPU oracle against facts that do not come from the oracle itself:
exact arithmetic, closed forms, the defining equations written out as a linear
system, the identities the paper proves, and exactly known Schur forms.

Paper references: Section 2.1 eqs. (7)-(10), Algorithm 2, Theorem 1; Section 2.2
Lemma 2; Section 2.3 Theorem 2; Section 2.4 eq. (alg:eq:NSmerged), Algorithm 4.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _exact_cmat_product(a, b, conj_a=False):
    """Exact product of Gaussian-integer matrices with Python integers."""
    if conj_a:
        a = a.conj().T
    m, k = a.shape
    n = b.shape[1]
    out = np.zeros((m, n), dtype=np.complex128)
    for i in range(m):
        for j in range(n):
            sr = si = 0
            for p in range(k):
                ar, ai = int(a[i, p].real), int(a[i, p].imag)
                br, bi = int(b[p, j].real), int(b[p, j].imag)
                sr += ar * br - ai * bi
                si += ar * bi + ai * br
            out[i, j] = complex(sr, si)
    return out


# ---------------------------------------------------------------- products ----

@pytest.mark.parametrize("opa", [0, 1])
def test_gemm_exact_on_gaussian_integers(opa):
    rng = np.random.default_rng(11)
    m, k, n = 5, 7, 6
    ash = (k, m) if opa else (m, k)
    a = rng.integers(-256, 257, ash) + 1j * rng.integers(-256, 257, ash)
    b = rng.integers(-256, 257, (k, n)) + 1j * rng.integers(-256, 257, (k, n))
    c = oracle.gemm(a, b, opa=opa)
    hi, lo = c.to_dd()
    assert np.array_equal(hi, _exact_cmat_product(a, b, conj_a=bool(opa)))
    assert not lo.any()


def test_gemm_dd_inputs_carry_low_parts():
    # (1 + 2^-60) * (1 + 2^-60) = 1 + 2^-59 + 2^-120: visible only beyond double.
    hi = np.ones((1, 1), dtype=np.complex128)
    lo = np.full((1, 1), 2.0 ** -60, dtype=np.complex128)
    c = oracle.gemm((hi, lo), (hi, lo))
    chi, clo = c.to_dd()
    assert chi[0, 0] == 1.0 and clo[0, 0] == 2.0 ** -59


# ----------------------------------------------------------------- the solve ----

def _upper_distinct(rng, n, scale=1.0):
    t = np.triu(_rand_c(rng, (n, n))) * scale
    t[np.diag_indices(n)] = np.arange(1, n + 1) * (1.0 + 0.5j) + 0.1 * _rand_c(rng, n)
    return np.asfortranarray(t)


def _kronecker_solve(t, e):
    """Solve stril(T L - L T) = -E from its definition: one unknown per strictly
    lower entry, one equation per strictly lower entry, columns of the system
    matrix obtained by applying the operator to unit matrices."""
    n = t.shape[0]
    idx = [(i, j) for j in range(n) for i in range(j + 1, n)]
    m = np.zeros((len(idx), len(idx)), dtype=np.complex128)
    for c, (i, j) in enumerate(idx):
        unit = np.zeros((n, n), dtype=np.complex128)
        unit[i, j] = 1.0
        img = np.tril(t @ unit - unit @ t, -1)
        m[:, c] = [img[p, q] for (p, q) in idx]
    rhs = -np.array([e[p, q] for (p, q) in idx])
    sol = np.linalg.solve(m, rhs)
    out = np.zeros((n, n), dtype=np.complex128)
    for c, (i, j) in enumerate(idx):
        out[i, j] = sol[c]
    return out


@pytest.mark.parametrize("n", [2, 3, 4, 6, 9])
def test_trisolve_matches_kronecker_system(n):
    rng = np.random.default_rng(100 + n)
    t = _upper_distinct(rng, n)
    e = np.asfortranarray(np.tril(_rand_c(rng, (n, n)), -1))
    ref = _kronecker_solve(t, e)
    for order in (0, 1):
        l_q, st = oracle.trisolve(t, e, lp="quad", order=order)
        assert st == "OK"
        assert np.linalg.norm(l_q.to_c128() - ref) <= 1e-12 * np.linalg.norm(ref)
    l_d, _ = oracle.trisolve(t, e, lp="double")
    assert np.linalg.norm(l_d.to_c128() - ref) <= 1e-12 * np.linalg.norm(ref)
    l_f, _ = oracle.trisolve(t, e, lp="float")
    assert np.linalg.norm(l_f.to_c128() - ref) <= 1e-4 * np.linalg.norm(ref)
    assert np.linalg.norm(l_f.to_c128() - ref) > 0  # float arithmetic really used


def test_trisolve_diagonal_t_closed_form():
    # Diagonal T decouples the equation: l_ij = -e_ij / (t_ii - t_jj) (sign of eq. (7)).
    rng = np.random.default_rng(7)
    n = 8
    d = np.arange(1, n + 1) + 0.25j * np.arange(n)
    t = np.asfortranarray(np.diag(d))
    e = np.asfortranarray(np.tril(_rand_c(rng, (n, n)), -1))
    l, _ = oracle.trisolve(t, e, lp="quad")
    expect = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        for i in range(j + 1, n):
            expect[i, j] = -e[i, j] / (d[i] - d[j])
    assert np.allclose(l.to_c128(), expect, rtol=1e-15, atol=0)


def test_trisolve_n2_closed_form():
    t = np.array([[1.0 + 1j, 5.0 - 2j], [0, -2.0 + 0.5j]], order="F")
    e = np.array([[0, 0], [0.3 - 0.7j, 0]], order="F")
    l, _ = oracle.trisolve(t, e, lp="quad")
    assert abs(l.to_c128()[1, 0] - (-(0.3 - 0.7j) / ((-2.0 + 0.5j) - (1.0 + 1j)))) < 1e-15


def test_trisolve_residual_float_n48():
    rng = np.random.default_rng(3)
    n = 48
    g = synth.schur_test_matrix(n, 5)
    t = g["T0"]
    e = np.asfortranarray(1e-6 * np.tril(_rand_c(rng, (n, n)), -1))
    l, st = oracle.trisolve(t, e, lp="float")
    assert st == "OK"
    lv = l.to_c128()
    t32 = np.triu(t).astype(np.complex64).astype(np.complex128)
    e32 = e.astype(np.complex64).astype(np.complex128)
    res = np.linalg.norm(np.tril(t32 @ lv - lv @ t32, -1) + e32)
    bound = 8 * n * U32 * (np.linalg.norm(t32) * np.linalg.norm(lv) + np.linalg.norm(e32))
    assert res <= bound
    assert np.abs(np.triu(lv)).max() == 0.0


def test_trisolve_orders_agree_theorem1():
    # Theorem 1: the solution is unique, so every admissible order gives it.
    rng = np.random.default_rng(21)
    n = 20
    t = _upper_distinct(rng, n)
    e = np.asfortranarray(np.tril(_rand_c(rng, (n, n)), -1))
    a, _ = oracle.trisolve(t, e, lp="quad", order=0)
    b, _ = oracle.trisolve(t, e, lp="quad", order=1)
    ah, al = a.to_dd()
    bh, bl = b.to_dd()
    diff = np.abs((ah - bh) + (al - bl)).max()
    assert diff <= 1e-28 * np.abs(ah).max()


def test_trisolve_equal_diagonal_breaks_down():
    t = np.asfortranarray(np.triu(np.ones((4, 4), dtype=np.complex128)))
    t[np.diag_indices(4)] = [1.0, 2.0, 1.0, 3.0]
    e = np.asfortranarray(np.tril(np.ones((4, 4), dtype=np.complex128), -1))
    _, st = oracle.trisolve(t, e, lp="quad")
    assert st == "BREAKDOWN"


def test_trisolve_truncation_device():
    rng = np.random.default_rng(4)
    n = 6
    t = _upper_distinct(rng, n)
    e = np.asfortranarray(np.tril(_rand_c(rng, (n, n)), -1))
    l, _ = oracle.trisolve(t, e, lp="quad", trunc=1e-5)
    # every entry of this L would be O(1); the device zeroes each as computed
    assert not l.to_c128().any()


def _fraction_trisolve(t, e, trunc):
    """Algorithm 2 in exact rational arithmetic, written out from eq. (9) (column
    index of L read as j), with the large-entry device of Example 4: an entry whose
    modulus exceeds trunc is set to zero as soon as it is computed, before any later
    entry uses it."""
    n = t.shape[0]
    fr = lambda z: (Fraction(z.real), Fraction(z.imag))
    T = [[fr(t[i, j]) for j in range(n)] for i in range(n)]
    E = [[fr(e[i, j]) for j in range(n)] for i in range(n)]
    zero = (Fraction(0), Fraction(0))
    L = [[zero] * n for _ in range(n)]
    mul = lambda a, b: (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])
    for j in range(n - 1):
        for i in range(n - 1, j, -1):
            s = E[i][j]
            for k in range(i + 1, n):
                p = mul(T[i][k], L[k][j])
                s = (s[0] + p[0], s[1] + p[1])
            for k in range(j):
                p = mul(L[i][k], T[k][j])
                s = (s[0] - p[0], s[1] - p[1])
            d = (T[i][i][0] - T[j][j][0], T[i][i][1] - T[j][j][1])
            den = d[0] * d[0] + d[1] * d[1]
            l = (-(s[0] * d[0] + s[1] * d[1]) / den, -(s[1] * d[0] - s[0] * d[1]) / den)
            if l[0] * l[0] + l[1] * l[1] > Fraction(trunc) ** 2:
                l = zero
            L[i][j] = l
    # double-double rounding of the exact result: (hi, lo) with hi + lo = L to ~2^-106
    def dd(x):
        h = float(x)
        return h, float(x - Fraction(h))
    hi = np.zeros((n, n), dtype=np.complex128)
    lo = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for j in range(n):
            (rh, rl), (ih, il) = dd(L[i][j][0]), dd(L[i][j][1])
            hi[i, j], lo[i, j] = complex(rh, ih), complex(rl, il)
    return hi, lo


def truncation_case(n, seed):
    """T with O(1) off-diagonal entries and separated diagonal; E of size 1e-8 except
    for entries early in every admissible order (bottom-left corner and one inside)
    whose L entries are far above 1e-5. Every other entry of L then depends on
    whether those are zeroed as computed or only afterwards."""
    rng = np.random.default_rng(seed)
    t = np.triu(_rand_c(rng, (n, n))) / np.sqrt(2)
    t[np.diag_indices(n)] = np.arange(1, n + 1) * (1.0 + 0.5j)
    e = np.tril(1e-8 * _rand_c(rng, (n, n)), -1)
    e[n - 1, 0] = 0.5
    e[n - 2, 1] = 0.3 - 0.2j
    e[(2 * n) // 3, n // 3] = 0.2j
    return np.asfortranarray(t), np.asfortranarray(e)


def test_trisolve_truncation_as_computed():
    """Example 4's device zeroes an entry of L while L is being computed, so entries
    computed later see the zero. Pinned against exact rational substitution that
    zeroes immediately; zeroing the large entries after the solve gives a different
    L (here the large entries drag every entry that depends on them above 1e-5)."""
    n, trunc = 10, 1e-5
    t, e = truncation_case(n, 2)
    ref, ref_lo = _fraction_trisolve(t, e, trunc)
    assert np.count_nonzero(np.tril(ref, -1)) >= n * (n - 1) // 2 - 4  # small entries survive
    lo = np.abs(ref[np.tril_indices(n, -1)])
    assert np.all((lo == 0) | (lo < 0.1 * trunc))  # no entry near the threshold
    l, st = oracle.trisolve(t, e, lp="quad", trunc=trunc)
    assert st == "OK"
    hi_, lo_ = l.to_dd()
    assert np.abs((hi_ - ref) + (lo_ - ref_lo)).max() <= 1e-30 * np.abs(ref).max()
    # the float solve takes the same zeroing decisions
    lf, _ = oracle.trisolve(t, e, lp="float", trunc=trunc)
    lf = lf.to_c128()
    assert np.array_equal(lf == 0, ref == 0)
    assert np.abs(lf - ref).max() <= 1e-5 * np.abs(ref).max()
    # zeroing after the fact is a different device
    full, _ = oracle.trisolve(t, e, lp="quad")
    full = full.to_c128()
    after = np.where(np.abs(full) > trunc, 0, full)
    assert np.abs(after - ref).max() >= 0.1 * np.abs(ref).max()


# ----------------------------------------------------------- orthogonalising ----

def _near_unitary(rng, n, size):
    q, _ = np.linalg.qr(_rand_c(rng, (n, n)))
    return np.asfortranarray(q + size * _rand_c(rng, (n, n)) / np.sqrt(n))


def test_newton_schulz_lemma2_identity():
    # Qn^H Qn - I = -3/4 Y^2 + 1/4 Y^3 with Y = Qh^H Qh - I (Lemma 2).
    rng = np.random.default_rng(5)
    n = 12
    qh = _near_unitary(rng, n, 1e-2)
    y = qh.conj().T @ qh - np.eye(n)
    qn = oracle.ns(qh).to_c128()
    lhs = qn.conj().T @ qn - np.eye(n)
    rhs = -0.75 * y @ y + 0.25 * y @ y @ y
    assert np.linalg.norm(lhs - rhs) <= 1e-10 * np.linalg.norm(rhs)
    assert np.linalg.norm(rhs) > 1e-6


def _skew(rng, n, size):
    lo = np.tril(_rand_c(rng, (n, n)), -1) * size
    return np.asfortranarray(lo - lo.conj().T)


def test_merged_update_equals_direct_newton_schulz():
    # eq. (alg:eq:NSmerged): 1/2 Q(I+W)(3I - (I+W)^H Q^H Q (I+W)) expands, with
    # W^H = -W, to 1/2 Q (2I + 2W - Y - YW + W^2 + W^3 + W^2 Y + W^2 Y W).
    rng = np.random.default_rng(6)
    n = 10
    q = _near_unitary(rng, n, 1e-3)
    w = _skew(rng, n, 1e-2)
    merged = oracle.ns_merged(q, w, lp="quad", full=True).to_c128()
    qh = q @ (np.eye(n) + w)
    direct = 0.5 * qh @ (3 * np.eye(n) - qh.conj().T @ qh)
    assert np.linalg.norm(merged - direct) <= 1e-14 * np.linalg.norm(direct)


def test_merged_update_truncation_error():
    # Dropping W^2 Y and W^2 Y W changes the result by exactly -1/2 Q (W^2 Y + W^2 Y W).
    rng = np.random.default_rng(8)
    n = 10
    q = _near_unitary(rng, n, 3e-2)
    w = _skew(rng, n, 3e-2)
    full = oracle.ns_merged(q, w, lp="quad", full=True)
    trunc = oracle.ns_merged(q, w, lp="quad", full=False)
    fh, fl = full.to_dd()
    th, tl = trunc.to_dd()
    diff = (th - fh) + (tl - fl)
    y = q.conj().T @ q - np.eye(n)
    expect = -0.5 * q @ (w @ w @ y + w @ w @ y @ w)
    assert np.linalg.norm(diff - expect) <= 1e-9 * np.linalg.norm(expect)
    assert np.linalg.norm(expect) > 1e-9


@pytest.mark.parametrize("lp,u", [("float", 2.0 ** -24), ("double", 2.0 ** -53)])
def test_merged_update_products_in_lp(lp, u):
    """Algorithm 4 forms YW, W^2 and W^3 in lp (and sums in hp): the result differs
    from the all-hp update by the lp rounding of those products, no less (a product
    formed in hp would give no difference) and no more (first-order bound of an lp
    product: operands rounded once, dot products of length n)."""
    rng = np.random.default_rng(9)
    n = 24
    q, _ = np.linalg.qr(_rand_c(rng, (n, n)))
    q = np.asfortranarray(q + 1e-3 * _rand_c(rng, (n, n)) / np.sqrt(n))
    w = _skew(rng, n, 3e-2)
    rh, rl = oracle.ns_merged(q, w, lp="quad").to_dd()
    h, l = oracle.ns_merged(q, w, lp=lp).to_dd()
    d = np.linalg.norm((h - rh) + (l - rl))
    y = q.conj().T @ q - np.eye(n)
    w2 = w @ w
    size = np.linalg.norm(y @ w) + np.linalg.norm(w2) + np.linalg.norm(w2 @ w)
    absb = (np.linalg.norm(np.abs(y) @ np.abs(w)) + np.linalg.norm(np.abs(w) @ np.abs(w))
            + np.linalg.norm(np.abs(w2) @ np.abs(w)))
    upper = 0.5 * np.linalg.norm(q, 2) * np.sqrt(2) * (n + 4) * u * absb
    assert 0.05 * u * size <= d <= upper, (d / (u * size), d / upper)


def test_merged_update_lp_precision_scales_with_u():
    rng = np.random.default_rng(10)
    n = 16
    q, _ = np.linalg.qr(_rand_c(rng, (n, n)))
    q = np.asfortranarray(q + 1e-3 * _rand_c(rng, (n, n)) / np.sqrt(n))
    w = _skew(rng, n, 3e-2)
    rh, rl = oracle.ns_merged(q, w, lp="quad").to_dd()
    d = {}
    for lp in ("float", "double"):
        h, l = oracle.ns_merged(q, w, lp=lp).to_dd()
        d[lp] = np.linalg.norm((h - rh) + (l - rl))
    ratio = d["float"] / d["double"] / 2.0 ** 29  # u32 / u64
    assert 0.1 <= ratio <= 10, ratio


# -------------------------------------------------------------- Algorithm 4 ----

def _fraction_matrix(hi, lo):
    n, m = hi.shape
    return [[(Fraction(hi[i, j].real) + Fraction(lo[i, j].real),
              Fraction(hi[i, j].imag) + Fraction(lo[i, j].imag)) for j in range(m)]
            for i in range(n)]


@pytest.mark.parametrize("n,lp,maxit", [(16, "quad", 6), (16, "float", 10), (64, "double", 8)])
def test_refine_recovers_exact_schur_form(n, lp, maxit):
    """Walsh-Hadamard test matrices have an exactly known Schur form (Q0, T0):
    the refined Q must equal Q0 D (D diagonal unitary) to binary128 accuracy."""
    h = synth.hadamard_exact(n, seed=n)
    q0, lam = h["Q0"].real, h["lam"]
    qh = synth.perturbed_start(h["Q0"], seed=1, delta=1e-6)
    r = oracle.refine(h["A"], qh, lp=lp, maxit=maxit, tol=1e-30)
    assert r["status"] == "OK", r
    qhi, qlo = r["Q"].to_dd()
    thi, tlo = r["T"].to_dd()
    # diag(T) equals diag(T0) (binary numbers) in the start's order
    dd = np.abs((np.diag(thi) - lam) + np.diag(tlo))
    assert dd.max() <= 1e-28
    # Q0^T Q is diagonal with unimodular entries, checked in exact rationals
    qf = _fraction_matrix(qhi, qlo)
    k = int(round(np.log2(n) / 2))
    s = Fraction(1, 2 ** k)
    worst_off, worst_mod = 0.0, 0.0
    cols = range(n) if n <= 16 else range(0, n, 7)
    for j in cols:
        for i in range(n):
            re = sum((s if q0[p, i] > 0 else -s) * qf[p][j][0] for p in range(n))
            im = sum((s if q0[p, i] > 0 else -s) * qf[p][j][1] for p in range(n))
            if i == j:
                worst_mod = max(worst_mod, abs(float(re * re + im * im - 1)))
            else:
                worst_off = max(worst_off, float(abs(re) + abs(im)))
    assert worst_off <= 1e-28 and worst_mod <= 1e-28


def test_refine_quadratic_convergence_theorem2():
    g = synth.schur_test_matrix(32, seed=9)
    qh = synth.lp_schur_start(g["A"])
    r = oracle.refine(g["A"], qh, lp="quad", maxit=8, tol=1e-31)
    h = r["hist"]
    assert r["status"] == "OK"
    assert h[0] < 1e-5
    for a, b in zip(h[:-1], h[1:]):
        assert b <= 1e3 * a * a or b <= 1e-31
    ev = oracle.evaluate(g["A"], r["Q"], r["T"])
    assert ev["orth"] <= 1e-31 and ev["stril"] <= 1e-31 and ev["tdiff"] == 0.0


def test_refine_float_lp_contracts_linearly_then_converges():
    # With the solve in float, each pass after the first gains at least five
    # decades until the high-precision floor (u_lp * conditioning per pass).
    g = synth.schur_test_matrix(64, seed=0)
    qh = synth.lp_schur_start(g["A"])
    r = oracle.refine(g["A"], qh, lp="float", maxit=8, tol=1e-30)
    h = r["hist"]
    assert r["status"] == "OK" and r["iters"] <= 6
    for a, b in zip(h[:-1], h[1:]):
        assert b <= 1e-5 * a
    assert np.argmax(h <= 1e-15) + 1 <= 3  # FP64 target reached by pass 3


@pytest.mark.parametrize("n", [2, 3, 4])
def test_refine_matches_eigenvector_schur_bruteforce(n):
    """Schur vectors from eigenvectors: Gram-Schmidt of the eigenvectors taken in
    the order of the start's diagonal gives the unique Schur basis (up to phases)."""
    rng = np.random.default_rng(40 + n)
    a = np.asfortranarray(_rand_c(rng, (n, n)))
    w, v = np.linalg.eig(a)
    qh = synth.lp_schur_start(a)
    r = oracle.refine(a, qh, lp="float", maxit=8, tol=1e-30)
    assert r["status"] == "OK"
    q = r["Q"].to_c128()
    t = r["T"].to_c128()
    order = [int(np.argmin(np.abs(w - t[i, i]))) for i in range(n)]
    assert sorted(order) == list(range(n))
    basis = np.zeros((n, n), dtype=np.complex128)
    for c, idx in enumerate(order):
        x = v[:, idx].copy()
        for p in range(c):
            x -= basis[:, p] * (basis[:, p].conj() @ x)
        basis[:, c] = x / np.linalg.norm(x)
    ph = np.array([basis[:, c].conj() @ q[:, c] for c in range(n)])
    ph /= np.abs(ph)
    assert np.linalg.norm(q - basis * ph[None, :]) <= 1e-12
    assert np.allclose(np.diag(t), w[order], rtol=0, atol=1e-13)


def test_refine_iteration_cap_and_counts():
    g = synth.schur_test_matrix(16, seed=2)
    qh = synth.lp_schur_start(g["A"])
    r = oracle.refine(g["A"], qh, lp="float", maxit=1, tol=1e-30)
    assert r["status"] == "NOT_CONVERGED" and r["iters"] == 1


def _rotated_start(q0, seed, delta):
    """q0 exp(H) with H skew-Hermitian of size delta: a unitary start rotated away
    from the Schur basis."""
    rng = np.random.default_rng(seed)
    n = q0.shape[0]
    x = delta * _rand_c(rng, (n, n))
    h = (x - x.conj().T) / 2
    w, v = np.linalg.eigh(1j * h)
    return np.asfortranarray(q0 @ (v @ np.diag(np.exp(-1j * w)) @ v.conj().T))


def test_refine_diverged_rule():
    """Reading of the stopping rule: DIVERGED when the residual rose on two
    consecutive passes. A start rotated far (0.15) from the Schur basis makes the
    residual wander: single rises followed by a fall do not stop the iteration, the
    first pair of consecutive rises does."""
    g = synth.schur_test_matrix(8, seed=5)
    qh = _rotated_start(g["Q0"], 5, 0.15)
    r = oracle.refine(g["A"], qh, lp="float", maxit=14, tol=1e-30)
    h = r["hist"]
    assert r["status"] == "DIVERGED"
    triples = [p for p in range(2, len(h)) if h[p] > h[p - 1] > h[p - 2]]
    assert triples == [len(h) - 1] and r["iters"] == len(h)
    isolated = [p for p in range(1, len(h) - 2) if h[p] > h[p - 1] and h[p + 1] < h[p]]
    assert isolated, h  # a single rise that did not stop it
    assert r["iters"] < 14


def test_refine_nan_input_breaks_down():
    g = synth.schur_test_matrix(8, seed=2)
    a = g["A"].copy()
    a[3, 2] = np.nan
    r = oracle.refine(a, synth.lp_schur_start(g["A"]), lp="float", maxit=4, tol=1e-30)
    assert r["status"] == "BREAKDOWN"


# ---------------------------------------------------------------- evaluation ----

def test_eval_exact_on_hadamard_and_agrees_with_numpy():
    h = synth.hadamard_exact(16, seed=3)
    ev = oracle.evaluate(h["A"], h["Q0"], h["T0"])
    assert ev["stril"] == 0.0 and ev["orth"] == 0.0 and ev["tdiff"] == 0.0
    rng = np.random.default_rng(1)
    q = h["Q0"] + 1e-3 * _rand_c(rng, (16, 16))
    t = np.triu(q.conj().T @ h["A"] @ q) + 1e-3
    ev = oracle.evaluate(h["A"], q, t)
    th = q.conj().T @ h["A"] @ q
    assert np.isclose(ev["stril"], np.linalg.norm(np.tril(th, -1)) / np.linalg.norm(h["A"]), rtol=1e-12)
    assert np.isclose(ev["orth"], np.linalg.norm(q.conj().T @ q - np.eye(16)), rtol=1e-10)
    assert np.isclose(ev["tdiff"], np.linalg.norm(t - np.triu(th)), rtol=1e-10)


def test_eval_rows_is_the_row_restricted_sum():
    rng = np.random.default_rng(2)
    n = 24
    a = np.asfortranarray(_rand_c(rng, (n, n)))
    q = np.asfortranarray(np.linalg.qr(_rand_c(rng, (n, n)))[0] + 1e-4 * _rand_c(rng, (n, n)))
    full = oracle.evaluate(a, q)
    allrows = oracle.evaluate_rows(a, q, np.arange(n))
    assert np.isclose(full["stril"], allrows["stril"], rtol=1e-14)
    assert np.isclose(full["orth"], allrows["orth"], rtol=1e-12)
    rows = np.array([3, 10, 17, 23])
    sub = oracle.evaluate_rows(a, q, rows)
    th = q.conj().T @ a @ q
    s = sum(np.linalg.norm(th[i, :i]) ** 2 for i in rows)
    assert np.isclose(sub["stril"], np.sqrt(n / rows.size * s) / np.linalg.norm(a), rtol=1e-12)


# ------------------------------------------------------------- lp Schur start ----

@pytest.mark.parametrize("lp,tol", [("float", 2e-5), ("double", 1e-13)])
def test_schur_qr_residual_and_spectrum(lp, tol):
    h = synth.hadamard_exact(16, seed=5)
    z, s = oracle.schur_qr(h["A"], lp=lp)
    a = h["A"]
    assert np.linalg.norm(z @ s @ z.conj().T - a) <= tol * np.linalg.norm(a)
    assert np.linalg.norm(z.conj().T @ z - np.eye(16)) <= tol
    assert not np.tril(s, -1).any()
    lam = h["lam"]
    d = np.diag(s)
    for x in lam:
        assert np.min(np.abs(d - x)) <= 50 * tol
