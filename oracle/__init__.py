"""CPU oracle for the Schur refinement: TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never calls it, and the two share no code.

This is a ctypes binding over liboracle.so (oracle.c, plain C in IEEE binary128).
It handles argument marshalling only: every step runs in the C code.

Matrices enter as complex128 numpy arrays (column-major), or as double-double
pairs (hi, lo). Binary128 results stay in `QMat` buffers and convert back to
double-double on request.

`oracle/exact.py` holds exact checks of multi-term results in Python integers
(residual and orthogonality rows past binary128's reach), pinned by its own tests.

Parity status: every entry point is pinned by the `-m "not gpu"` tests in
tests/test_oracle_*.py. Per-pass residual values have no published figures, so
they are pinned only through convergence laws, not value by value.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_LIB = None

LP = {"float": 0, "double": 1, "quad": 2}
STATUS = {0: "OK", 1: "NOT_CONVERGED", 3: "BREAKDOWN", 4: "DIVERGED"}
FULL_NS = 1
TRUNC = 2


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP, libquadmath)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _SO,
               os.path.join(_HERE, "oracle.c"), "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
    return _SO


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_double
        L.orc_from_dd.argtypes = [i64, vp, vp, vp]
        L.orc_to_dd.argtypes = [i64, vp, vp, vp]
        L.orc_gemm.argtypes = [i32, i32, i32, i32, vp, vp, vp]
        L.orc_trisolve.argtypes = [i32, i32, i32, vp, vp, vp, f64]
        L.orc_trisolve.restype = i32
        L.orc_ns.argtypes = [i32, vp, vp]
        L.orc_ns_merged.argtypes = [i32, i32, vp, vp, i32, vp]
        L.orc_refine.argtypes = [i32, i32, vp, vp, i32, f64, i32, vp, vp, vp, vp]
        L.orc_refine.restype = i32
        L.orc_eval.argtypes = [i32, vp, vp, vp, vp]
        L.orc_eval_rows.argtypes = [i32, vp, vp, i32, vp, vp]
        L.orc_schur_qr.argtypes = [i32, i32, vp, vp, vp]
        L.orc_schur_qr.restype = i32
        L.orc_reorder.argtypes = [i32, vp, vp, f64, vp, vp]
        L.orc_trisolve_real.argtypes = [i32, i32, vp, vp, vp, vp]
        L.orc_trisolve_real.restype = i32
        L.orc_refine_real.argtypes = [i32, i32, vp, vp, vp, i32, f64, vp, vp, vp, vp]
        L.orc_refine_real.restype = i32
        L.orc_eval_real.argtypes = [i32, vp, vp, vp, vp, vp]
        _LIB = L
    return _LIB


class QMat:
    """An m x n binary128 complex matrix (column-major), held as raw bytes."""

    def __init__(self, m: int, n: int):
        self.m, self.n = int(m), int(n)
        self.buf = np.zeros(self.m * self.n * 32, dtype=np.uint8)

    @property
    def ptr(self):
        return self.buf.ctypes.data

    @classmethod
    def from_dd(cls, hi, lo=None) -> "QMat":
        hi = np.asfortranarray(np.asarray(hi, dtype=np.complex128))
        if hi.ndim != 2:
            raise ValueError("expected a matrix")
        q = cls(*hi.shape)
        lo_p = None
        if lo is not None:
            lo = np.asfortranarray(np.asarray(lo, dtype=np.complex128))
            assert lo.shape == hi.shape
            lo_p = lo.ctypes.data
        lib().orc_from_dd(hi.size, hi.ctypes.data, lo_p, q.ptr)
        return q

    def to_dd(self):
        hi = np.zeros((self.m, self.n), dtype=np.complex128, order="F")
        lo = np.zeros((self.m, self.n), dtype=np.complex128, order="F")
        lib().orc_to_dd(self.m * self.n, self.ptr, hi.ctypes.data, lo.ctypes.data)
        return hi, lo

    def to_c128(self) -> np.ndarray:
        return self.to_dd()[0]


def _q(x) -> QMat:
    if isinstance(x, QMat):
        return x
    if isinstance(x, tuple):
        return QMat.from_dd(*x)
    return QMat.from_dd(x)


def gemm(a, b, opa: int = 0) -> QMat:
    """op(a) @ b in binary128 (opa = 1: conjugate transpose of a)."""
    a, b = _q(a), _q(b)
    m, k = (a.n, a.m) if opa else (a.m, a.n)
    assert b.m == k
    c = QMat(m, b.n)
    lib().orc_gemm(opa, m, b.n, k, a.ptr, b.ptr, c.ptr)
    return c


def trisolve(t, e, lp: str = "float", order: int = 0, trunc: float = 0.0):
    """L with stril(T L - L T) = -E, solved in lp; returns (L as QMat, status)."""
    t, e = _q(t), _q(e)
    n = t.n
    out = QMat(n, n)
    rc = lib().orc_trisolve(LP[lp], order, n, t.ptr, e.ptr, out.ptr, float(trunc))
    return out, STATUS.get(rc, rc)


def ns(qh) -> QMat:
    qh = _q(qh)
    out = QMat(qh.n, qh.n)
    lib().orc_ns(qh.n, qh.ptr, out.ptr)
    return out


def ns_merged(q, w, lp: str = "quad", full: bool = False) -> QMat:
    q, w = _q(q), _q(w)
    out = QMat(q.n, q.n)
    lib().orc_ns_merged(LP[lp], q.n, q.ptr, w.ptr, int(bool(full)), out.ptr)
    return out


def refine(a, qh, lp: str = "float", maxit: int = 6, tol: float = 1e-15,
           full_ns: bool = False, trunc: bool = False) -> dict:
    """Algorithm 4 from the start qh; returns Q, T (QMat), eps history, passes, status."""
    a, qh = _q(a), _q(qh)
    n = a.n
    qo, to = QMat(n, n), QMat(n, n)
    hist = np.zeros(maxit, dtype=np.float64)
    it = ctypes.c_int(0)
    flags = (FULL_NS if full_ns else 0) | (TRUNC if trunc else 0)
    rc = lib().orc_refine(LP[lp], n, a.ptr, qh.ptr, int(maxit), float(tol), flags,
                          qo.ptr, to.ptr, hist.ctypes.data, ctypes.byref(it))
    return {"Q": qo, "T": to, "hist": hist[: it.value].copy(), "iters": it.value,
            "status": STATUS.get(rc, rc)}


def reorder(a, qh, theta: float):
    """Reordered start (see oracle.h): returns (Q, perm) with Q a QMat."""
    a, qh = _q(a), _q(qh)
    n = a.n
    qo = QMat(n, n)
    perm = np.zeros(n, dtype=np.int32)
    lib().orc_reorder(n, a.ptr, qh.ptr, float(theta), qo.ptr, perm.ctypes.data)
    return qo, perm


def evaluate(a, q, t=None) -> dict:
    """Binary128 checks: relative stril residual, orthogonality, T consistency."""
    a, q = _q(a), _q(q)
    tq = _q(t) if t is not None else None
    out = np.zeros(4, dtype=np.float64)
    lib().orc_eval(a.n, a.ptr, q.ptr, tq.ptr if tq is not None else None, out.ctypes.data)
    return {"stril": out[0], "orth": out[1], "tdiff": out[2], "normA": out[3]}


def evaluate_rows(a, q, rows) -> dict:
    """Row-sampled binary128 checks (unbiased Frobenius estimates over `rows`)."""
    a, q = _q(a), _q(q)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32))
    out = np.zeros(4, dtype=np.float64)
    lib().orc_eval_rows(a.n, a.ptr, q.ptr, rows.size, rows.ctypes.data, out.ctypes.data)
    return {"stril": out[0], "stril_rowmax": out[1], "orth": out[2], "normA": out[3]}


def schur_qr(a, lp: str = "float"):
    """Complex Schur form of lp(A) by the shifted QR algorithm: (Z, S) as complex128."""
    a = _q(a)
    z, s = QMat(a.n, a.n), QMat(a.n, a.n)
    rc = lib().orc_schur_qr(LP[lp], a.n, a.ptr, z.ptr, s.ptr)
    if rc != 0:
        raise RuntimeError("QR algorithm did not converge")
    return z.to_c128(), s.to_c128()


# ------------------------------------------------------------ real Schur variant

def _blk(blk, n):
    b = np.zeros(n, dtype=np.int32) if blk is None else np.ascontiguousarray(np.asarray(blk, dtype=np.int32))
    assert b.size == n
    return b


def trisolve_real(t, e, blk, lp: str = "float"):
    """Block strictly lower L with block-stril(T L - L T) = -E (real Schur form with
    2 x 2 blocks marked by blk), solved in lp; returns (L as QMat, status)."""
    t, e = _q(t), _q(e)
    n = t.n
    b = _blk(blk, n)
    out = QMat(n, n)
    rc = lib().orc_trisolve_real(LP[lp], n, b.ctypes.data, t.ptr, e.ptr, out.ptr)
    return out, STATUS.get(rc, rc)


def refine_real(a, qh, blk, lp: str = "float", maxit: int = 6, tol: float = 1e-15) -> dict:
    """Algorithm 4 for the real Schur form (2 x 2 blocks marked by blk)."""
    a, qh = _q(a), _q(qh)
    n = a.n
    b = _blk(blk, n)
    qo, to = QMat(n, n), QMat(n, n)
    hist = np.zeros(maxit, dtype=np.float64)
    it = ctypes.c_int(0)
    rc = lib().orc_refine_real(LP[lp], n, a.ptr, qh.ptr, b.ctypes.data, int(maxit), float(tol), qo.ptr, to.ptr,
                               hist.ctypes.data, ctypes.byref(it))
    return {"Q": qo, "T": to, "hist": hist[: it.value].copy(), "iters": it.value, "status": STATUS.get(rc, rc)}


def evaluate_real(a, q, t, blk) -> dict:
    """Binary128 checks with the block strictly lower part of the real Schur form."""
    a, q = _q(a), _q(q)
    tq = _q(t) if t is not None else None
    b = _blk(blk, a.n)
    out = np.zeros(4, dtype=np.float64)
    lib().orc_eval_real(a.n, a.ptr, q.ptr, tq.ptr if tq is not None else None, b.ctypes.data, out.ctypes.data)
    return {"stril": out[0], "orth": out[1], "tdiff": out[2], "normA": out[3]}
