"""MI355X (gfx950) refinement of Schur decompositions: Python binding.

A thin ctypes layer over libschurrefine.so (C interface in include/schur_refine.h).
It marshals arguments only: every step of the refinement runs in the library's
HIP kernels. PyTorch supplies device memory and the current stream.

Matrices are torch tensors on the GPU in column-major storage: shape (m, n) with
strides (1, m), the layout of `colmajor(x)` below (the transpose view of a
row-major tensor). complex128 unless a function says complex64.

Importing the package does not load the library; the first call does, and raises
if libschurrefine.so has not been built (`python -m paper_2203_10879_amd.build`).
There is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libschurrefine.so")
_LIB = None

STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "STAGNATED", 3: "BREAKDOWN", 4: "DIVERGED",
          -1: "EINVAL", -2: "EHIP", -3: "ENOMEM", -4: "ENOSYS"}
GEMM_MODES = {"fp64": 0, "ozaki_i8": 1, "ozaki_bf16": 2, "ozaki_i8_all": 3, "ozaki_crt": 4}


class SrOpts(ctypes.Structure):
    _fields_ = [("gemm", ctypes.c_int), ("slices", ctypes.c_int), ("update_slices", ctypes.c_int),
                ("compensated", ctypes.c_int), ("gate_lp_terms", ctypes.c_int),
                ("trunc", ctypes.c_int), ("timing", ctypes.c_int), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("stream", ctypes.c_void_p),
                ("strict_stop", ctypes.c_int), ("solver", ctypes.c_int), ("rec_leaf", ctypes.c_int),
                ("skip_orth", ctypes.c_int), ("lp_digits", ctypes.c_int)]


class SrInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("updates", ctypes.c_int),
                ("hp_gemms", ctypes.c_int), ("lp_products", ctypes.c_int),
                ("resid", ctypes.c_double), ("orth", ctypes.c_double),
                ("resid_hist", ctypes.c_double * 16), ("norm_w_hist", ctypes.c_double * 16),
                ("ms_total", ctypes.c_float), ("ms_hp_gemm", ctypes.c_float),
                ("hp_gemm_launches", ctypes.c_int), ("ms_solve", ctypes.c_float),
                ("update_slices_hist", ctypes.c_int * 16), ("hp_gemm_herm_launches", ctypes.c_int),
                ("ms_hp_gemm_herm", ctypes.c_float), ("ms_oz_full", ctypes.c_float),
                ("oz_full_launches", ctypes.c_int), ("oz_full_pairs", ctypes.c_int)]

    def as_dict(self) -> dict:
        k = min(self.iters, 16)
        u = min(self.updates, 16)
        return {"status": STATUS.get(self.status, self.status), "iters": self.iters,
                "updates": self.updates, "hp_gemms": self.hp_gemms,
                "lp_products": self.lp_products, "resid": self.resid, "orth": self.orth,
                "resid_hist": list(self.resid_hist[:k]), "norm_w_hist": list(self.norm_w_hist[:u]),
                "ms_total": self.ms_total, "ms_hp_gemm": self.ms_hp_gemm,
                "hp_gemm_launches": self.hp_gemm_launches, "ms_solve": self.ms_solve,
                "update_slices_hist": list(self.update_slices_hist[:min(u + 1, 16)]),
                "hp_gemm_herm_launches": self.hp_gemm_herm_launches,
                "ms_hp_gemm_herm": self.ms_hp_gemm_herm, "ms_oz_full": self.ms_oz_full,
                "oz_full_launches": self.oz_full_launches, "oz_full_pairs": self.oz_full_pairs}


# name -> (restype, argtypes); mirrors include/schur_refine.h
_vp, _i, _d, _f, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_float, ctypes.c_size_t
_SIGS = {
    "sr_default_opts": (None, [ctypes.POINTER(SrOpts)]),
    "sr_workspace_bytes": (_sz, [_i, ctypes.POINTER(SrOpts)]),
    "schur_refine": (_i, [_vp, _vp, _vp, _i, _i, _d, ctypes.POINTER(SrOpts), ctypes.POINTER(SrInfo)]),
    "schur_refine_batched": (_i, [_i, _vp, _vp, _vp, _vp, _i, _d, ctypes.POINTER(SrOpts),
                                  ctypes.POINTER(SrInfo)]),
    "schur_refine_dd": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _d, ctypes.POINTER(SrOpts),
                             ctypes.POINTER(SrInfo)]),
    "sr_status_string": (ctypes.c_char_p, [_i]),
    "sr_zgemm": (_i, [_i, _i, _i, _i, _vp, _i, _vp, _i, _vp, _i, _vp, _i, _i, _vp]),
    "sr_cgemm": (_i, [_i, _i, _i, _vp, _i, _vp, _i, _vp, _i, _vp]),
    "sr_residual": (_i, [_vp, _vp, _i, _vp, _vp, _vp, ctypes.POINTER(_d), _i, _vp, _vp]),
    "sr_trisolve": (_i, [_vp, _vp, _vp, _i, _f, _vp, _vp]),
    "sr_trisolve64": (_i, [_vp, _vp, _vp, _i, _vp, _vp]),
    "sr_trisolve_static": (_i, [_vp, _vp, _vp, _i, _f, _vp, _vp]),
    "sr_reorder_ws_bytes": (_sz, [_i]),
    "sr_reorder_start": (_i, [_vp, _vp, _i, ctypes.c_double, _vp, _vp, _sz, _vp]),
    "sr_update": (_i, [_vp, _vp, _vp, _i, _i, _i, ctypes.POINTER(_d), _vp, _vp]),
    "sr_ns_init": (_i, [_vp, _vp, _i, _i, _vp, _vp]),
    "sr_ozaki_ws_bytes": (_sz, [_i, _i, _i, _i, _i]),
    "sr_ozaki_zgemm": (_i, [_i, _i, _i, _i, _vp, _i, _vp, _i, _vp, _i, _vp, _i, _i, _i, _i, _vp, _sz, _vp]),
    "sr_ozaki_zgemm_dd": (_i, [_i, _i, _i, _i, _vp, _vp, _i, _vp, _vp, _i, _vp, _vp, _i, _vp, _vp, _i,
                               _i, _i, _i, _vp, _sz, _vp]),
    "sr_workspace_bytes_dd": (_sz, [_i, ctypes.POINTER(SrOpts)]),
    "schur_refine_real": (_i, [_vp, _vp, _vp, _vp, _i, _i, _d, ctypes.POINTER(SrOpts), ctypes.POINTER(SrInfo)]),
    "sr_workspace_bytes_real": (_sz, [_i, ctypes.POINTER(SrOpts)]),
    "sr_dgemm": (_i, [_i, _i, _i, _i, _vp, _i, _vp, _i, _vp, _i, _vp, _i, _i, _vp]),
    "sr_trisolve_real_ws_bytes": (_sz, [_i]),
    "sr_trisolve_real": (_i, [_vp, _vp, _vp, _vp, _i, _vp, _sz, _vp]),
    "schur_refine_td": (_i, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                             ctypes.POINTER(ctypes.c_void_p), _i, _i, _d, ctypes.POINTER(SrOpts),
                             ctypes.POINTER(SrInfo)]),
    "sr_workspace_bytes_td": (_sz, [_i, ctypes.POINTER(SrOpts)]),
    "sr_ozaki_cgemm": (_i, [_i, _i, _i, _vp, _i, _vp, _i, _vp, _i, _i, _i, _vp, _sz, _vp]),
    "sr_ozaki_zgemm_td": (_i, [_i, _i, _i, _i, ctypes.POINTER(ctypes.c_void_p), _i,
                               ctypes.POINTER(ctypes.c_void_p), _i, ctypes.POINTER(ctypes.c_void_p), _i,
                               ctypes.POINTER(ctypes.c_void_p), _i, _i, _vp, _sz, _vp]),
    "sr_batched_tile_grid": (_i, [_i]),
    "sr_tuning_save": (_i, [ctypes.c_char_p]),
    "sr_tuning_load": (_i, [ctypes.c_char_p]),
    "sr_tuning_reset": (None, []),
    "sr_tuning_runs": (_i, []),
    "sr_trisolve_rec_ws_bytes": (_sz, [_i, _i]),
    "sr_trisolve_rec": (_i, [_vp, _vp, _vp, _i, _i, ctypes.c_float, _vp, _sz, _vp]),
    "sr_crt_moduli": (_i, [_i, _i]),
    "sr_crt_ws_bytes": (_sz, [_i, _i, _i, _i]),
    "sr_crt_zgemm": (_i, [_i, _i, _i, _i, _vp, _i, _vp, _i, _vp, _i, _vp, _i, _i, _vp, _sz, _vp]),
    "sr_workspace_bytes_batched": (_sz, [_i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(SrOpts)]),
    "sr_batched_tile_edge": (_i, [_i]),
    "sr_batched_graph_builds": (_i, []),
    "sr_diag_mfma": (_i, [_i, _vp, _vp, _vp]),
}
EXPORTS = tuple(_SIGS)


def lib():
    """Load libschurrefine.so (raises if it is missing)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is not built; run `python -m paper_2203_10879_amd.build`")
        L = ctypes.CDLL(SO_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


# ------------------------------------------------------------------ helpers

def colmajor(x, device="cuda"):
    """A (m, n) torch tensor on `device` holding x in column-major storage."""
    import torch

    if isinstance(x, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(x).T))
    else:
        t = x.detach().T.contiguous()
    return t.to(device).T


def colmajor_empty(m, n, dtype=None, device="cuda"):
    import torch

    dtype = dtype or torch.complex128
    return torch.zeros((n, m), dtype=dtype, device=device).T


def to_numpy(t) -> np.ndarray:
    """Host copy (column-major numpy array) of a column-major tensor."""
    return np.asfortranarray(t.T.contiguous().cpu().numpy().T)


def _mat(t, dtype_name: str, rows: int | None = None, cols: int | None = None):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA/HIP torch tensor")
    want = {"c128": torch.complex128, "c64": torch.complex64, "f64": torch.float64, "f32": torch.float32}[dtype_name]
    if t.dtype != want:
        raise TypeError(f"expected {want}, got {t.dtype}")
    if t.dim() != 2 or (t.shape[0] > 1 and t.stride(0) != 1) or (t.shape[1] > 1 and t.stride(1) < t.shape[0]):
        raise ValueError("expected a column-major matrix (strides (1, ld))")
    if rows is not None and t.shape[0] != rows:
        raise ValueError("row count mismatch")
    if cols is not None and t.shape[1] != cols:
        raise ValueError("column count mismatch")
    return ctypes.c_void_p(t.data_ptr())


def _ld(t) -> int:
    """Leading dimension of a column-major tensor (strides of size-1 dimensions are
    arbitrary in torch)."""
    if t is None:
        return 0
    return int(t.stride(1)) if t.shape[1] > 1 else max(1, int(t.shape[0]))


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


SOLVERS = {"wavefront": 0, "recursive": 1}


def make_opts(gemm="fp64", slices=0, update_slices=0, compensated=True, gate=True, trunc=False,
              timing=False, workspace=None, stream=None, strict_stop=False, solver="wavefront",
              rec_leaf=0, skip_orth=False, lp_digits=0) -> SrOpts:
    o = SrOpts()
    lib().sr_default_opts(ctypes.byref(o))
    o.gemm = GEMM_MODES[gemm] if isinstance(gemm, str) else int(gemm)
    o.slices = int(slices)
    o.update_slices = int(update_slices)
    o.compensated = int(bool(compensated))
    o.gate_lp_terms = int(bool(gate))
    o.trunc = int(bool(trunc))
    o.timing = int(bool(timing))
    o.strict_stop = int(bool(strict_stop))
    o.solver = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    o.rec_leaf = int(rec_leaf)
    o.skip_orth = int(bool(skip_orth))
    o.lp_digits = int(lp_digits)
    if workspace is not None:
        o.workspace = ctypes.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.stream = _stream(stream)
    return o


def workspace(n: int, device="cuda", **kw):
    """A device workspace tensor large enough for size n under the options `kw`
    (as for make_opts)."""
    import torch

    o = make_opts(**kw) if kw else None
    nbytes = lib().sr_workspace_bytes(int(n), ctypes.byref(o) if o is not None else None)
    return torch.empty(max(1, nbytes), dtype=torch.uint8, device=device)


def sr_workspace_bytes(n: int) -> int:
    return int(lib().sr_workspace_bytes(int(n), None))


def sr_status_string(code: int) -> str:
    return lib().sr_status_string(int(code)).decode()


# ------------------------------------------------------------ entry points

def schur_refine(A, Q, T, iters: int = 6, tol: float = 1e-15, **kw) -> dict:
    """Refine (Q, T) for A in place; returns the info record as a dict."""
    n = A.shape[0]
    a = _mat(A, "c128", n, n)
    q = _mat(Q, "c128", n, n)
    t = _mat(T, "c128", n, n)
    o = make_opts(**kw)
    info = SrInfo()
    rc = lib().schur_refine(a, q, t, n, int(iters), float(tol), ctypes.byref(o), ctypes.byref(info))
    d = info.as_dict()
    d["rc"] = rc
    return d


def workspace_batched(sizes, device="cuda", **kw):
    """A device workspace tensor for schur_refine_batched over matrices of `sizes`."""
    import torch

    b = len(sizes)
    ns = (ctypes.c_int * max(1, b))(*[int(x) for x in sizes])
    o = make_opts(**kw)
    nbytes = int(lib().sr_workspace_bytes_batched(b, ns, ctypes.byref(o)))
    return torch.empty(max(1, nbytes), dtype=torch.uint8, device=device)


def schur_refine_batched(As, Qs, Ts, iters: int = 6, tol: float = 1e-15, **kw):
    b = len(As)
    ns = (ctypes.c_int * b)(*[int(a.shape[0]) for a in As])
    pa = (ctypes.c_void_p * b)(*[_mat(a, "c128").value for a in As])
    pq = (ctypes.c_void_p * b)(*[_mat(q, "c128").value for q in Qs])
    pt = (ctypes.c_void_p * b)(*[_mat(t, "c128").value for t in Ts])
    o = make_opts(**kw)
    infos = (SrInfo * max(1, b))()
    rc = lib().schur_refine_batched(b, ns, pa, pq, pt, int(iters), float(tol), ctypes.byref(o), infos)
    return rc, [infos[i].as_dict() for i in range(b)]


def workspace_dd(n: int, device="cuda", **kw):
    """A device workspace tensor for schur_refine_dd at size n under `kw`."""
    import torch

    o = make_opts(**kw)
    return torch.empty(max(1, int(lib().sr_workspace_bytes_dd(int(n), ctypes.byref(o)))),
                       dtype=torch.uint8, device=device)


def schur_refine_dd(A_hi, A_lo, Q_hi, Q_lo, T_hi, T_lo, iters: int = 8, tol: float = 1e-28, **kw):
    """Double-double refinement of (Q_hi + Q_lo, T_hi + T_lo) for A_hi + A_lo, in place."""
    n = A_hi.shape[0]
    args = [_mat(x, "c128", n, n) for x in (A_hi, A_lo, Q_hi, Q_lo, T_hi, T_lo)]
    o = make_opts(**kw)
    info = SrInfo()
    rc = lib().schur_refine_dd(*args, n, int(iters), float(tol), ctypes.byref(o), ctypes.byref(info))
    d = info.as_dict()
    d["rc"] = rc
    return d


def sr_zgemm(A, B, C, opa: int = 0, Cin=None, compensated: bool = False, stream=None) -> int:
    m, n = C.shape
    k = B.shape[0]
    return lib().sr_zgemm(int(opa), m, n, k, _mat(A, "c128"), _ld(A), _mat(B, "c128"),
                          _ld(B), _mat(Cin, "c128") if Cin is not None else None,
                          _ld(Cin), _mat(C, "c128"), _ld(C),
                          int(bool(compensated)), _stream(stream))


def sr_ozaki_zgemm(A, B, C, opa: int = 0, slices_a: int = 7, slices_b: int = 7, dmax=None, Cin=None,
                   ws=None, stream=None) -> int:
    """Ozaki split product on INT8 MFMA (see include/schur_refine.h)."""
    import torch

    m, n = C.shape
    k = B.shape[0]
    need = int(lib().sr_ozaki_ws_bytes(m, n, k, int(slices_a), int(slices_b)))
    if ws is None:
        ws = torch.empty(max(1, need), dtype=torch.uint8, device=C.device)
    d = int(dmax) if dmax is not None else int(slices_a) + int(slices_b)
    return lib().sr_ozaki_zgemm(int(opa), m, n, k, _mat(A, "c128"), _ld(A), _mat(B, "c128"),
                                _ld(B), _mat(Cin, "c128") if Cin is not None else None,
                                _ld(Cin), _mat(C, "c128"), _ld(C),
                                int(slices_a), int(slices_b), d, ctypes.c_void_p(ws.data_ptr()),
                                ws.numel() * ws.element_size(), _stream(stream))


def sr_crt_zgemm(A, B, C, opa: int = 0, bits: int = 55, Cin=None, ws=None, stream=None) -> int:
    """Ozaki scheme II (CRT) product on INT8 MFMA (see include/schur_refine.h)."""
    import torch

    m, n = C.shape
    k = B.shape[0]
    need = int(lib().sr_crt_ws_bytes(m, n, k, int(bits)))
    if ws is None:
        ws = torch.empty(max(1, need), dtype=torch.uint8, device=C.device)
    return lib().sr_crt_zgemm(int(opa), m, n, k, _mat(A, "c128"), _ld(A), _mat(B, "c128"), _ld(B),
                              _mat(Cin, "c128") if Cin is not None else None, _ld(Cin), _mat(C, "c128"),
                              _ld(C), int(bits), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel() * ws.element_size(), _stream(stream))


def sr_ozaki_zgemm_dd(A_hi, A_lo, B_hi, B_lo, C_hi, C_lo, opa: int = 0, slices_a: int = 14,
                      slices_b: int = 14, dmax=None, Cin_hi=None, Cin_lo=None, ws=None,
                      stream=None) -> int:
    """Double-double Ozaki split product (see include/schur_refine.h)."""
    import torch

    m, n = C_hi.shape
    k = B_hi.shape[0]
    need = int(lib().sr_ozaki_ws_bytes(m, n, k, int(slices_a), int(slices_b)))
    if ws is None:
        ws = torch.empty(max(1, need), dtype=torch.uint8, device=C_hi.device)
    d = int(dmax) if dmax is not None else int(slices_a) + 1
    opt = lambda x: _mat(x, "c128") if x is not None else None
    return lib().sr_ozaki_zgemm_dd(
        int(opa), m, n, k, _mat(A_hi, "c128"), opt(A_lo), _ld(A_hi), _mat(B_hi, "c128"),
        opt(B_lo), _ld(B_hi), opt(Cin_hi), opt(Cin_lo),
        _ld(Cin_hi), _mat(C_hi, "c128"), _mat(C_lo, "c128"),
        _ld(C_hi), int(slices_a), int(slices_b), d, ctypes.c_void_p(ws.data_ptr()),
        ws.numel() * ws.element_size(), _stream(stream))


def sr_ozaki_cgemm(A, B, C, slices: int = 3, herm: int = 0, ws=None, stream=None) -> int:
    """Complex64 product C = A B from INT8 digits, optionally Hermitian (1) or
    skew-Hermitian (-1) (see include/schur_refine.h)."""
    import torch

    m, n = C.shape
    k = B.shape[0]
    need = int(lib().sr_ozaki_ws_bytes(m, n, k, int(slices), int(slices)))
    if ws is None:
        ws = torch.empty(max(1, need), dtype=torch.uint8, device=C.device)
    return lib().sr_ozaki_cgemm(m, n, k, _mat(A, "c64"), _ld(A), _mat(B, "c64"), _ld(B), _mat(C, "c64"), _ld(C),
                                int(slices), int(herm), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel() * ws.element_size(), _stream(stream))


def sr_ozaki_zgemm_td(As, Bs, Cs, opa: int = 0, slices: int = 22, Cins=None, ws=None,
                      stream=None) -> int:
    """Triple-double Ozaki split product (see include/schur_refine.h): As, Bs, Cs
    (and Cins) are three complex128 column-major tensors each, largest term first."""
    import torch

    m, n = Cs[0].shape
    k = Bs[0].shape[0]
    need = int(lib().sr_ozaki_ws_bytes(m, n, k, int(slices), int(slices)))
    if ws is None:
        ws = torch.empty(max(1, need), dtype=torch.uint8, device=Cs[0].device)
    for xs in (As, Bs, Cs) + ((Cins,) if Cins is not None else ()):
        if len(xs) != 3 or len({_ld(x) for x in xs}) != 1 or len({tuple(x.shape) for x in xs}) != 1:
            raise ValueError("expected three terms of one shape and leading dimension")
    arr = lambda xs: (ctypes.c_void_p * 3)(*[_mat(x, "c128").value for x in xs])
    return lib().sr_ozaki_zgemm_td(
        int(opa), m, n, k, arr(As), _ld(As[0]), arr(Bs), _ld(Bs[0]),
        arr(Cins) if Cins is not None else None, _ld(Cins[0]) if Cins is not None else 1,
        arr(Cs), _ld(Cs[0]), int(slices), ctypes.c_void_p(ws.data_ptr()),
        ws.numel() * ws.element_size(), _stream(stream))


def sr_cgemm(A, B, C, stream=None) -> int:
    m, n = C.shape
    k = B.shape[0]
    return lib().sr_cgemm(m, n, k, _mat(A, "c64"), _ld(A), _mat(B, "c64"), _ld(B),
                          _mat(C, "c64"), _ld(C), _stream(stream))


def sr_residual(A, Q, T, T_lp, E_lp, ws, want_eps=True, compensated=True, stream=None):
    n = A.shape[0]
    eps = ctypes.c_double(0.0)
    rc = lib().sr_residual(_mat(A, "c128", n, n), _mat(Q, "c128", n, n), n, _mat(T, "c128", n, n),
                           _mat(T_lp, "c64", n, n), _mat(E_lp, "c64", n, n),
                           ctypes.byref(eps) if want_eps else None, int(bool(compensated)),
                           ctypes.c_void_p(ws.data_ptr()), _stream(stream))
    return rc, eps.value


def sr_trisolve(T_lp, E_lp, L_lp, ws, trunc: float = 0.0, stream=None) -> int:
    n = T_lp.shape[0]
    return lib().sr_trisolve(_mat(T_lp, "c64", n, n), _mat(E_lp, "c64", n, n),
                             _mat(L_lp, "c64", n, n), n, float(trunc),
                             ctypes.c_void_p(ws.data_ptr()), _stream(stream))


def sr_trisolve_static(T_lp, E_lp, L_lp, status, trunc: float = 0.0, stream=None) -> int:
    """The no-allocation solve: status is a device int32 tensor of one element
    (cleared, then nonzero on breakdown)."""
    import torch

    n = T_lp.shape[0]
    if not (isinstance(status, torch.Tensor) and status.is_cuda and status.dtype == torch.int32
            and status.numel() >= 1):
        raise TypeError("status must be an int32 CUDA tensor")
    return lib().sr_trisolve_static(_mat(T_lp, "c64", n, n), _mat(E_lp, "c64", n, n),
                                    _mat(L_lp, "c64", n, n), n, float(trunc),
                                    ctypes.c_void_p(status.data_ptr()), _stream(stream))


def sr_trisolve64(T, E, L, ws, stream=None) -> int:
    n = T.shape[0]
    return lib().sr_trisolve64(_mat(T, "c128", n, n), _mat(E, "c128", n, n), _mat(L, "c128", n, n), n,
                               ctypes.c_void_p(ws.data_ptr()), _stream(stream))


def reorder_start(A, Q, theta: float, perm=None, ws=None, stream=None) -> int:
    """Reorder the start Q in place (see sr_reorder_start); perm: optional int32 device
    tensor of length n for the original position of each new diagonal entry."""
    import torch

    n = A.shape[0]
    nb = lib().sr_reorder_ws_bytes(n)
    if ws is None:
        ws = torch.empty(nb, dtype=torch.uint8, device=A.device)
    if perm is not None and (perm.dtype != torch.int32 or perm.numel() != n or not perm.is_cuda):
        raise ValueError("perm must be an int32 CUDA tensor of length n")
    return lib().sr_reorder_start(_mat(A, "c128", n, n), _mat(Q, "c128", n, n), n, float(theta),
                                  ctypes.c_void_p(perm.data_ptr()) if perm is not None else None,
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                  _stream(stream))


def sr_update(Q, L_lp, Q_out, ws, gate=True, compensated=True, stream=None):
    n = Q.shape[0]
    norms = (ctypes.c_double * 2)()
    rc = lib().sr_update(_mat(Q, "c128", n, n), _mat(L_lp, "c64", n, n), _mat(Q_out, "c128", n, n), n,
                         int(bool(gate)), int(bool(compensated)), norms,
                         ctypes.c_void_p(ws.data_ptr()), _stream(stream))
    return rc, (norms[0], norms[1])


def sr_ns_init(Qh, Q, ws, compensated=True, stream=None) -> int:
    n = Qh.shape[0]
    return lib().sr_ns_init(_mat(Qh, "c128", n, n), _mat(Q, "c128", n, n), n,
                            int(bool(compensated)), ctypes.c_void_p(ws.data_ptr()), _stream(stream))


def sr_diag_mfma(A: np.ndarray, B: np.ndarray, kind: int = 0) -> np.ndarray:
    """kind 0: FP64 16x16x4 instruction, kind 1: FP32 16x16x4 instruction."""
    a = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(B, dtype=np.float64)
    d = np.zeros((16, 16), dtype=np.float64)
    rc = lib().sr_diag_mfma(int(kind), a.ctypes.data_as(ctypes.c_void_p),
                            b.ctypes.data_as(ctypes.c_void_p), d.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise RuntimeError(f"sr_diag_mfma failed: {rc}")
    return d


# ------------------------------------------------------------ real Schur variant

def _blocks(blocks, n):
    if blocks is None:
        return None
    b = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32))
    if b.size != n:
        raise ValueError("blocks must hold n markers")
    return b


def workspace_real(n: int, device="cuda"):
    import torch

    return torch.empty(max(1, int(lib().sr_workspace_bytes_real(int(n), None))), dtype=torch.uint8, device=device)


def schur_refine_real(A, Q, T, blocks, iters: int = 6, tol: float = 1e-15, **kw) -> dict:
    """Refine the real Schur form (Q, T) of the real A in place (float64 column-major
    tensors); blocks: the 2 x 2 block markers of the start (length n)."""
    n = A.shape[0]
    b = _blocks(blocks, n)
    o = make_opts(**kw)
    info = SrInfo()
    rc = lib().schur_refine_real(_mat(A, "f64", n, n), _mat(Q, "f64", n, n), _mat(T, "f64", n, n),
                                 b.ctypes.data_as(ctypes.c_void_p) if b is not None else None, n, int(iters),
                                 float(tol), ctypes.byref(o), ctypes.byref(info))
    d = info.as_dict()
    d["rc"] = rc
    return d


def sr_dgemm(A, B, C, opa: int = 0, Cin=None, compensated: bool = False, stream=None) -> int:
    m, n = C.shape
    k = B.shape[0]
    return lib().sr_dgemm(int(opa), m, n, k, _mat(A, "f64"), _ld(A), _mat(B, "f64"), _ld(B),
                          _mat(Cin, "f64") if Cin is not None else None, _ld(Cin), _mat(C, "f64"), _ld(C),
                          int(bool(compensated)), _stream(stream))


def sr_trisolve_real(T_lp, E_lp, L_lp, blocks, ws=None, stream=None) -> int:
    import torch

    n = T_lp.shape[0]
    b = _blocks(blocks, n)
    need = int(lib().sr_trisolve_real_ws_bytes(n))
    if ws is None:
        ws = torch.empty(max(1, need), dtype=torch.uint8, device=T_lp.device)
    return lib().sr_trisolve_real(_mat(T_lp, "f32", n, n), _mat(E_lp, "f32", n, n), _mat(L_lp, "f32", n, n),
                                  b.ctypes.data_as(ctypes.c_void_p) if b is not None else None, n,
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), _stream(stream))


def sr_trisolve_rec(T_lp, E_lp, L_lp, leaf_rows: int = 0, trunc: float = 0.0, ws=None, stream=None) -> int:
    """FP32 solve of stril(T L - L T) = -E by the recursive block algorithm."""
    import torch

    n = T_lp.shape[0]
    need = int(lib().sr_trisolve_rec_ws_bytes(n, int(leaf_rows)))
    if ws is None:
        ws = torch.empty(max(1, need), dtype=torch.uint8, device=T_lp.device)
    return lib().sr_trisolve_rec(_mat(T_lp, "c64", n, n), _mat(E_lp, "c64", n, n), _mat(L_lp, "c64", n, n), n,
                                 int(leaf_rows), float(trunc), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel() * ws.element_size(), _stream(stream))


# ------------------------------------------------------------ triple-double tier

def schur_refine_td(As, Qs, Ts, iters: int = 6, tol: float = 1e-40, **kw) -> dict:
    """Triple-double refinement: As, Qs, Ts are three complex128 column-major tensors
    each (the terms of the expansions, largest first); Qs and Ts are written."""
    n = As[0].shape[0]
    pa = (ctypes.c_void_p * 3)(*[_mat(a, "c128", n, n).value for a in As])
    pq = (ctypes.c_void_p * 3)(*[_mat(q, "c128", n, n).value for q in Qs])
    pt = (ctypes.c_void_p * 3)(*[_mat(t, "c128", n, n).value for t in Ts])
    o = make_opts(**kw)
    info = SrInfo()
    rc = lib().schur_refine_td(pa, pq, pt, n, int(iters), float(tol), ctypes.byref(o), ctypes.byref(info))
    d = info.as_dict()
    d["rc"] = rc
    return d
